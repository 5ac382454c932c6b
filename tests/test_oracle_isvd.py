"""Pins for Alg. 3 (incremental SVD) and Prop. 1 (its error evolution).

Prop. 1 is an equality: appending a row whose complement e is ignored adds
exactly ||e||^2 to the squared error; keeping e adds nothing. With eps = 0 the
update must agree with numpy.linalg.svd of the stacked matrix.
"""

import numpy as np
import pytest

from oracle import isvd


def _approx_svd(m, n, r, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    a += noise * rng.standard_normal((m, n))
    uu, ss, vt = np.linalg.svd(a, full_matrices=False)
    return a, uu[:, :r], ss[:r], vt[:r].T


def _err2(a, u, s, v):
    return float(np.sum((a - u @ np.diag(s) @ v.T) ** 2))


@pytest.mark.parametrize("ignore", [True, False])
def test_prop1_error_evolution_is_exact(ignore):
    a, u, s, v = _approx_svd(30, 20, 4, seed=1, noise=1e-3)
    rng = np.random.default_rng(2)
    b = v @ rng.standard_normal(4) + 0.05 * rng.standard_normal(20)
    before = _err2(a, u, s, v)
    e = b - v @ (v.T @ b)
    q = np.linalg.norm(e)
    eps = 2 * q if ignore else 0.5 * q
    u2, s2, v2, info = isvd(u, s, v, b, eps)
    assert info["ignored"] == ignore
    assert s2.shape[0] == (4 if ignore else 5)
    after = _err2(np.vstack([a, b]), u2, s2, v2)
    expected = before + (q * q if ignore else 0.0)
    np.testing.assert_allclose(after, expected, rtol=1e-10)
    np.testing.assert_allclose(u2.T @ u2, np.eye(s2.shape[0]), atol=1e-13)
    np.testing.assert_allclose(v2.T @ v2, np.eye(s2.shape[0]), atol=1e-13)
    assert np.all(s2 > 0) and np.all(np.diff(s2) <= 0)


def test_isvd_exact_equals_svd_of_stacked_matrix():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((8, 12))
    uu, ss, vt = np.linalg.svd(a, full_matrices=False)
    u, s, v = uu, ss, vt.T
    rows = [a]
    for _ in range(4):
        b = rng.standard_normal(12)
        u, s, v, _ = isvd(u, s, v, b, 0.0)
        rows.append(b[None, :])
    stacked = np.vstack(rows)
    ref = np.linalg.svd(stacked, compute_uv=False)
    np.testing.assert_allclose(s, ref[:s.shape[0]], rtol=1e-12)
    np.testing.assert_allclose(u @ np.diag(s) @ v.T, stacked, atol=1e-12)


def test_isvd_qr_branch_keeps_the_factorization():
    """The QR fix of Alg. 3 only re-expresses S' V'^T; the result must match."""
    a, u, s, v = _approx_svd(25, 15, 3, seed=4, noise=1e-2)
    b = np.random.default_rng(5).standard_normal(15)
    _, s_plain, _, info_plain = isvd(u, s, v, b, 0.0, eps_m=1.0)
    u_qr, s_qr, v_qr, info_qr = isvd(u, s, v, b, 0.0, eps_m=0.0)
    assert not info_plain["qr"] and info_qr["qr"]
    np.testing.assert_allclose(s_qr, s_plain, rtol=1e-12)
    np.testing.assert_allclose(v_qr.T @ v_qr, np.eye(4), atol=1e-13)


def test_isvd_zero_row_is_ignored():
    a, u, s, v = _approx_svd(10, 6, 2, seed=6)
    u2, s2, v2, info = isvd(u, s, v, np.zeros(6), 0.0)
    assert info["ignored"] and info["q"] == 0.0
    np.testing.assert_allclose(s2, s, rtol=1e-14)
    np.testing.assert_allclose(np.abs(u2[-1]), 0.0, atol=1e-15)
