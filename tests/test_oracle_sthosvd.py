"""Pins for Alg. 1 (truncated Gram SVD) and Alg. 2 (ST-HOSVD).

Checked against numpy.linalg.svd, the exact error split of Sec. 2.3, the
Eckart-Young truncation for d = 2, exact recovery of exactly low-rank tensors
and the closed-form sine-wave ranks 2 f_k + 1 of Sec. 5.1.
"""

import json
import os

import numpy as np
import pytest

from oracle import multi_ttm, reconstruct, sthosvd, tsvd_gram, ttm, unfold
from synth import SineWaveTensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lowrank(shape, ranks, seed):
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    mats = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in zip(shape, ranks)]
    return multi_ttm(core, mats)


@pytest.mark.parametrize("m,n,eps", [(6, 40, 0.5), (10, 30, 2.0), (8, 8, 1e-9)])
def test_tsvd_gram_matches_svd(m, n, eps):
    a = np.random.default_rng(m * n).standard_normal((m, n))
    a[:, :3] *= 10.0
    r, u, s, tail, lam = tsvd_gram(a, eps)
    sv = np.linalg.svd(a, compute_uv=False)
    np.testing.assert_allclose(np.sqrt(lam), sv, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(s, sv[:r], rtol=1e-10)
    # discarded energy is exactly the tail, and it is within the tolerance
    resid = a - u @ (u.T @ a)
    assert abs(np.sum(resid ** 2) - tail) <= 1e-9 * np.sum(a ** 2)
    assert tail <= eps ** 2
    # minimality: one fewer vector would exceed the tolerance
    if r > 0:
        assert np.sum(sv[r - 1:] ** 2) > eps ** 2
    # optional outputs of Alg. 1: V = A^T U S^-1 is orthonormal, A ~ U S V^T
    if r > 0:
        v = a.T @ u / s
        np.testing.assert_allclose(v.T @ v, np.eye(r), atol=1e-8)
        assert np.linalg.norm(a - u @ np.diag(s) @ v.T) <= eps * (1 + 1e-9)


def test_tsvd_rank_rule_equality_truncates():
    a = np.zeros((3, 5))
    a[0, 0], a[1, 1], a[2, 2] = 3.0, 2.0, 1.0
    assert tsvd_gram(a, 1.0)[0] == 2  # tail 1 <= 1: the third vector is dropped
    assert tsvd_gram(a, 0.999)[0] == 3
    assert tsvd_gram(a, np.sqrt(14.0))[0] == 0


@pytest.mark.parametrize("shape,tau", [((6, 7, 8), 0.3), ((5, 4, 6, 3), 0.2),
                                       ((9, 11), 0.1)])
def test_sthosvd_error_split_is_exact(shape, tau):
    rng = np.random.default_rng(sum(shape))
    ranks = tuple(max(1, n // 2) for n in shape)
    x = _lowrank(shape, ranks, sum(shape)) + 0.05 * rng.standard_normal(shape)
    res = sthosvd(x, tau)
    assert any(r < n for r, n in zip(res["core"].shape, shape))  # truncation happened
    xhat = reconstruct(res["core"], res["factors"])
    err2 = np.sum((x - xhat) ** 2)
    # squared error is the exact sum of the per-mode discarded tails
    assert sum(res["tails"]) > 0
    np.testing.assert_allclose(err2, sum(res["tails"]), rtol=1e-9)
    # and each tail is the partial-core error of its mode
    c = x
    for k, u in enumerate(res["factors"]):
        c_next = ttm(c, u.T, k)
        np.testing.assert_allclose(np.sum((c - ttm(c_next, u, k)) ** 2), res["tails"][k],
                                   rtol=1e-8, atol=1e-12)
        c = c_next
    assert np.sqrt(err2) <= tau * np.linalg.norm(x) * (1 + 1e-12)


def test_sthosvd_d2_is_truncated_svd():
    rng = np.random.default_rng(3)
    uu = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    vv = np.linalg.qr(rng.standard_normal((15, 12)))[0]
    sv = np.array([10, 8, 6, 4, 2, 1, 0.5, 0.3, 0.2, 0.1, 0.05, 0.02])
    x = uu @ np.diag(sv) @ vv.T
    tau = 0.1
    res = sthosvd(x, tau)
    xhat = reconstruct(res["core"], res["factors"])
    r = min(res["core"].shape)
    # Eckart-Young: the rank-r truncated SVD
    best = uu[:, :r] @ np.diag(sv[:r]) @ vv[:, :r].T
    np.testing.assert_allclose(xhat, best, atol=1e-11)
    eps = tau * np.linalg.norm(x) / np.sqrt(2)
    assert res["core"].shape[0] == int(np.argmax(np.r_[np.cumsum((sv ** 2)[::-1])[::-1], 0] <= eps ** 2))


def test_sthosvd_exact_low_rank_recovery():
    x = _lowrank((10, 9, 12, 7), (3, 4, 2, 5), seed=11)
    res = sthosvd(x, 1e-6)
    assert res["core"].shape == (3, 4, 2, 5)
    xhat = reconstruct(res["core"], res["factors"])
    assert np.linalg.norm(x - xhat) <= 1e-12 * np.linalg.norm(x)


def test_sthosvd_fixed_ranks():
    x = np.random.default_rng(5).standard_normal((6, 7, 8))
    res = sthosvd(x, 0.0, ranks=(2, 3, 4))
    assert res["core"].shape == (2, 3, 4)
    for u in res["factors"]:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=1e-13)


def test_sine_wave_closed_form_ranks():
    """Sec. 5.1: the sampled sine-wave tensor has mode-k rank 2 f_k + 1."""
    with open(os.path.join(GOLDEN, "sine_wave_ranks.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        sw = SineWaveTensor(dims=tuple(case["dims"]), freqs=tuple(case["freqs"]),
                            seed=case["seed"])
        for k, r in enumerate(case["expected_ranks"]):
            sv = np.linalg.svd(unfold(sw.full, k), compute_uv=False)
            assert np.sum(sv > 1e-9 * sv[0]) == r
        # tau above sqrt(machine eps): the Gram route resolves ranks (Sec. 2.3)
        res = sthosvd(sw.full, 1e-6)
        assert list(res["core"].shape) == case["expected_ranks"]
