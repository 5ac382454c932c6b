"""GPU parity of the library's small symmetric eigensolver (st_symeig: the
eigendecomposition step of Alg. 1 after the Gram) against the oracle's
TruncatedSVD (tsvd_gram: numpy's eigh of A A^T) and against numpy on
indefinite matrices: every eigenvalue within a few u ||A||, the rank rule's
decision from the GPU eigenvalues equal to the oracle's, the kept subspace
(projector) within u ||A|| / gap, residuals and orthonormality of the vectors,
and the degenerate cases (order 1 and 2, zero, diagonal and tridiagonal
matrices, a multiple top eigenvalue, a graded spectrum, many kept vectors with
isolated and clustered eigenvalues, the upper triangle ignored, argument
errors).
"""

import numpy as np
import pytest

from oracle import tsvd_gram

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _symeig(a, k):
    import torch

    import paper_2308_16395_amd.binding as bd

    w, q = bd.symeig(torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda(), k)
    return w.cpu().numpy(), q.cpu().numpy()


def _check_vectors(a, w, q, tol):
    n, k = q.shape
    nrm = max(np.abs(np.linalg.eigvalsh(a)).max(), 1e-300)
    lam = w[::-1][:k]
    assert np.max(np.abs(a @ q - q * lam[None, :])) <= tol * nrm
    assert np.max(np.abs(q.T @ q - np.eye(k))) <= tol * max(1, n / 8)


@pytest.mark.parametrize("n,f,seed", [(16, 40, 1), (48, 300, 2), (100, 60, 3), (128, 500, 4),
                                      (128, 20, 5), (127, 900, 6)])
def test_gram_eigen_matches_oracle_tsvd(n, f, seed):
    rng = np.random.default_rng(seed)
    # graded columns: a decaying spectrum like a residual or data Gram
    a = rng.standard_normal((n, f)) * np.logspace(0, -4, f)[None, :]
    a = a @ rng.standard_normal((f, f)) / np.sqrt(f)
    lam_all = np.linalg.eigvalsh(a @ a.T)[::-1]
    # a tolerance halfway (in the log) between two tail sums, away from any tie
    tails = np.cumsum(np.maximum(lam_all, 0)[::-1])[::-1]
    # (inside the numerical rank, min(n, f): below it the eigenvalues are rounding)
    j = max(1, min(n - 2, n // 6, f // 2))
    eps = np.sqrt(np.sqrt(tails[j] * tails[j + 1]))
    r, p, s, tail, lam = tsvd_gram(a, eps)
    g = a @ a.T
    w, q = _symeig(g, r)
    np.testing.assert_allclose(w[::-1], lam, rtol=0, atol=16 * n * U * lam[0])
    # the rank rule of Alg. 1 on the GPU's eigenvalues
    lg = np.maximum(w[::-1], 0.0)
    tg = np.zeros(n + 1)
    tg[:n] = np.cumsum(lg[::-1])[::-1]
    assert int(np.argmax(tg <= eps * eps)) == r
    # kept subspace: projector distance within u ||G|| / gap
    gap = lam[r - 1] - (lam[r] if r < n else 0.0)
    dist = np.linalg.norm(q @ q.T - p @ p.T, 2)
    assert dist <= 64 * n * U * lam[0] / gap + 1e-13, (dist, gap)
    _check_vectors(g, w, q, 64 * U * n)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 33, 64, 65, 100, 128])
def test_random_symmetric(n):
    rng = np.random.default_rng(100 + n)
    b = rng.standard_normal((n, n))
    a = b + b.T
    w, q = _symeig(a, min(n, 7))
    ref = np.linalg.eigvalsh(a)
    nrm = np.abs(ref).max()
    np.testing.assert_allclose(w, ref, rtol=0, atol=8 * n * U * nrm)
    _check_vectors(a, w, q, 64 * U * n)


def test_degenerate_matrices():
    rng = np.random.default_rng(7)
    n = 128
    # zero matrix: eigenvalues 0, any orthonormal vectors
    w, q = _symeig(np.zeros((n, n)), 5)
    assert np.abs(w).max() <= 1e-300
    np.testing.assert_allclose(q.T @ q, np.eye(5), atol=1e-13)
    # identity times 3: one eigenvalue of multiplicity n
    w, q = _symeig(3.0 * np.eye(n), 4)
    np.testing.assert_allclose(w, 3.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(q.T @ q, np.eye(4), atol=1e-13)
    # diagonal (already reduced: every reflection is the identity)
    dg = rng.random(n)
    w, q = _symeig(np.diag(dg), 6)
    np.testing.assert_allclose(w, np.sort(dg), rtol=0, atol=4 * U)
    top = np.argsort(dg)[::-1][:6]
    np.testing.assert_allclose(np.abs(q[top, np.arange(6)]), 1.0, atol=1e-14)
    # tridiagonal
    t = np.diag(rng.random(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    w, q = _symeig(t, 5)
    np.testing.assert_allclose(w, np.linalg.eigvalsh(t), rtol=0, atol=1e-13)
    _check_vectors(t, w, q, 1e-13)
    # a triple top eigenvalue: the three vectors span its eigenspace
    qq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.r_[np.full(3, 2.0), np.linspace(0.0, 1.0, n - 3)]
    a = (qq * d) @ qq.T
    a = 0.5 * (a + a.T)
    w, q = _symeig(a, 3)
    np.testing.assert_allclose(w[-3:], 2.0, atol=1e-13)
    np.testing.assert_allclose(q @ q.T, qq[:, :3] @ qq[:, :3].T, atol=1e-12)
    _check_vectors(a, w, q, 1e-13)


def test_small_orders_and_upper_triangle_ignored():
    w, q = _symeig(np.array([[-2.5]]), 1)
    assert w[0] == pytest.approx(-2.5, rel=4 * U) and abs(q[0, 0]) == 1.0
    w, q = _symeig(np.array([[1.0, 2.0], [2.0, 1.0]]), 2)
    np.testing.assert_allclose(w, [-1.0, 3.0], atol=1e-15)
    np.testing.assert_allclose(np.abs(q), np.full((2, 2), np.sqrt(0.5)), atol=1e-15)
    rng = np.random.default_rng(9)
    b = rng.standard_normal((40, 40))
    a = b + b.T
    junk = a.copy()
    junk[np.triu_indices(40, 1)] = np.nan
    w1, q1 = _symeig(a, 4)
    w2, q2 = _symeig(junk, 4)
    np.testing.assert_array_equal(w1, w2)
    np.testing.assert_array_equal(q1, q2)


def test_graded_spectrum_like_an_initial_gram():
    """The data Gram at initialisation keeps r of n eigenpairs whose
    eigenvalues span many decades, with a large cluster near zero below."""
    rng = np.random.default_rng(11)
    n, r = 128, 30
    a = rng.standard_normal((n, r)) * np.logspace(0, -6, r)[None, :]
    g = a @ a.T
    w, q = _symeig(g, r)
    lam, p = np.linalg.eigh(g)
    lam, p = lam[::-1], p[:, ::-1]
    np.testing.assert_allclose(w[::-1], lam, rtol=0, atol=16 * n * U * lam[0])
    for c in range(r):
        gap = min(lam[c - 1] - lam[c] if c > 0 else np.inf, lam[c] - lam[c + 1])
        assert 1.0 - abs(q[:, c] @ p[:, c]) <= (64 * n * U * lam[0] / gap) ** 2 + 1e-14
    _check_vectors(g, w, q, 64 * U * n)


@pytest.mark.parametrize("n,k", [(128, 128), (100, 50), (64, 33)])
def test_many_vectors_isolated_and_clustered(n, k):
    """Many kept vectors at once: the isolated ones are found in parallel in
    batches (several batches here), the clustered ones one by one with
    orthogonalisation; all must be eigenvectors and orthonormal together."""
    rng = np.random.default_rng(300 + n)
    qq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = np.linspace(1.0, 2.0, n)
    m = n // 2
    d[m:m + 3] = d[m] + np.array([0.0, 1e-9, 2e-9])  # a tight cluster of three
    d[5:7] = d[5]  # and a double eigenvalue
    a = (qq * d) @ qq.T
    a = 0.5 * (a + a.T)
    w, q = _symeig(a, k)
    np.testing.assert_allclose(w, np.sort(d), rtol=0, atol=16 * n * U * 2.0)
    _check_vectors(a, w, q, 64 * U * n)


def test_argument_errors():
    import torch

    import paper_2308_16395_amd.binding as bd

    with pytest.raises(bd.StError) as ei:
        bd.symeig(torch.zeros((129, 129), dtype=torch.float64, device="cuda"), 1)
    assert ei.value.code == bd.ST_EINVAL
    with pytest.raises(bd.StError) as ei:
        bd.symeig(torch.zeros((8, 8), dtype=torch.float64, device="cuda"), 9)
    assert ei.value.code == bd.ST_EINVAL
