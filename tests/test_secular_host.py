"""CPU unit test of the library's secular-equation SVD of the ISVD matrix S'.

The device code in secular.hpp is compiled for the host with plain loops and
compared with numpy.linalg.svd of S' = [[diag(s), 0], [p^T, q]] (new
direction kept) or [diag(s); p^T] (ignored): singular values to high relative
accuracy, orthonormal singular vectors, and U'' S~ V''^T = S'.
"""

import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2308_16395_amd", "csrc")
OUT = os.path.join(HERE, "_build", "libsecular_host.so")


@pytest.fixture(scope="module")
def sec():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    src = os.path.join(HERE, "host", "secular_host.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, src, "-o", OUT],
                   check=True)
    lib = C.CDLL(OUT)
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    lib.sec_svd_host.argtypes = [C.c_int, dp, dp, C.c_double, C.c_int, C.c_double, dp, dp, dp, ip]
    lib.sec_svd_host.restype = C.c_int
    return lib


def _run(lib, s, p, q, grow):
    r = len(s)
    n = r + 1
    tol = 8 * 2.0 ** -53 * max(s[0], np.abs(p).max(initial=0.0), q)
    u2 = np.zeros((n, n), order="F")
    v2 = np.zeros((n, n), order="F")
    sn = np.zeros(n)
    counts = np.zeros(3, dtype=np.int32)
    ntrip = lib.sec_svd_host(r, np.ascontiguousarray(s), np.ascontiguousarray(p), q, int(grow),
                             tol, u2.ravel(order="F"), v2.ravel(order="F"), sn, counts)
    # the ravel of an F-ordered array is a view only when contiguous; copy back explicitly
    return ntrip, counts


def _svd(lib, s, p, q, grow):
    r = len(s)
    n = r + 1
    tol = 8 * 2.0 ** -53 * max(s[0], np.abs(p).max(initial=0.0), q)
    u2 = np.zeros(n * n)
    v2 = np.zeros(n * n)
    sn = np.zeros(n)
    counts = np.zeros(3, dtype=np.int32)
    c = lib.sec_svd_host(r, np.ascontiguousarray(s, dtype=np.float64),
                         np.ascontiguousarray(p, dtype=np.float64), float(q), int(grow), tol,
                         u2, v2, sn, counts)
    u2 = u2.reshape((n, n), order="F")[:, :c]
    v2 = v2.reshape((n, n), order="F")[:, :c]
    return u2, sn[:c], v2, counts


def _sprime(s, p, q, grow):
    r = len(s)
    if grow:
        m = np.zeros((r + 1, r + 1))
        m[:r, :r] = np.diag(s)
        m[r, :r] = p
        m[r, r] = q
    else:
        m = np.vstack([np.diag(s), p[None, :]])
    return m


def _check(lib, s, p, q, grow, rtol_s=1e-12):
    m = _sprime(s, p, q, grow)
    u2, sn, v2, counts = _svd(lib, s, p, q, grow)
    c = m.shape[1]
    assert sn.shape[0] == c
    ref = np.linalg.svd(m, compute_uv=False)
    np.testing.assert_allclose(sn, ref, rtol=rtol_s, atol=1e-15 * ref[0])
    assert np.all(np.diff(sn) <= 0)
    v2 = v2[:c, :] if grow else v2[:c, :]
    np.testing.assert_allclose(u2.T @ u2, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(v2.T @ v2, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(u2 @ np.diag(sn) @ v2.T, m, atol=2e-14 * ref[0])
    return counts


@pytest.mark.parametrize("r", [1, 2, 5, 40, 300])
@pytest.mark.parametrize("grow", [True, False])
def test_random(sec, r, grow):
    rng = np.random.default_rng(r + 100 * grow)
    s = np.sort(rng.uniform(0.1, 10.0, r))[::-1].copy()
    p = rng.standard_normal(r)
    q = 0.7 if grow else 0.0
    _check(sec, s, p, q, grow)


@pytest.mark.parametrize("grow", [True, False])
def test_streaming_like_spectrum(sec, grow):
    """Singular values over many decades, small p, q near the tolerance."""
    rng = np.random.default_rng(7)
    r = 120
    s = np.sort(10.0 ** rng.uniform(-4, 2, r))[::-1].copy()
    p = 1e-2 * rng.standard_normal(r)
    q = 4.5e-5 if grow else 0.0
    _check(sec, s, p, q, grow, rtol_s=1e-10)


def test_deflation_small_weights_and_equal_poles(sec):
    rng = np.random.default_rng(9)
    r = 30
    s = np.sort(rng.uniform(1.0, 5.0, r))[::-1].copy()
    s[10] = s[11]            # exactly equal poles
    s[20] = s[21] * (1 + 1e-17)
    p = rng.standard_normal(r)
    p[3] = 0.0               # zero weight
    p[5] = 1e-30             # below the tolerance
    counts = _check(sec, s, p, 0.3, True)
    assert counts[2] >= 1    # a close-pole rotation happened
    assert counts[1] >= 2    # deflated entries


def test_zero_row_is_identity(sec):
    s = np.array([3.0, 2.0, 1.0])
    u2, sn, v2, counts = _svd(sec, s, np.zeros(3), 0.0, False)
    np.testing.assert_allclose(sn, s, rtol=1e-15)
    np.testing.assert_allclose(np.abs(v2[:3, :]), np.eye(3), atol=1e-15)


def _block_rows_svd(lib, S, P, X):
    """The block middle-matrix SVD as the library forms it: b row appends to
    [diag(S), 0] (c = rd + l columns, l zero poles), each a secular solve of a
    diagonal matrix plus one row without a new column, with the same flat
    buffer layouts as the kernels (V_K: ld c + 1, U_K: ld c + b; the padding
    rows rd..c-1 of U_K dropped at the end)."""
    rd, b = P.shape
    ell = X.shape[1]
    c = rd + ell
    ldv, ldu = c + 1, c + b
    vk = np.zeros(ldv * c)
    uk = np.zeros(ldu * c)
    for i in range(c):
        vk[i + ldv * i] = 1.0
        uk[i + ldu * i] = 1.0
    sig = np.concatenate([S, np.zeros(ell)])
    kmat = np.zeros((rd + b, c))
    kmat[:rd, :rd] = np.diag(S)
    kmat[rd:, :rd] = P.T
    kmat[rd:, rd:] = X
    for j in range(b):
        vkm = vk.reshape((ldv, c), order="F")[:c, :]
        z = vkm.T @ kmat[rd + j, :]
        tol = 8 * 2.0 ** -53 * max(S[0], np.sqrt((P ** 2).sum() + (X ** 2).sum()))
        u2 = np.zeros((c + 1) * c)
        v2 = np.zeros((c + 1) * c)
        sn = np.zeros(c + 1)
        counts = np.zeros(3, dtype=np.int32)
        nt = lib.sec_svd_host(c, np.ascontiguousarray(sig), np.ascontiguousarray(z), 0.0, 0, tol,
                              u2, v2, sn, counts)
        assert nt == c
        u2m = u2.reshape((c + 1, c), order="F")
        v2m = v2.reshape((c + 1, c), order="F")
        vk = np.zeros(ldv * c)
        vk.reshape((ldv, c), order="F")[:c, :] = vkm @ v2m[:c, :]
        m = c + j  # rows of U_K so far
        ukm = uk.reshape((ldu, c), order="F")
        new = np.zeros((ldu, c))
        new[:m, :] = ukm[:m, :] @ u2m[:c, :]
        new[m, :] = u2m[c, :]
        uk = new.ravel(order="F")
        sig = sn[:c].copy()
    ukm = uk.reshape((ldu, c), order="F")
    u = np.vstack([ukm[:rd, :], ukm[c:c + b, :]])
    pad = ukm[rd:c, :]
    return u, sig, vk.reshape((ldv, c), order="F")[:c, :], kmat, pad


@pytest.mark.parametrize("rd,b,ell", [(12, 4, 4), (40, 4, 2), (60, 16, 16), (110, 16, 3),
                                      (30, 3, 0), (5, 1, 1)])
def test_block_middle_matrix_by_row_appends(sec, rd, b, ell):
    """The block update's middle matrix [[diag S, 0], [P^T, X]] by b secular
    row appends equals its SVD (numpy), with the l zero poles deflating and the
    padding rows of U vanishing."""
    rng = np.random.default_rng(1000 + rd + b + ell)
    S = np.sort(10.0 ** rng.uniform(-3, 3, rd))[::-1].copy()
    P = 1e-2 * rng.standard_normal((rd, b))
    X = 1e-4 * rng.standard_normal((b, ell))
    u, sig, v, kmat, pad = _block_rows_svd(sec, S, P, X)
    c = rd + ell
    ref = np.linalg.svd(kmat, compute_uv=False)
    np.testing.assert_allclose(sig, ref, rtol=1e-10, atol=1e-15 * ref[0])
    assert np.all(np.diff(sig) <= 0)
    assert np.max(np.abs(pad), initial=0.0) <= 1e-13
    np.testing.assert_allclose(u.T @ u, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(v.T @ v, np.eye(c), atol=1e-13)
    np.testing.assert_allclose(u @ np.diag(sig) @ v.T, kmat, atol=4e-15 * ref[0] * np.sqrt(c))
