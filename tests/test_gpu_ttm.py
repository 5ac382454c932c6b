"""GPU: the mode-k TTM kernel (st_ttm) against numpy, FP32 and bf16x3.

Covers contiguous (mode 1) and strided fibres, ragged sizes that are not
multiples of the 16 x 32 MFMA tiles, one and several output-row tiles, and the
fused residual norm ||X - (X x_k U^T) x_k U||^2 with ||X||^2.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(dims, mode, rows, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(dims).astype(np.float32)
    u, _ = np.linalg.qr(rng.standard_normal((dims[mode], rows)))
    return x, u.astype(np.float32)


def _ref(x, a, mode):
    x64 = x.astype(np.float64)
    a64 = a.astype(np.float64)
    y = np.moveaxis(np.tensordot(a64, x64, axes=([1], [mode])), 0, mode)
    back = np.moveaxis(np.tensordot(a64.T, y, axes=([1], [mode])), 0, mode)
    return y, np.sum((x64 - back) ** 2), np.sum(x64 ** 2)


CASES = [
    ((128, 64, 3), 0, 33),
    ((32, 40, 7), 1, 5),
    ((20, 37, 9, 3), 2, 9),
    ((16, 16, 16, 16), 3, 16),
    ((33, 17, 5), 0, 1),
    ((64, 48, 5), 1, 48),
    ((200, 30), 0, 130),
    ((12, 300), 1, 260),
    ((320, 6, 2), 0, 300),   # fused residual with more than 256 rows (20 tiles)
    ((24, 380), 1, 370),     # 24 tiles
    # contiguous FP32 fibres with n <= 128, n % 4 == 0 (the persistent tile kernel)
    ((128, 128, 16), 0, 39),  # the mode-1 shape of the 128^3 x 16 stream, 32 tiles
    ((96, 37, 3), 0, 17),     # ragged last tile (111 fibres)
    ((36, 50), 0, 64),        # n padded to 64 inside the kernel, rows clipped to 36
    ((64, 129), 0, 7),        # one fibre in the last tile
    ((4, 70), 0, 3),          # shortest fibre
    ((128, 40000), 0, 64),    # more tiles than blocks (persistent loop), 4 row tiles
]


@pytest.mark.parametrize("precision,rtol", [("fp32", 2e-5), ("bf16x3", 2e-4), ("fp64", 1e-12)])
@pytest.mark.parametrize("dims,mode,rows", CASES)
def test_ttm_projection_and_residual(dims, mode, rows, precision, rtol):
    import torch

    from paper_2308_16395_amd.binding import ttm

    rows = min(rows, dims[mode])
    x, u = _case(dims, mode, rows, sum(dims) + rows)
    # column-major device layout: the C-ordered array of the reversed axes
    xd = torch.from_numpy(np.ascontiguousarray(x.ravel(order="F"))).cuda()
    a = torch.from_numpy(np.ascontiguousarray(u.T)).cuda()  # rows x n, row-major
    want_norms = rows <= 384
    res = ttm(xd, dims, mode, a, precision=precision, norms=want_norms)
    out, norms = (res if want_norms else (res, None))
    y_ref, e2_ref, x2_ref = _ref(x, u.T, mode)
    out_dims = list(dims)
    out_dims[mode] = rows
    y = out.cpu().numpy().reshape(out_dims, order="F").astype(np.float64)
    scale = np.abs(y_ref).max()
    if precision == "fp64":
        # exact products and FP64 sums: only the final rounding to FP32 remains
        np.testing.assert_allclose(y, y_ref, rtol=2 ** -23, atol=1e-12 * scale)
    else:
        np.testing.assert_allclose(y, y_ref, rtol=0, atol=rtol * scale * np.sqrt(dims[mode]))
    if want_norms:
        e2, x2 = norms
        np.testing.assert_allclose(x2, x2_ref, rtol=1e-12)
        # the residual norm squared is accurate to the product precision relative to ||X||^2
        tol = {"fp32": 1e-5, "bf16x3": 1e-3, "fp64": 1e-12}[precision]
        assert abs(e2 - e2_ref) <= tol * x2_ref


GRAM_CASES = [
    ((32, 320), 0, 0),
    ((128, 40, 3), 0, 33),
    ((20, 37, 9, 3), 2, 0),
    ((24, 17, 5), 1, 6),
    ((9, 20), 1, 0),
    ((260, 7), 0, 40),
    ((400, 6), 0, 0),        # FP64: E too long for LDS, formed over row-chunk pairs
    ((400, 6), 0, 24),
    ((7, 512, 2), 1, 37),
]


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-13), ("fp32", 1e-5), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("dims,mode,rows", GRAM_CASES)
def test_gram_against_numpy(dims, mode, rows, precision, rtol):
    import torch

    from paper_2308_16395_amd.binding import gram

    x, u = _case(dims, mode, max(rows, 1), sum(dims) + 7 * rows)
    xd = torch.from_numpy(np.ascontiguousarray(x.ravel(order="F"))).cuda()
    a = torch.from_numpy(np.ascontiguousarray(u.T)).cuda() if rows > 0 else None
    g = gram(xd, dims, mode, a, precision=precision)
    x64 = np.moveaxis(x.astype(np.float64), mode, 0).reshape(dims[mode], -1)
    if rows > 0:
        u64 = u.astype(np.float64)
        x64 = x64 - u64 @ (u64.T @ x64)
    ref = x64 @ x64.T
    xx = np.sum(x.astype(np.float64) ** 2) / dims[mode]
    if rows == 0:
        tol = rtol * np.abs(ref).max()
    elif precision == "fp64":
        # residual formed with FP64 products and kept in FP64
        tol = 1e-13 * xx
    else:
        # the residual is formed in FP32, so its Gram is accurate to ~1e-6 of ||X||^2
        tol = max(rtol * np.abs(ref).max(), 1e-5 * xx)
    np.testing.assert_allclose(g, ref, rtol=0, atol=tol)


def test_gram_rejects_fibres_longer_than_512():
    import torch

    from paper_2308_16395_amd.binding import StError, gram

    dims = (520, 3)
    xd = torch.zeros(520 * 3, device="cuda")
    with pytest.raises(StError):
        gram(xd, dims, 0, None, precision="fp64")


@pytest.mark.parametrize("precision,rtol", [("fp32", 2e-5), ("bf16x3", 2e-4)])
@pytest.mark.parametrize("dims,rows", [((128, 300), 39), ((36, 50), 20)])
def test_contiguous_projection_without_norms(dims, rows, precision, rtol):
    """The projection alone (no residual) on contiguous fibres."""
    import torch

    from paper_2308_16395_amd.binding import ttm

    x, u = _case(dims, 0, rows, 5 + rows)
    xd = torch.from_numpy(np.ascontiguousarray(x.ravel(order="F"))).cuda()
    a = torch.from_numpy(np.ascontiguousarray(u.T)).cuda()
    out = ttm(xd, dims, 0, a, precision=precision, norms=False)
    y_ref, _, _ = _ref(x, u.T, 0)
    got = out.cpu().numpy().astype(np.float64).reshape([rows] + list(dims[1:]), order="F")
    assert np.linalg.norm(got - y_ref) <= rtol * np.linalg.norm(y_ref)
