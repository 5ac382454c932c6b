"""GPU parity of Reconstruct / Project and their VJPs (st_tucker_fwd/bwd)
against the FP64 oracle (oracle/grad.py), through the C ABI.

Inputs: blob windows with factors from the oracle's fixed-rank ST-HOSVD and a
perturbed core (so the gradients are not zero), and random orthonormal factors
for ragged shapes. Both sides consume the same float32 values. Tolerances are
relative Frobenius errors: FP32 MFMA products 1e-5, split bf16 1e-4, FP64
products 1e-6 (the products are exact, but every intermediate of the chain and
the output are FP32 arrays, so each of the d steps rounds once: ~d 2^-24).
At the 96^3 x 8 x 16 window with ranks (24, 24, 24, 6, 8) every output of
the GPU is compared element by element with the oracle evaluated on the host
(the largest difference relative to the largest entry).
"""

import numpy as np
import pytest

from oracle import (multi_ttm, sthosvd, tucker_project, tucker_project_vjp, tucker_reconstruct,
                    tucker_reconstruct_loss_grad)
from synth import BlobStream

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-4, "fp64": 1e-6}


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _blob_instance(space, n_vars, window, ranks, seed):
    bs = BlobStream(space, n_vars, 4, (1.5, 3.0), 0.5, n_slices=window, seed=seed)
    x = np.stack([bs.slice(t) for t in range(window)], axis=-1)
    res = sthosvd(x, 0.0, ranks=ranks)
    rng = np.random.default_rng(seed)
    core = res["core"] + 1e-2 * np.linalg.norm(res["core"]) * rng.standard_normal(
        res["core"].shape) / np.sqrt(res["core"].size)
    return _f32(x), _f32(core), [_f32(u) for u in res["factors"]]


def _random_instance(dims, ranks, seed):
    rng = np.random.default_rng(seed)
    factors = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in zip(dims, ranks)]
    core = rng.standard_normal(ranks)
    x = multi_ttm(core, factors) + 0.1 * rng.standard_normal(dims)
    return _f32(x), _f32(core), [_f32(u) for u in factors]


CASES = [
    ("blob_window_12x12x12x4x4", lambda: _blob_instance((12, 12, 12), 4, 4, (3, 3, 3, 2, 2), 3)),
    ("ragged_37x20x9", lambda: _random_instance((37, 20, 9), (5, 7, 3), 11)),
    ("matrix_64x48", lambda: _random_instance((64, 48), (16, 9), 12)),
    ("vector_17", lambda: _random_instance((17,), (4,), 13)),
    ("full_rank_6x5x4", lambda: _random_instance((6, 5, 4), (6, 5, 4), 14)),
    ("wide_130x3x40", lambda: _random_instance((130, 3, 40), (33, 2, 17), 15)),
]


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32).ravel(order="F"))).cuda()


def _devu(u):
    from paper_2308_16395_amd.autodiff import colmajor

    import torch

    return colmajor(torch.from_numpy(np.asarray(u, np.float32)).cuda())


def _host(t, shape):
    return t.detach().cpu().numpy().astype(np.float64).reshape(shape, order="F")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_forward_and_vjps_match_oracle(name, make, precision):
    import paper_2308_16395_amd.autodiff as ad

    x, core, factors = make()
    dims, ranks = x.shape, core.shape
    tol = TOL[precision]
    U = [_devu(u) for u in factors]
    # Reconstruct
    xhat = _host(ad.tucker_reconstruct(_dev(core), U, precision), dims)
    ref = tucker_reconstruct(core, factors)
    assert _rel(xhat, ref) <= tol, ("reconstruct", _rel(xhat, ref))
    # Project
    g = _host(ad.tucker_project(_dev(x), U, precision), ranks)
    assert _rel(g, tucker_project(x, factors)) <= tol
    # Reconstruct VJP at the loss ||X^ - X||^2: upstream 2 (X^ - X) from the oracle
    loss, g_core_ref, g_u_ref = tucker_reconstruct_loss_grad(core, factors, x)
    upstream = 2.0 * (ref - x)
    g_core, g_u = ad.tucker_reconstruct_vjp(_dev(core), U, _dev(upstream), precision)
    assert _rel(_host(g_core, ranks), g_core_ref) <= tol
    for k, (gu, gr) in enumerate(zip(g_u, g_u_ref)):
        got = gu.detach().cpu().numpy().astype(np.float64)
        assert _rel(got, gr) <= tol, ("dU", k, _rel(got, gr))
    # Project VJP for an upstream core gradient
    rng = np.random.default_rng(99)
    gbar = _f32(rng.standard_normal(ranks))
    g_x, g_u = ad.tucker_project_vjp(_dev(x), U, _dev(gbar), precision)
    gx_ref, gu_ref = tucker_project_vjp(x, factors, gbar)
    assert _rel(_host(g_x, dims), gx_ref) <= tol
    for k, (gu, gr) in enumerate(zip(g_u, gu_ref)):
        got = gu.detach().cpu().numpy().astype(np.float64)
        assert _rel(got, gr) <= tol, ("dU proj", k, _rel(got, gr))


def test_autograd_loss_gradients_match_oracle():
    import torch

    from paper_2308_16395_amd.autodiff import colmajor, project, reconstruct

    x, core, factors = _blob_instance((12, 12, 12), 4, 4, (3, 3, 3, 2, 2), 5)
    xd = _dev(x)
    c = _dev(core).requires_grad_(True)
    U = [colmajor(torch.from_numpy(np.asarray(u, np.float32)).cuda()).requires_grad_(True)
         for u in factors]
    loss = ((reconstruct(c, U) - xd) ** 2).sum()
    loss.backward()
    loss_ref, g_core_ref, g_u_ref = tucker_reconstruct_loss_grad(core, factors, x)
    assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
    assert _rel(_host(c.grad, core.shape), g_core_ref) <= 1e-4
    for u, gr in zip(U, g_u_ref):
        assert _rel(u.grad.cpu().numpy().astype(np.float64), gr) <= 1e-4
    # Project through autograd: d/dX of <Project(X), Gb> is Gb x_k U_k
    xg = _dev(x).requires_grad_(True)
    U2 = [u.detach().clone().requires_grad_(True) for u in U]
    gbar = np.random.default_rng(7).standard_normal(core.shape)
    (project(xg, U2) * _dev(gbar)).sum().backward()
    gx_ref, gu_ref = tucker_project_vjp(x, factors, _f32(gbar))
    assert _rel(_host(xg.grad, x.shape), gx_ref) <= 1e-5
    for u, gr in zip(U2, gu_ref):
        assert _rel(u.grad.cpu().numpy().astype(np.float64), gr) <= 1e-5


def test_only_requested_outputs_are_written():
    import torch

    from paper_2308_16395_amd.autodiff import _bwd, _prepare, ST_RECONSTRUCT

    x, core, factors = _random_instance((20, 12, 7), (4, 3, 2), 21)
    U = [_devu(u) for u in factors]
    shapes = _prepare(_dev(core), U, "core", "fp32")
    gin, gfac = _bwd(ST_RECONSTRUCT, _dev(core), U, _dev(x), shapes, need_in=False,
                     need_factors=[False, True, False])
    assert gin is None and gfac[0] is None and gfac[2] is None
    # with upstream X (not 2 (X^ - X)) the factor gradient is (X x_{j!=k} U_j^T)_(k) G_(k)^T
    from oracle import unfold

    ref = unfold(multi_ttm(x, factors, transpose=True, skip=1), 1) @ unfold(core, 1).T
    assert _rel(gfac[1].cpu().numpy().astype(np.float64), ref) <= 1e-5
    torch.cuda.synchronize()


def test_bad_arguments_are_rejected():
    import ctypes as C

    from paper_2308_16395_amd.binding import (ST_EINVAL, ST_ESMALL, st_tucker_fwd,
                                              st_tucker_workspace)

    dims = (C.c_int64 * 3)(8, 8, 8)
    bad = (C.c_int64 * 3)(4, 9, 2)  # r_2 > n_2
    ranks = (C.c_int64 * 3)(4, 4, 2)
    nb = C.c_int64()
    assert st_tucker_workspace(3, dims, bad, 0, C.byref(nb)) == ST_EINVAL
    assert st_tucker_workspace(3, dims, ranks, 5, C.byref(nb)) == ST_EINVAL
    assert st_tucker_workspace(3, dims, ranks, 0, C.byref(nb)) == 0 and nb.value > 0
    import torch

    x = torch.zeros(512, device="cuda")
    out = torch.zeros(32, device="cuda")
    us = [torch.zeros(8, r, device="cuda") for r in (4, 4, 2)]
    ptrs = (C.c_void_p * 3)(*[u.data_ptr() for u in us])
    work = torch.zeros(nb.value, dtype=torch.uint8, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert st_tucker_fwd(1, 3, dims, ranks, C.c_void_p(x.data_ptr()), ptrs,
                         C.c_void_p(out.data_ptr()), 0, C.c_void_p(work.data_ptr()),
                         nb.value - 1, s) == ST_ESMALL
    assert st_tucker_fwd(7, 3, dims, ranks, C.c_void_p(x.data_ptr()), ptrs,
                         C.c_void_p(out.data_ptr()), 0, C.c_void_p(work.data_ptr()),
                         nb.value, s) == ST_EINVAL
    null_ptrs = (C.c_void_p * 3)(us[0].data_ptr(), None, us[2].data_ptr())
    assert st_tucker_fwd(1, 3, dims, ranks, C.c_void_p(x.data_ptr()), null_ptrs,
                         C.c_void_p(out.data_ptr()), 0, C.c_void_p(work.data_ptr()),
                         nb.value, s) == ST_EINVAL


def _maxrel(a, b):
    """Largest element-wise difference relative to the largest reference entry."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


_FULL = {}


def _full_window_instance():
    """Inputs and FP64 oracle outputs of the full window, built once per run."""
    if not _FULL:
        dims, ranks = (96, 96, 96, 8, 16), (24, 24, 24, 6, 8)
        rng = np.random.default_rng(2024)
        factors = [_f32(np.linalg.qr(rng.standard_normal((n, r)))[0])
                   for n, r in zip(dims, ranks)]
        core = _f32(rng.standard_normal(ranks))
        ref = tucker_reconstruct(core, factors)
        x = _f32(ref + 0.1 * np.sqrt(np.mean(ref ** 2)) * rng.standard_normal(dims))
        gbar = _f32(rng.standard_normal(ranks))
        _, g_core_ref, g_u_ref = tucker_reconstruct_loss_grad(core, factors, x)
        gx_ref, gu_ref = tucker_project_vjp(x, factors, gbar)
        _FULL.update(dims=dims, ranks=ranks, factors=factors, core=core, x=x, gbar=gbar,
                     upstream=_f32(2.0 * (ref - x)), ref=ref, g_core_ref=g_core_ref,
                     g_u_ref=g_u_ref, proj_ref=tucker_project(x, factors), gx_ref=gx_ref,
                     gu_ref=gu_ref)
    return _FULL


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_window_96cubed_x8_x16(precision):
    """The 96^3 x 8 variables x 16-slice window with ranks (24, 24, 24, 6, 8):
    Reconstruct, Project and both VJPs (dG and every dU_k) against the FP64
    oracle evaluated on the host from the same float32 inputs, element by
    element."""
    import paper_2308_16395_amd.autodiff as ad

    f = _full_window_instance()
    dims, ranks, tol = f["dims"], f["ranks"], TOL[precision]
    U = [_devu(u) for u in f["factors"]]
    g = _dev(f["core"])
    xhat = _host(ad.tucker_reconstruct(g, U, precision), dims)
    assert _maxrel(xhat, f["ref"]) <= tol, ("reconstruct", _maxrel(xhat, f["ref"]))
    del xhat
    # Reconstruct VJP at the loss ||X^ - X||^2 (upstream 2 (X^ - X))
    g_core, g_u = ad.tucker_reconstruct_vjp(g, U, _dev(f["upstream"]), precision)
    assert _maxrel(_host(g_core, ranks), f["g_core_ref"]) <= tol, "dG"
    for k, (gu, gr) in enumerate(zip(g_u, f["g_u_ref"])):
        got = gu.detach().cpu().numpy().astype(np.float64)
        assert _maxrel(got, gr) <= tol, ("dU", k, _maxrel(got, gr))
    # Project and its VJP for an upstream core gradient
    xd = _dev(f["x"])
    gp = _host(ad.tucker_project(xd, U, precision), ranks)
    assert _maxrel(gp, f["proj_ref"]) <= tol, "project"
    g_x, g_u = ad.tucker_project_vjp(xd, U, _dev(f["gbar"]), precision)
    assert _maxrel(_host(g_x, dims), f["gx_ref"]) <= tol, "dX"
    for k, (gu, gr) in enumerate(zip(g_u, f["gu_ref"])):
        got = gu.detach().cpu().numpy().astype(np.float64)
        assert _maxrel(got, gr) <= tol, ("project dU", k, _maxrel(got, gr))
