"""Reconstruct / Project of a Tucker model with their VJPs, as torch autograd
functions over st_tucker_fwd / st_tucker_bwd (argument marshalling only).

Tensors follow the library's layout: a tensor of shape (n_1, ..., n_d) is a
flat float32 CUDA tensor in column-major order (first index fastest); a factor
U_k is an (n_k, r_k) float32 CUDA tensor stored column-major (``colmajor``
makes one). Every TTM and every gradient contraction runs in the library.
"""

from __future__ import annotations

import ctypes as C
import math

from .binding import (PRECISIONS, ST_OK, ST_PROJECT, ST_RECONSTRUCT, StError, _ready,
                      st_last_error, st_tucker_bwd, st_tucker_fwd, st_tucker_workspace)


def colmajor(u):
    """The same matrix stored column-major (stride (1, rows))."""
    return u.t().contiguous().t()


def _check_factor(u, n, r):
    if tuple(u.shape) != (n, r) or u.dtype.itemsize != 4 or not u.is_cuda:
        raise ValueError(f"factor must be a float32 CUDA tensor of shape ({n}, {r})")
    if r > 1 and n > 1 and u.stride() != (1, n):
        raise ValueError("factor must be column-major; use colmajor(u)")


class _Shapes:
    def __init__(self, dims, ranks, precision):
        self.dims = tuple(int(n) for n in dims)
        self.ranks = tuple(int(r) for r in ranks)
        if len(self.dims) != len(self.ranks):
            raise ValueError("dims and ranks differ in length")
        self.d = len(self.dims)
        self.cdims = (C.c_int64 * self.d)(*self.dims)
        self.cranks = (C.c_int64 * self.d)(*self.ranks)
        self.prec = PRECISIONS[precision]
        nbytes = C.c_int64()
        rc = st_tucker_workspace(self.d, self.cdims, self.cranks, self.prec, C.byref(nbytes))
        if rc != ST_OK:
            raise StError(rc, st_last_error(None).decode())
        self.work_bytes = nbytes.value
        self.n_full = math.prod(self.dims)
        self.n_core = math.prod(self.ranks)


_workspaces = {}


def _workspace(shapes, device):
    import torch

    key = (shapes.dims, shapes.ranks, shapes.prec, str(device))
    w = _workspaces.get(key)
    if w is None:
        w = torch.empty(max(shapes.work_bytes, 1), dtype=torch.uint8, device=device)
        _workspaces[key] = w
    return w


def _ptrs(tensors):
    return (C.c_void_p * len(tensors))(*[C.c_void_p(t.data_ptr()) if t is not None else None
                                          for t in tensors])


def _stream():
    # the library runs on its own runtime's null stream after torch's work is done
    _ready()
    return None


def _fwd(op, x, factors, shapes):
    import torch

    n_out = shapes.n_full if op == ST_RECONSTRUCT else shapes.n_core
    out = torch.empty(n_out, dtype=torch.float32, device=x.device)
    work = _workspace(shapes, x.device)
    rc = st_tucker_fwd(op, shapes.d, shapes.cdims, shapes.cranks, C.c_void_p(x.data_ptr()),
                       _ptrs(factors), C.c_void_p(out.data_ptr()), shapes.prec,
                       C.c_void_p(work.data_ptr()), shapes.work_bytes, _stream())
    if rc != ST_OK:
        raise StError(rc, st_last_error(None).decode())
    return out


def _bwd(op, x, factors, gout, shapes, need_in=True, need_factors=None):
    import torch

    n_in = shapes.n_core if op == ST_RECONSTRUCT else shapes.n_full
    gin = torch.empty(n_in, dtype=torch.float32, device=x.device) if need_in else None
    if need_factors is None:
        need_factors = [True] * shapes.d
    gfac = [colmajor(torch.empty(n, r, dtype=torch.float32, device=x.device)) if need else None
            for n, r, need in zip(shapes.dims, shapes.ranks, need_factors)]
    work = _workspace(shapes, x.device)
    rc = st_tucker_bwd(op, shapes.d, shapes.cdims, shapes.cranks, C.c_void_p(x.data_ptr()),
                       _ptrs(factors), C.c_void_p(gout.data_ptr()),
                       C.c_void_p(gin.data_ptr()) if gin is not None else None, _ptrs(gfac),
                       shapes.prec, C.c_void_p(work.data_ptr()), shapes.work_bytes, _stream())
    if rc != ST_OK:
        raise StError(rc, st_last_error(None).decode())
    return gin, gfac


def _prepare(x, factors, expect, precision):
    dims = tuple(int(u.shape[0]) for u in factors)
    ranks = tuple(int(u.shape[1]) for u in factors)
    shapes = _Shapes(dims, ranks, precision)
    for u, n, r in zip(factors, dims, ranks):
        _check_factor(u, n, r)
    want = shapes.n_core if expect == "core" else shapes.n_full
    if x.dim() != 1 or x.numel() != want or not x.is_contiguous():
        raise ValueError(f"expected a flat contiguous tensor of {want} elements")
    return shapes


def tucker_reconstruct(core, factors, precision="fp32"):
    """X^ = G x_1 U_1 ... x_d U_d (flat, column-major)."""
    shapes = _prepare(core, factors, "core", precision)
    return _fwd(ST_RECONSTRUCT, core, factors, shapes)


def tucker_project(x, factors, precision="fp32"):
    """G = X x_1 U_1^T ... x_d U_d^T (flat, column-major)."""
    shapes = _prepare(x, factors, "full", precision)
    return _fwd(ST_PROJECT, x, factors, shapes)


def tucker_reconstruct_vjp(core, factors, g_xhat, precision="fp32"):
    """(dG, [dU_k]) of Reconstruct at (G, U) for the upstream gradient g_xhat."""
    shapes = _prepare(core, factors, "core", precision)
    return _bwd(ST_RECONSTRUCT, core, factors, g_xhat.contiguous(), shapes)


def tucker_project_vjp(x, factors, g_core, precision="fp32"):
    """(dX, [dU_k]) of Project at (X, U) for the upstream gradient g_core."""
    shapes = _prepare(x, factors, "full", precision)
    return _bwd(ST_PROJECT, x, factors, g_core.contiguous(), shapes)


def _autograd():
    import torch

    class TuckerReconstruct(torch.autograd.Function):
        """apply(core, precision, *factors) -> X^ (flat)."""

        @staticmethod
        def forward(ctx, core, precision, *factors):
            shapes = _prepare(core, factors, "core", precision)
            ctx.shapes = shapes
            ctx.save_for_backward(core, *factors)
            return _fwd(ST_RECONSTRUCT, core, factors, shapes)

        @staticmethod
        def backward(ctx, g):
            core, *factors = ctx.saved_tensors
            need = ctx.needs_input_grad
            gin, gfac = _bwd(ST_RECONSTRUCT, core, factors, g.contiguous(), ctx.shapes,
                             need_in=need[0], need_factors=list(need[2:]))
            return (gin, None, *gfac)

    class TuckerProject(torch.autograd.Function):
        """apply(x, precision, *factors) -> G (flat)."""

        @staticmethod
        def forward(ctx, x, precision, *factors):
            shapes = _prepare(x, factors, "full", precision)
            ctx.shapes = shapes
            ctx.save_for_backward(x, *factors)
            return _fwd(ST_PROJECT, x, factors, shapes)

        @staticmethod
        def backward(ctx, g):
            x, *factors = ctx.saved_tensors
            need = ctx.needs_input_grad
            gin, gfac = _bwd(ST_PROJECT, x, factors, g.contiguous(), ctx.shapes,
                             need_in=need[0], need_factors=list(need[2:]))
            return (gin, None, *gfac)

    return TuckerReconstruct, TuckerProject


_fns = None


def reconstruct(core, factors, precision="fp32"):
    """Differentiable X^ = G x_1 U_1 ... x_d U_d."""
    global _fns
    if _fns is None:
        _fns = _autograd()
    return _fns[0].apply(core, precision, *factors)


def project(x, factors, precision="fp32"):
    """Differentiable G = X x_1 U_1^T ... x_d U_d^T."""
    global _fns
    if _fns is None:
        _fns = _autograd()
    return _fns[1].apply(x, precision, *factors)
