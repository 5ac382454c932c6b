"""Pins for the oracle's Tucker gradients (multi-TTM chains of Sec. 2.1).

FP64 central differences (h = 1e-6) on a 12 x 12 x 12 x 4 window of 4 slices
with ranks (3, 3, 3, 2, 2), the closed form of the core gradient for
orthonormal factors, and a zero gradient at an exact fit.
"""

import numpy as np

from oracle import (multi_ttm, sthosvd, tucker_project, tucker_project_vjp,
                    tucker_reconstruct, tucker_reconstruct_loss_grad)
from synth import BlobStream


def _instance(seed=3):
    bs = BlobStream((12, 12, 12), 4, 4, (1.5, 3.0), 0.5, n_slices=4, seed=seed)
    x = np.stack([bs.slice(t) for t in range(4)], axis=-1)
    res = sthosvd(x, 0.0, ranks=(3, 3, 3, 2, 2))
    rng = np.random.default_rng(seed)
    core = res["core"] + 1e-2 * np.linalg.norm(res["core"]) * rng.standard_normal(res["core"].shape)
    return x, core, res["factors"]


def _loss(core, factors, x):
    return float(np.sum((tucker_reconstruct(core, factors) - x) ** 2))


def test_reconstruct_grad_central_differences():
    x, core, factors = _instance()
    loss, g_core, g_u = tucker_reconstruct_loss_grad(core, factors, x)
    assert abs(loss - _loss(core, factors, x)) <= 1e-12 * loss
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(40):
        idx = tuple(rng.integers(0, n) for n in core.shape)
        cp, cm = core.copy(), core.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (_loss(cp, factors, x) - _loss(cm, factors, x)) / (2 * h)
        assert abs(fd - g_core[idx]) <= 1e-6 * max(1.0, np.abs(g_core).max())
    for k, u in enumerate(factors):
        for _ in range(15):
            i, j = rng.integers(0, u.shape[0]), rng.integers(0, u.shape[1])
            fp = [f.copy() for f in factors]
            fm = [f.copy() for f in factors]
            fp[k][i, j] += h
            fm[k][i, j] -= h
            fd = (_loss(core, fp, x) - _loss(core, fm, x)) / (2 * h)
            assert abs(fd - g_u[k][i, j]) <= 1e-6 * max(1.0, np.abs(g_u[k]).max())


def test_core_grad_closed_form_and_zero_at_exact_fit():
    x, core, factors = _instance(4)
    _, g_core, _ = tucker_reconstruct_loss_grad(core, factors, x)
    # orthonormal U_k: dL/dG = 2 (G - X x_k U_k^T)
    np.testing.assert_allclose(g_core, 2.0 * (core - multi_ttm(x, factors, transpose=True)),
                               atol=1e-11 * np.abs(g_core).max())
    xfit = tucker_reconstruct(core, factors)
    loss, g_core0, g_u0 = tucker_reconstruct_loss_grad(core, factors, xfit)
    assert loss <= 1e-24 * np.sum(xfit ** 2)
    assert np.abs(g_core0).max() <= 1e-12 * np.abs(core).max()
    for g in g_u0:
        assert np.abs(g).max() <= 1e-11 * np.abs(core).max() * np.abs(xfit).max()


def test_project_vjp_central_differences():
    x, _, factors = _instance(5)
    rng = np.random.default_rng(1)
    g_up = rng.standard_normal(tucker_project(x, factors).shape)
    g_x, g_u = tucker_project_vjp(x, factors, g_up)

    def functional(xx, ff):
        return float(np.sum(g_up * tucker_project(xx, ff)))

    h = 1e-6
    for _ in range(20):
        idx = tuple(rng.integers(0, n) for n in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (functional(xp, factors) - functional(xm, factors)) / (2 * h)
        assert abs(fd - g_x[idx]) <= 1e-7 * max(1.0, np.abs(g_x).max())
    for k, u in enumerate(factors):
        for _ in range(10):
            i, j = rng.integers(0, u.shape[0]), rng.integers(0, u.shape[1])
            fp = [f.copy() for f in factors]
            fm = [f.copy() for f in factors]
            fp[k][i, j] += h
            fm[k][i, j] -= h
            fd = (functional(x, fp) - functional(x, fm)) / (2 * h)
            assert abs(fd - g_u[k][i, j]) <= 1e-6 * max(1.0, np.abs(g_u[k]).max())
