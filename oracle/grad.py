"""FP64 gradients of Tucker reconstruction and projection (test infrastructure).

Both maps are multi-TTM chains (Sec. 2.1, eq. tucker_matrix): with
K_k = U_d (x) ... (x) U_{k+1} (x) U_{k-1} (x) ... (x) U_1,

* Reconstruct: X^ = G x_1 U_1 ... x_d U_d, so X^_(k) = U_k G_(k) K_k^T.
  For L = ||X^ - X||_F^2 and R = 2 (X^ - X):
  dL/dG = R x_1 U_1^T ... x_d U_d^T and dL/dU_k = (R x_{j != k} U_j^T)_(k) G_(k)^T.
* Project: G = X x_1 U_1^T ... x_d U_d^T, so G_(k) = U_k^T X_(k) K_k.
  For an upstream gradient Gbar: dX = Gbar x_1 U_1 ... x_d U_d and
  dU_k = (X x_{j != k} U_j^T)_(k) Gbar_(k)^T.

Only the test suite and the benchmark's CPU-baseline leg use this module.
"""

from __future__ import annotations

import numpy as np

from .tucker import multi_ttm, unfold


def tucker_reconstruct(core, factors):
    return multi_ttm(np.asarray(core, dtype=np.float64), factors)


def tucker_reconstruct_loss_grad(core, factors, x):
    """Loss ||G x_k U_k - X||^2 and its gradients (dG, [dU_k])."""
    core = np.asarray(core, dtype=np.float64)
    xhat = multi_ttm(core, factors)
    resid = 2.0 * (xhat - x)
    loss = float(np.sum((xhat - x) ** 2))
    g_core = multi_ttm(resid, factors, transpose=True)
    g_u = []
    for k in range(core.ndim):
        part = multi_ttm(resid, factors, transpose=True, skip=k)
        g_u.append(unfold(part, k) @ unfold(core, k).T)
    return loss, g_core, g_u


def tucker_project(x, factors):
    return multi_ttm(np.asarray(x, dtype=np.float64), factors, transpose=True)


def tucker_project_vjp(x, factors, g_core):
    """Vector-Jacobian product of Project at X for the upstream gradient."""
    x = np.asarray(x, dtype=np.float64)
    g_x = multi_ttm(np.asarray(g_core, dtype=np.float64), factors)
    g_u = []
    for k in range(x.ndim):
        part = multi_ttm(x, factors, transpose=True, skip=k)
        g_u.append(unfold(part, k) @ unfold(g_core, k).T)
    return g_x, g_u
