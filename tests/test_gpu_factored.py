"""GPU parity of the factored streaming form (V = V0 M, C = V x_d S) against
the FP64 oracle run with the same core update, through the C ABI.

Checked as for the literal form: ranks identical after every slice and the
reconstructions of the new slice and of probe slices within 1e-5 (FP32) /
1e-4 (bf16x3) of the oracle's, relative to the slice norm. The rank decisions
do not depend on the core update, so the factored and literal GPU forms must
agree on them, and the factored core must equal V x_d S.
"""

import math

import numpy as np
import pytest

from synth import BlobStream, LowRankStream, make_stream
from tests._parity import run_parity, slices32

pytestmark = pytest.mark.gpu


def test_lowrank_3way_full_stream_factored():
    s = make_stream(0)
    res, gpu, orc = run_parity(s, 100, 10, 1e-3, core_update="factored")
    assert res["diverged_at"] is None, (res["diverged_at"], res["gpu_ranks"][-1])
    assert gpu.ranks == orc.ranks == (4, 4, 6)
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    bound, _ = gpu.recon_error()
    np.testing.assert_allclose(bound, orc.recon_error_bound(), rtol=1e-3)


@pytest.mark.parametrize("precision,err_tol", [("fp32", 1e-5), ("bf16x3", 1e-4)])
def test_blobs_with_rank_growth_factored(precision, err_tol):
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    res, gpu, orc = run_parity(s, 36, 6, 1e-3, precision=precision, err_tol=err_tol,
                               core_update="factored")
    assert sum(any(st["grew"]) for st in res["stats"]) > 0
    if res["diverged_at"] is not None:
        assert res["margin_at_divergence"] is not None and res["margin_at_divergence"] < 1e-3
    assert res["worst_err"] <= err_tol, res["worst_err"]


def test_blobs_tau1e4_d5_medium_factored_fp64():
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=80, seed=41)
    res, gpu, orc = run_parity(s, 80, 10, 1e-4, precision="fp64", probe_every=5,
                               core_update="factored")
    assert res["diverged_at"] is None, (res["diverged_at"], res["margin_at_divergence"])
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    assert sum(st["isvd_ignored"] for st in res["stats"]) == sum(h["ignored"] for h in orc.history)


def test_matrix_stream_d2_factored():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((50, 6)) @ rng.standard_normal((6, 40)) + 1e-3 * rng.standard_normal((50, 40))

    class M:
        dims = (40,)

        def slice_flat(self, t):
            return a[t]

    res, gpu, orc = run_parity(M(), 50, 4, 1e-2, core_update="factored")
    assert res["diverged_at"] is None
    assert res["worst_err"] <= 1e-5, res["worst_err"]


def test_ragged_factored_meets_tau_and_matches_literal_ranks():
    import torch

    import paper_2308_16395_amd as pkg

    s = BlobStream((19, 13, 7), 5, 5, (1.5, 3.0), 0.6, n_slices=30, seed=33)
    tau = 2e-3
    res, gpu, orc = run_parity(s, 30, 5, tau, core_update="factored")
    assert res["diverged_at"] is None
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    flat, _ = slices32(s, 30)
    lit = pkg.StreamingTucker(s.dims, tau)
    lit.init(torch.from_numpy(np.concatenate(flat[:5])).cuda(), 5)
    for t in range(5, 30):
        lit.update(torch.from_numpy(flat[t]).cuda())
    assert lit.ranks == gpu.ranks
    err2 = nrm2 = 0.0
    for t in range(30):
        g = gpu.reconstruct_slice(t).cpu().numpy().astype(np.float64)
        err2 += np.sum((g - flat[t].astype(np.float64)) ** 2)
        nrm2 += np.sum(flat[t].astype(np.float64) ** 2)
    assert math.sqrt(err2 / nrm2) <= tau * (1 + 1e-3)
    # C = V x_d S and V has orthonormal columns
    v = gpu.aux_v()
    sv = np.asarray(gpu.sv())
    core = gpu.core().double().cpu().numpy()
    vs = (v.cpu().numpy() * sv[None, :]).ravel(order="F")
    np.testing.assert_allclose(core, vs, rtol=0, atol=1e-6 * np.abs(vs).max())
    g = v.T @ v
    assert torch.max(torch.abs(g - torch.eye(g.shape[0], device=g.device, dtype=g.dtype))) < 1e-6


def test_factored_errors_leave_state_unchanged():
    import torch

    import paper_2308_16395_amd as pkg
    from paper_2308_16395_amd.binding import ST_ENONFINITE, StError

    s = LowRankStream((16, 12), 20, (3, 2, 4), 1e-3, seed=4)
    flat, _ = slices32(s, 20)
    gpu = pkg.StreamingTucker(s.dims, 1e-2, core_update="factored")
    gpu.init(torch.from_numpy(np.concatenate(flat[:5])).cuda(), 5)
    gpu.update(torch.from_numpy(flat[5]).cuda())
    core0 = gpu.core().cpu().numpy().copy()
    ranks0, nd0 = gpu.ranks, gpu.n_slices
    bad = flat[6].copy()
    bad[3] = np.inf
    with pytest.raises(StError) as ei:
        gpu.update(torch.from_numpy(bad).cuda())
    assert ei.value.code == ST_ENONFINITE
    assert gpu.ranks == ranks0 and gpu.n_slices == nd0
    np.testing.assert_array_equal(gpu.core().cpu().numpy(), core0)
    for t in range(6, 20):
        gpu.update(torch.from_numpy(flat[t]).cuda())
    assert gpu.n_slices == 20
