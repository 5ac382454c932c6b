"""GPU parity of the full streaming update (Alg. 5) against the FP64 oracle.

Both sides consume the same float32 slices. Checked at every slice: ranks
identical to the oracle's, and the GPU reconstruction of the new slice and of
probe slices within 1e-5 (FP32) / 1e-4 (bf16x3) of the oracle's, relative to
the slice norm. In the small cases below a rank mismatch is accepted only where
the oracle's own threshold test was within 1e-3 of eps; the comparison stops
there. The tau = 1e-4 cases require every decision to match.
"""

import math

import numpy as np
import pytest

from synth import BlobStream, LowRankStream, make_stream
from oracle import vec
from tests._parity import run_parity, slices32

pytestmark = pytest.mark.gpu


def _assert_parity(res, err_tol):
    if res["diverged_at"] is not None:
        m = res["margin_at_divergence"]
        assert m is not None and m < 1e-3, (res["diverged_at"], m, res["gpu_ranks"][-2:],
                                            res["orc_ranks"][-2:])
    assert res["worst_err"] <= err_tol, res["worst_err"]


def test_lowrank_3way_full_stream():
    """32 x 32 x 100, exact ranks (4, 4, 6) plus noise, tau = 1e-3, init 10."""
    s = make_stream(0)
    res, gpu, orc = run_parity(s, 100, 10, 1e-3)
    assert res["diverged_at"] is None, (res["diverged_at"], res["gpu_ranks"][-1],
                                        res["orc_ranks"][-1])
    assert gpu.ranks == orc.ranks == (4, 4, 6)
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    bound, nx = gpu.recon_error()
    assert bound <= 1e-3
    np.testing.assert_allclose(bound, orc.recon_error_bound(), rtol=1e-3)


@pytest.mark.parametrize("precision,err_tol", [("fp32", 1e-5), ("bf16x3", 1e-4)])
def test_blobs_with_rank_growth(precision, err_tol):
    """4-way slices (space 24 x 20 x 16, 3 variables) with growing ranks."""
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    res, gpu, orc = run_parity(s, 36, 6, 1e-3, precision=precision, err_tol=err_tol)
    grew = sum(any(st["grew"]) for st in res["stats"])
    assert grew > 0  # the case exercises Alg. 4 growth
    _assert_parity(res, err_tol)


def test_blobs_tau1e4_d5_medium_fp64_products():
    """The benchmark's regime at 1/38 of its size: d = 5 (48^3 space x 8
    variables), tau = 1e-4, 80 slices, growth in every mode early on. With exact
    FP64 products on the FP32 data every rank decision matches the oracle."""
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=80, seed=41)
    res, gpu, orc = run_parity(s, 80, 10, 1e-4, precision="fp64", probe_every=5)
    assert res["diverged_at"] is None, (res["diverged_at"], res["margin_at_divergence"])
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    ign_gpu = sum(st["isvd_ignored"] for st in res["stats"])
    ign_orc = sum(h["ignored"] for h in orc.history)
    assert ign_gpu == ign_orc
    # Alg. 3's orthogonality check on the new direction, over all columns of V.
    # After two Gram-Schmidt passes V^T v is about ||V^T V - I||^2 ||d|| / q: V
    # from the Gram-based initial SVD (Alg. 1) is orthonormal to about 1e-8, so
    # the check sits near eps_m = 1e-12 on both sides (the oracle's reaches
    # 2.8e-13 here) and whether it crosses eps_m on a given slice depends on how
    # each side's rounding of V lines up. Checked: the GPU's values are of the
    # oracle's order, and the GPU takes the QR fix exactly where its own check
    # exceeds eps_m.
    grow_gpu = [st["orth_check"] for st in res["stats"] if not st["isvd_ignored"]]
    grow_orc = [h["orth_check"] for h in orc.history if not h["ignored"]]
    assert len(grow_gpu) == len(grow_orc) > 0
    assert all(bool(st["qr_fired"]) == (st["orth_check"] > 1e-12) for st in res["stats"])
    assert max(grow_gpu) <= 10.0 * max(grow_orc), (sorted(grow_gpu)[-5:], max(grow_orc))


FAST = [("fp32", "literal", 1e-5), ("fp32", "factored", 1e-5), ("bf16x3", "literal", 1e-4),
        ("bf16x3", "factored", 1e-4)]


@pytest.mark.parametrize("precision,core_update,err_tol", FAST,
                         ids=[f"{p}-{c}" for p, c, _ in FAST])
def test_blobs_tau1e4_d5_medium_fast_forms(precision, core_update, err_tol):
    """Same stream with FP32-accumulated or split-bf16 products. Decisions near
    a threshold (the guard band) and every growth are taken on FP64 products,
    so every rank decision matches the oracle's and the model stays within the
    error bar of the oracle's at every probe."""
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=80, seed=41)
    res, gpu, orc = run_parity(s, 80, 10, 1e-4, precision=precision, probe_every=5,
                               core_update=core_update)
    assert res["diverged_at"] is None, (res["diverged_at"], res["margin_at_divergence"])
    assert res["worst_err"] <= err_tol, res["worst_err"]
    refined = sum(st["refined_isvd"] or st["refined_modes"] for st in res["stats"])
    grew = sum(not h["ignored"] or any(h["grew"]) for h in orc.history)
    # every growing slice was decided on FP64 products
    assert refined >= grew


def test_matrix_stream_d2():
    """d = 2: the update reduces to the incremental SVD of a growing matrix."""
    rng = np.random.default_rng(5)
    a = rng.standard_normal((50, 6)) @ rng.standard_normal((6, 40)) + 1e-3 * rng.standard_normal((50, 40))

    class M:
        dims = (40,)

        def slice_flat(self, t):
            return a[t]

    res, gpu, orc = run_parity(M(), 50, 4, 1e-2)
    _assert_parity(res, 1e-5)


def test_ragged_sizes_and_guarantee():
    """Slice dims that are not multiples of the MFMA tiles; tau met by the GPU model."""
    s = BlobStream((19, 13, 7), 5, 5, (1.5, 3.0), 0.6, n_slices=30, seed=33)
    tau = 2e-3
    res, gpu, orc = run_parity(s, 30, 5, tau)
    _assert_parity(res, 1e-5)
    import torch  # noqa: F401

    flat, shaped = slices32(s, 30)
    err2 = 0.0
    nrm2 = 0.0
    for t in range(30):
        g = gpu.reconstruct_slice(t).cpu().numpy().astype(np.float64)
        err2 += np.sum((g - flat[t].astype(np.float64)) ** 2)
        nrm2 += np.sum(flat[t].astype(np.float64) ** 2)
    assert math.sqrt(err2 / nrm2) <= tau * (1 + 1e-3)


def test_errors_leave_state_unchanged():
    import torch

    import paper_2308_16395_amd as pkg
    from paper_2308_16395_amd.binding import ST_ENONFINITE, ST_ESTATE, StError

    s = LowRankStream((16, 12), 20, (3, 2, 4), 1e-3, seed=4)
    flat, _ = slices32(s, 20)
    gpu = pkg.StreamingTucker(s.dims, 1e-2)
    with pytest.raises(StError) as ei:
        gpu.update(torch.from_numpy(flat[0]).cuda())
    assert ei.value.code == ST_ESTATE
    gpu.init(torch.from_numpy(np.concatenate(flat[:5])).cuda(), 5)
    gpu.update(torch.from_numpy(flat[5]).cuda())
    core0 = gpu.core().cpu().numpy().copy()
    ranks0, nd0 = gpu.ranks, gpu.n_slices
    bad = flat[6].copy()
    bad[7] = np.nan
    with pytest.raises(StError) as ei:
        gpu.update(torch.from_numpy(bad).cuda())
    assert ei.value.code == ST_ENONFINITE
    assert gpu.ranks == ranks0 and gpu.n_slices == nd0
    np.testing.assert_array_equal(gpu.core().cpu().numpy(), core0)
    # a zero slice is a valid update that changes no rank
    gpu.update(torch.zeros(len(flat[0]), device="cuda"))
    assert gpu.ranks == ranks0 and gpu.n_slices == nd0 + 1
    assert torch.count_nonzero(gpu.reconstruct_slice(nd0)).item() == 0


@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_streaming_rank_past_500(core_update):
    """Noise slices of 24 x 24 (R = 576): every slice adds a direction, so the
    streaming rank passes 500, where the host buffers for the per-update results
    (p, p2, S) regrow. Ranks after every slice and S against the oracle."""
    import torch

    import paper_2308_16395_amd as pkg
    from oracle import StreamingTucker as Oracle

    rng = np.random.default_rng(77)
    n_init, n = 490, 505
    x = rng.standard_normal((n, 24 * 24)).astype(np.float32)
    shaped = [x[t].astype(np.float64).reshape((24, 24), order="F") for t in range(n)]
    tau = 1e-7
    orc = Oracle(np.stack(shaped[:n_init], axis=-1), tau, core_update=core_update)
    gpu = pkg.StreamingTucker((24, 24), tau, precision="fp64", core_update=core_update)
    gpu.init(torch.from_numpy(x[:n_init].reshape(-1)).cuda(), n_init)
    assert gpu.ranks == orc.ranks == (24, 24, n_init)
    for t in range(n_init, n):
        gpu.update(torch.from_numpy(x[t]).cuda())
        orc.update(shaped[t])
        assert gpu.ranks == orc.ranks, (t, gpu.ranks, orc.ranks)
    assert gpu.ranks[-1] > 500
    np.testing.assert_allclose(gpu.sv(), orc.S, rtol=1e-9)
    for probe in (0, n_init, n - 1):
        g = gpu.reconstruct_slice(probe).cpu().numpy().astype(np.float64)
        o = vec(orc.reconstruct_slice(probe))
        assert np.linalg.norm(g - o) <= 1e-5 * np.linalg.norm(shaped[probe])
