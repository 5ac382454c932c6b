"""GPU parity of the block update (b slices per call, st_update_block) against
the oracle's update_block on the same float32 slices: ranks after every block,
the number of kept residual directions, reconstructions of probe slices
(within 1e-5 of the slice norm: the literal core is stored in FP32), the
singular values and the certified bound; a ragged last block; the forced QR
fix of the block orthogonality check; b = 1 against the single-slice update;
the factored core form; threshold blocks.
"""

import numpy as np
import pytest

from oracle import StreamingTucker as Oracle
from oracle import vec
from synth import BlobStream
from tests._parity import slices32

pytestmark = pytest.mark.gpu


def _run(s, n, n_init, tau, bsize, precision="fp64", orth_tol=0.0, eps_m=1e-12,
         core_update="literal"):
    import torch

    import paper_2308_16395_amd as pkg

    flat, shaped = slices32(s, n)
    orc = Oracle(np.stack(shaped[:n_init], axis=-1), tau, eps_m=eps_m, core_update=core_update)
    gpu = pkg.StreamingTucker(s.dims, tau, precision=precision, orth_tol=orth_tol,
                              core_update=core_update)
    gpu.init(torch.from_numpy(np.concatenate(flat[:n_init])).cuda(), n_init)
    assert gpu.ranks == orc.ranks
    worst, t, stats = 0.0, n_init, []
    while t < n:
        b = min(bsize, n - t)
        y = torch.from_numpy(np.concatenate(flat[t:t + b])).cuda()
        gpu.update_block(y, b)
        rec = orc.update_block(np.stack(shaped[t:t + b], axis=-1))
        st = gpu.stats()
        stats.append((st, rec))
        assert gpu.ranks == orc.ranks, (t, gpu.ranks, orc.ranks, rec["lam"], rec["eps"])
        t += b
        for probe in sorted({0, t - 1, (n_init + t) // 2}):
            g = gpu.reconstruct_slice(probe).cpu().numpy().astype(np.float64)
            o = vec(orc.reconstruct_slice(probe))
            worst = max(worst, np.linalg.norm(g - o) / np.linalg.norm(shaped[probe]))
    return gpu, orc, worst, stats


def _check_s_and_bound(gpu, orc, rel):
    s_gpu, s_orc = np.asarray(gpu.sv()), np.asarray(orc.S)
    assert s_gpu.shape == s_orc.shape
    assert np.max(np.abs(s_gpu - s_orc)) <= rel * s_orc[0], np.max(np.abs(s_gpu - s_orc))
    bound, _ = gpu.recon_error()
    np.testing.assert_allclose(bound, orc.recon_error_bound(), rtol=1e-3)
    assert bound <= orc.tau


@pytest.mark.parametrize("bsize", [3, 4])
def test_block_updates_fp64_products(bsize):
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    gpu, orc, worst, stats = _run(s, 36, 6, 1e-3, bsize)
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9)
    assert gpu.ranks[-1] == orc.ranks[-1] and sum(rec["ell"] for _, rec in stats) > 5


@pytest.mark.parametrize("precision,bsize", [("fp32", 3), ("bf16x3", 5)])
def test_block_updates_fast_forms(precision, bsize):
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    gpu, orc, worst, _ = _run(s, 36, 6, 1e-3, bsize, precision=precision)
    assert worst <= (1e-5 if precision == "fp32" else 1e-4), worst
    _check_s_and_bound(gpu, orc, 1e-5)


def test_block_updates_medium_stream():
    """48^3 x 8 blobs, tau = 1e-4 (growth in every mode), blocks of 4."""
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=42, seed=41)
    gpu, orc, worst, _ = _run(s, 42, 10, 1e-4, 4)
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9)


def test_block_qr_fix_forced():
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    gpu, orc, worst, stats = _run(s, 36, 6, 1e-3, 3, orth_tol=1e-300, eps_m=0.0)
    fired_gpu = [bool(st["qr_fired"]) for st, _ in stats]
    fired_orc = [bool(rec["qr"]) for _, rec in stats]
    assert fired_gpu == fired_orc and sum(fired_gpu) >= 5
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9)
    v = gpu.aux_v()
    import torch

    g = v.T @ v
    assert torch.max(torch.abs(g - torch.eye(g.shape[0], device=g.device, dtype=g.dtype))) < 1e-8


def test_block_of_one_is_update():
    import torch

    import paper_2308_16395_amd as pkg

    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=20, seed=21)
    flat, _ = slices32(s, 20)
    x0 = torch.from_numpy(np.concatenate(flat[:6])).cuda()
    a = pkg.StreamingTucker(s.dims, 1e-3, precision="fp64")
    b = pkg.StreamingTucker(s.dims, 1e-3, precision="fp64")
    a.init(x0, 6)
    b.init(x0, 6)
    for t in range(6, 20):
        y = torch.from_numpy(flat[t]).cuda()
        a.update(y)
        b.update_block(y, 1)
        assert a.ranks == b.ranks
    np.testing.assert_array_equal(np.asarray(a.sv()), np.asarray(b.sv()))


@pytest.mark.parametrize("precision,bsize", [("fp64", 3), ("fp64", 4), ("fp32", 5)])
def test_block_updates_factored(precision, bsize):
    """The factored core form (V = V0 M): the block's residual directions Q are
    appended to V0 and M, G0 = V0^T V0 extended; against the oracle's factored
    block updates."""
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    gpu, orc, worst, stats = _run(s, 36, 6, 1e-3, bsize, precision=precision,
                                  core_update="factored")
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9 if precision == "fp64" else 1e-5)
    assert sum(rec["ell"] for _, rec in stats) > 5
    # V = V0 M stays orthonormal
    import torch

    v = gpu.aux_v()
    g = v.T @ v
    assert torch.max(torch.abs(g - torch.eye(g.shape[0], device=g.device, dtype=g.dtype))) < 1e-9


def test_block_updates_factored_medium_stream_and_qr_fix():
    """48^3 x 8 blobs in blocks of 4 in the factored form; then the forced QR
    fix of the block orthogonality check in the factored form."""
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=42, seed=41)
    gpu, orc, worst, _ = _run(s, 42, 10, 1e-4, 4, core_update="factored")
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9)
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    gpu, orc, worst, stats = _run(s, 36, 6, 1e-3, 3, orth_tol=1e-300, eps_m=0.0,
                                  core_update="factored")
    fired_gpu = [bool(st["qr_fired"]) for st, _ in stats]
    fired_orc = [bool(rec["qr"]) for _, rec in stats]
    assert fired_gpu == fired_orc and sum(fired_gpu) >= 5
    assert worst <= 1e-5, worst
    _check_s_and_bound(gpu, orc, 1e-9)


@pytest.mark.parametrize("level", [0.55, 0.60, 0.80])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_block_threshold_decisions(level, precision):
    """The oracle's block-tolerance pins (residual parts of level * tau ||Y_B||
    in both slice modes and the streaming mode, eps_B = tau ||Y_B|| / sqrt(3))
    through st_update_block: the same growth decisions and ranks, and the
    certified bound up to the products' rounding."""
    import torch

    import paper_2308_16395_amd as pkg
    from tests.test_oracle_block import _block_threshold_case

    x0, yb, tau = _block_threshold_case(level)
    orc = Oracle(x0, tau)
    rec = orc.update_block(yb)
    gpu = pkg.StreamingTucker(x0.shape[:-1], tau, precision=precision)
    flat = lambda a: torch.from_numpy(  # noqa: E731
        np.concatenate([vec(a[..., t]) for t in range(a.shape[-1])]).astype(np.float32)).cuda()
    gpu.init(flat(x0), x0.shape[-1])
    gpu.update_block(flat(yb), yb.shape[-1])
    assert gpu.ranks == orc.ranks, (gpu.ranks, orc.ranks, rec["grew"], rec["ell"])
    bound, _ = gpu.recon_error()
    # FP32 Gram products leave rounding-level eigenvalues (about u32 ||E||^2)
    # in the discarded tail: an absolute 5e-5 of ||X|| at tau = 0.1
    atol = 1e-7 if precision == "fp64" else 5e-5
    assert bound == pytest.approx(orc.recon_error_bound(), rel=1e-4, abs=atol)
