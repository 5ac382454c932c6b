"""GPU runs of the sine-wave workload of Sec. 5.1 at the paper's size.

100 x 100 x 5000 (two blocks of 2500 slices, streaming-mode rank 11 then 15),
eta = 1e-3, tau = 1e-2. The streaming path (initial ST-HOSVD on 200 slices,
then Alg. 5 slice by slice) is compared with the FP64 oracle on the same
float32 slices: rank decisions at every slice (a divergence is accepted only
at a tie the oracle itself decided within 1e-3 of eps), reconstructions of
probe slices within 1e-5 of the slice norm, the certified bound against the
oracle's, and the rank bump at the first slice of the second block. The
batch path (Alg. 2 over all 5000 slices at once) must return the closed-form
ranks (11, 11, 15) with a true error equal to its certified bound, below tau.
"""

import numpy as np
import pytest

from synth import SINE_WAVE, make_stream
from tests._parity import run_parity

pytestmark = pytest.mark.gpu

TAU = SINE_WAVE["eps"]


@pytest.fixture(scope="module")
def stream():
    return make_stream(SINE_WAVE)


def test_sine_wave_streaming_parity(stream):
    n_init = SINE_WAVE["n_init"]
    res, gpu, orc = run_parity(stream, stream.n_slices, n_init, TAU, probe_every=250)
    if res["diverged_at"] is not None:
        m = res["margin_at_divergence"]
        assert m is not None and m < 1e-3, (res["diverged_at"], m)
    assert res["worst_err"] <= 1e-5, res["worst_err"]
    ranks = res["gpu_ranks"]  # ranks[i]: after slice n_init + i - 1 (i = 0: after init)
    assert all(r[:2] == (11, 11) for r in ranks)
    if res["diverged_at"] is None:
        assert gpu.ranks == orc.ranks
        h = stream.n_half
        assert ranks[h - n_init + 1][2] > ranks[h - n_init][2]  # grows at slice n_half
        assert gpu.ranks[2] >= stream.expected_ranks()[2]
        bound, _ = gpu.recon_error()
        assert bound <= TAU
        np.testing.assert_allclose(bound, orc.recon_error_bound(), rtol=1e-3)


def test_sine_wave_batch_closed_form_ranks(stream):
    import torch

    import paper_2308_16395_amd as pkg

    n = stream.n_slices
    x0 = torch.from_numpy(
        np.concatenate([stream.slice_flat(t).astype(np.float32) for t in range(n)])).cuda()
    gpu = pkg.StreamingTucker(stream.dims, TAU)
    gpu.init(x0, n)
    (r1, r2), _, rb = stream.expected_ranks()
    assert gpu.ranks == (r1, r2, rb)
    bound, xnorm = gpu.recon_error()
    ny = int(np.prod(stream.dims))
    err2 = torch.zeros((), dtype=torch.float64, device="cuda")
    for t in range(n):
        g = gpu.reconstruct_slice(t).double()
        err2 += torch.sum((g - x0[t * ny:(t + 1) * ny].double()) ** 2)
    true_err = float(err2.sqrt()) / xnorm
    # for ST-HOSVD the squared error is exactly the sum of the discarded
    # eigenvalues (Sec. 2.3), so the certified bound is the error itself, up to
    # the FP32 rounding of the data and of the reconstruction
    assert bound <= TAU
    np.testing.assert_allclose(true_err, bound, rtol=1e-3)
