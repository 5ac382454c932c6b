"""GPU parity of Alg. 3's QR fix: the orthogonality check of the new direction
v against every column of V and, when it exceeds eps_m, the re-factorisation
[V v] = Q R with S' replaced by S' R^T and its SVD taken densely.

The check sits at the rounding level on ordinary streams (it never fires at the
paper's small eps_m), so the fix is forced: the GPU runs with orth_tol = 1e-300
and the oracle with eps_m = 0, and both take it on every growing slice. Ranks
must agree after every update, the fix must fire on exactly the oracle's
slices, reconstructions must agree with the oracle's to the FP32 rounding of
the reconstructed slice (and of the literal form's FP32 core), and the singular
values (FP64) and the orthonormality of V must be those of the oracle.
"""

import numpy as np
import pytest

from synth import BlobStream
from tests._parity import run_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_qr_fix_forced_on_every_growth(core_update):
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    res, gpu, orc = run_parity(s, 36, 6, 1e-3, precision="fp64", core_update=core_update,
                               orth_tol=1e-300, eps_m=0.0)
    assert res["diverged_at"] is None, (res["diverged_at"], res["margin_at_divergence"])
    fired_gpu = [bool(st["qr_fired"]) for st in res["stats"]]
    fired_orc = [bool(h["qr"]) for h in orc.history]
    assert fired_gpu == fired_orc and sum(fired_gpu) >= 5, (fired_gpu, fired_orc)
    assert res["worst_err"] <= 2e-6, res["worst_err"]
    np.testing.assert_allclose(gpu.sv(), orc.S, rtol=1e-9)
    v = gpu.aux_v().double()
    import torch

    g = v.T @ v
    assert torch.max(torch.abs(g - torch.eye(g.shape[0], device=g.device, dtype=g.dtype))) < 1e-8


def test_qr_fix_forced_medium_stream():
    """The 48^3 x 8 blob stream at tau = 1e-4 (growth on every slice)."""
    s = BlobStream((48, 48, 48), 8, 16, (3.0, 8.0), 0.5, n_slices=40, seed=41)
    res, gpu, orc = run_parity(s, 40, 10, 1e-4, precision="fp64", probe_every=5,
                               orth_tol=1e-300, eps_m=0.0)
    assert res["diverged_at"] is None, (res["diverged_at"], res["margin_at_divergence"])
    fired_gpu = [bool(st["qr_fired"]) for st in res["stats"]]
    assert fired_gpu == [bool(h["qr"]) for h in orc.history]
    assert sum(fired_gpu) >= 20
    assert res["worst_err"] <= 2e-6, res["worst_err"]
    # 36 singular values spanning five decades: the small ones carry the
    # absolute rounding of 30 FP64 updates at the scale of the largest
    s_gpu, s_orc = np.asarray(gpu.sv()), np.asarray(orc.S)
    assert s_gpu.shape == s_orc.shape
    assert np.max(np.abs(s_gpu - s_orc)) <= 1e-10 * s_orc[0], np.max(np.abs(s_gpu - s_orc))
