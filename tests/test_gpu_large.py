"""GPU on the 512 x 512 x 256 random-Fourier stream (tau = 1e-4): the
workload with the longest fibres (n = 512, so the FP64 Gram of the initial
decomposition runs over row-chunk pairs) and ranks near 128 in every spatial
mode.

The oracle cannot run at this size inside a test, so the checks are properties
that hold at any size: the certified bound and the true error of the stored
slices are within tau after init and after each form's updates, the spatial
factors and V are orthonormal, S is positive and sorted, the FP32 and bf16x3
forms agree on the spatial ranks, and the factored core equals V x_d S.
"""

import math

import pytest

pytestmark = pytest.mark.gpu

N_INIT, N_UPD, TAU = 20, 10, 1e-4


def _stream():
    from synth import make_stream

    return make_stream(4)


def _true_error(st, s, ts):
    import torch

    err2 = nrm2 = 0.0
    for t in ts:
        y = s.slice_torch(t, torch.device("cuda:0"), torch.float32).double()
        r = st.reconstruct_slice(t).double()
        err2 += torch.sum((r - y) ** 2).item()
        nrm2 += torch.sum(y ** 2).item()
    return math.sqrt(err2 / nrm2)


def _run(precision, core_update):
    import torch

    import paper_2308_16395_amd as pkg

    s = _stream()
    dev = torch.device("cuda:0")
    x0 = torch.cat([s.slice_torch(t, dev, torch.float32) for t in range(N_INIT)])
    st = pkg.StreamingTucker(s.dims, TAU, precision=precision, core_update=core_update)
    st.init(x0, N_INIT)
    del x0
    assert st.recon_error()[0] <= TAU
    for t in range(N_INIT, N_INIT + N_UPD):
        st.update(s.slice_torch(t, dev, torch.float32))
    return st, s


@pytest.mark.parametrize("precision,core_update",
                         [("fp32", "factored"), ("bf16x3", "factored"), ("fp32", "literal")])
def test_fourier_512_stream_meets_tau(precision, core_update):
    import torch

    st, s = _run(precision, core_update)
    bound, _ = st.recon_error()
    assert bound <= TAU
    ts = [0, 7, N_INIT - 1, N_INIT, N_INIT + N_UPD - 1]
    assert _true_error(st, s, ts) <= TAU
    ranks = st.ranks
    assert all(60 <= r <= n for r, n in zip(ranks[:3], s.dims))
    for k in range(3):
        u = st.factor(k)
        g = u.T @ u
        assert torch.max(torch.abs(g - torch.eye(g.shape[0], device=g.device, dtype=g.dtype))) < 1e-6
    sv = st.sv()
    assert all(x > 0 for x in sv) and all(a >= b for a, b in zip(sv, sv[1:]))
    if core_update == "factored":
        # V from the Gram-based initial SVD (Alg. 1) is orthonormal to about
        # u (s_1 / s_r)^2: the tail rule may keep a last singular value far
        # below eps, as it does on this stream
        v = st.aux_v()
        gv = v.T @ v
        tol = max(1e-6, 64 * 2.0 ** -52 * (sv[0] / sv[-1]) ** 2)
        assert torch.max(torch.abs(gv - torch.eye(gv.shape[0], device=gv.device,
                                                  dtype=gv.dtype))).item() < tol
        # C = V x_d S: column j of the mode-d unfolding transposed is S_j V(:, j)
        core = st.core().double()
        svt = torch.tensor(sv, device=v.device, dtype=v.dtype)
        ref = (v * svt[None, :]).T.contiguous().reshape(-1)
        assert torch.max(torch.abs(core - ref)).item() <= 1e-5 * torch.max(torch.abs(ref)).item()
    st.close()
