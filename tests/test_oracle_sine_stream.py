"""Pins for the oracle on the sine-wave stream of Sec. 5.1 (Fig. 3, Table 1).

The noise-free stream has closed-form ranks: 2 f_k + 1 in the spatial modes,
2 f_a + 1 in the streaming mode over the first block and 2 f_b + 1 over the
whole stream. With eta = 1e-3 far below tau = 1e-2 the batch ST-HOSVD (Alg. 2)
must return exactly those ranks. The streaming update (Alg. 5) keeps the
spatial ranks, grows the streaming rank at the first slice of the second
block (the bump the paper reports) and never ends below the batch rank, with
the true error below the certified bound of App. D and that bound below tau.
Reduced size (40 x 40 spatial grid, 2 x 500 slices); the GPU test streams
the paper's 100 x 100 x 5000.
"""

import numpy as np

from oracle import StreamingTucker, sthosvd
from synth import SINE_WAVE, SineWaveStream

TAU = SINE_WAVE["eps"]


def _stream():
    return SineWaveStream(dims=(40, 40), n_half=500, freqs=SINE_WAVE["freqs"],
                          f_a=SINE_WAVE["f_a"], f_b=SINE_WAVE["f_b"], eta=SINE_WAVE["eta"],
                          seed=SINE_WAVE["seed"])


def _tensor(s):
    return np.stack([s.slice(t) for t in range(s.n_slices)], axis=-1)


def test_generator_noise_ratio_and_exact_ranks():
    s = _stream()
    clean = np.stack([s._clean(t) for t in range(s.n_slices)], axis=1)
    noisy = np.stack([s.slice_flat(t) for t in range(s.n_slices)], axis=1)
    np.testing.assert_allclose(np.linalg.norm(noisy - clean), s.eta * np.linalg.norm(clean),
                               rtol=1e-12)
    (r1, r2), ra, rb = s.expected_ranks()
    sv_a = np.linalg.svd(clean[:, :s.n_half], compute_uv=False)
    sv_all = np.linalg.svd(clean, compute_uv=False)
    assert int(np.sum(sv_a > 1e-10 * sv_a[0])) == ra == 11
    assert int(np.sum(sv_all > 1e-10 * sv_all[0])) == rb == 15
    assert (r1, r2) == (11, 11)


def test_batch_sthosvd_closed_form_ranks():
    s = _stream()
    x = _tensor(s)
    (r1, r2), ra, rb = s.expected_ranks()
    assert sthosvd(x, TAU)["core"].shape == (r1, r2, rb)
    assert sthosvd(x[..., :s.n_half], TAU)["core"].shape == (r1, r2, ra)


def test_streaming_detects_rank_bump_within_bound():
    s = _stream()
    x = _tensor(s)
    n_init = 80
    st = StreamingTucker(x[..., :n_init], TAU)
    r3 = {}
    for t in range(n_init, s.n_slices):
        st.update(x[..., t])
        assert st.ranks[:2] == (11, 11), (t, st.ranks)
        r3[t] = st.ranks[2]
    # the streaming rank grows on the first slice of the second block
    assert r3[s.n_half] > r3[s.n_half - 1]
    (_, _), _, rb = s.expected_ranks()
    assert st.ranks[2] >= rb
    true_err = np.linalg.norm(x - st.reconstruct()) / np.linalg.norm(x)
    assert true_err <= st.recon_error_bound() <= TAU, (true_err, st.recon_error_bound())
