"""Pins of the oracle's block update (several slices per update; the paper's
Sec. 6 future work, built as the block form of Alg. 5 with Alg. 3 generalised
to a residual block whose directions are chosen by the TruncatedSVD of Alg. 1).

What fixes it, independently of its own code:
  * b = 1 is the single-slice update: identical eps, decisions, singular
    values and reconstructions (the block form reduces to Alg. 3 / Alg. 5);
  * the guarantee of App. D carried to blocks: after a stream cut into blocks
    the true relative error is at most the certified bound, which is <= tau;
  * exact data: an exactly low-rank stream is reproduced to rounding with its
    exact ranks;
  * matrices (d = 2) without truncation: the singular values after block
    updates are those of the whole matrix (numpy.linalg.svd).
"""

import numpy as np
import pytest

from oracle import StreamingTucker, block_isvd, vec
from synth import BlobStream, LowRankStream


def _slices32(s, n):
    return [s.slice_flat(t).astype(np.float32).astype(np.float64).reshape(s.dims, order="F")
            for t in range(n)]


def test_block_of_one_is_the_single_slice_update():
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    sl = _slices32(s, 36)
    x0 = np.stack(sl[:6], axis=-1)
    a, b = StreamingTucker(x0, 1e-3), StreamingTucker(x0, 1e-3)
    grew = 0
    for t in range(6, 36):
        ra = a.update(sl[t])
        rb = b.update_block(sl[t][..., None])
        assert rb["eps"] == ra["eps"]
        assert a.ranks == b.ranks
        assert rb["ell"] == (0 if ra["ignored"] else 1)
        grew += rb["ell"]
    assert grew > 5
    np.testing.assert_allclose(b.S, a.S, rtol=1e-13)
    assert b.recon_error_bound() == pytest.approx(a.recon_error_bound(), rel=1e-13)
    for t in (0, 17, 35):
        np.testing.assert_allclose(vec(b.reconstruct_slice(t)), vec(a.reconstruct_slice(t)),
                                   atol=1e-12 * np.linalg.norm(sl[t]))


@pytest.mark.parametrize("bsize,core_update", [(3, "literal"), (4, "literal"), (5, "factored")])
def test_block_stream_meets_its_bound(bsize, core_update):
    s = BlobStream((24, 20, 16), 3, 6, (2.0, 5.0), 0.7, n_slices=36, seed=21)
    sl = _slices32(s, 36)
    tau = 1e-3
    orc = StreamingTucker(np.stack(sl[:6], axis=-1), tau, core_update=core_update)
    t = 6
    while t < 36:
        bb = min(bsize, 36 - t)
        rec = orc.update_block(np.stack(sl[t:t + bb], axis=-1))
        d = len(s.dims) + 1
        assert rec["eps"] == pytest.approx(tau * rec["ynorm"] / np.sqrt(d), rel=1e-15)
        t += bb
    assert orc.n_slices == 36
    x = np.stack(sl, axis=-1)
    err = np.linalg.norm(orc.reconstruct() - x) / np.linalg.norm(x)
    bound = orc.recon_error_bound()
    assert err <= bound * (1 + 1e-9) and bound <= tau
    # the kept residual directions of each block never exceed its size
    assert all(0 <= h["ell"] <= h["b"] for h in orc.history)


def test_exact_low_rank_stream_in_blocks():
    s = LowRankStream((30, 26), 48, (4, 3, 5), noise_rel=0.0, seed=77)
    sl = [s.slice(t) for t in range(48)]
    # tau well above the rounding of the Gram-based SVD (about u ||X||^2)
    orc = StreamingTucker(np.stack(sl[:8], axis=-1), 1e-6)
    for t0 in range(8, 48, 4):
        orc.update_block(np.stack(sl[t0:t0 + 4], axis=-1))
    assert orc.ranks == (4, 3, 5)
    x = np.stack(sl, axis=-1)
    assert np.linalg.norm(orc.reconstruct() - x) <= 1e-11 * np.linalg.norm(x)


def test_matrix_block_updates_equal_the_full_svd():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((40, 7)) @ rng.standard_normal((7, 60))  # rank 7, 40 x 60
    # d = 2: slices are the 40-vectors a[:, t]; the streaming factor has 60 rows
    orc = StreamingTucker(a[:, :10], 1e-6)
    for t0 in range(10, 60, 5):
        orc.update_block(a[:, t0:t0 + 5])
    s_ref = np.linalg.svd(a, compute_uv=False)[:7]
    assert orc.ranks == (7, 7)
    np.testing.assert_allclose(orc.S, s_ref, rtol=1e-10)
    np.testing.assert_allclose(orc.reconstruct(), a, atol=1e-10 * np.linalg.norm(a))


def test_block_isvd_middle_matrix_reproduces_the_rows():
    """[V Q] S' and U'' reproduce the old rows and the new block up to the
    discarded tail (the defining property of the block middle matrix)."""
    rng = np.random.default_rng(11)
    R, r, n, b = 50, 4, 12, 3
    v, _ = np.linalg.qr(rng.standard_normal((R, r)))
    u, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = np.array([9.0, 5.0, 2.0, 1.0])
    bmat = v @ rng.standard_normal((r, b)) + 1e-3 * rng.standard_normal((R, b))
    u_new, s_new, v_new, info = block_isvd(u, s, v, bmat, eps=1e-12)
    assert info["ell"] == b and u_new.shape == (n + b, r + b)
    a_old = u @ np.diag(s) @ v.T
    full = np.vstack([a_old, bmat.T])
    np.testing.assert_allclose(u_new @ np.diag(s_new) @ v_new.T, full, atol=1e-12)
    np.testing.assert_allclose(v_new.T @ v_new, np.eye(r + b), atol=1e-12)
    np.testing.assert_allclose(u_new.T @ u_new, np.eye(r + b), atol=1e-12)


def _block_threshold_case(level, alpha=0.1, n=8, tau=0.1):
    """Old data: two rank-one slices of norm alpha (ranks (2, 2, 2)). New block
    of two slices, ||Y_B|| = 1, holding three orthogonal parts of norm
    level * tau: one outside the mode-1 span (slice 1), one outside the mode-2
    span and one inside both spans but outside the span of the streaming-mode
    auxiliary matrix V (core coordinate (1, 2); slice 2)."""
    q_, _ = np.linalg.qr(np.random.default_rng(31).standard_normal((n, 3)))
    a1, a2, a3 = q_.T
    q_, _ = np.linalg.qr(np.random.default_rng(32).standard_normal((n, 3)))
    b1, b2, b3 = q_.T
    x0 = np.stack([alpha * np.outer(a1, b1), alpha * np.outer(a2, b2)], axis=-1)
    g = level * tau
    m = np.sqrt((1.0 - 3.0 * g * g) / 2.0)
    y1 = m * np.outer(a1, b1) + g * np.outer(a3, b1)
    y2 = m * np.outer(a1, b1) + g * np.outer(a1, b3) + g * np.outer(a1, b2)
    return x0, np.stack([y1, y2], axis=-1), tau


@pytest.mark.parametrize("level", [0.60, 0.80])
def test_block_tolerance_grows_residuals_above_tau_over_sqrt_d(level):
    """eps_B = tau ||Y_B|| / sqrt(d) (d = 3): residual parts of level * tau
    ||Y_B|| with level > 1/sqrt(3) grow both slice modes and the streaming rank,
    and nothing is lost: once the slice modes hold the two outer parts, they
    join the third as residual directions of the streaming mode (E^T E has
    eigenvalues 2 g^2 and g^2, g = level tau, both above eps_B^2), so both are
    kept. A tolerance of tau ||Y_B|| keeps the slice modes and loses
    3 level^2 tau^2."""
    x0, yb, tau = _block_threshold_case(level)
    st = StreamingTucker(x0, tau)
    rec = st.update_block(yb)
    g = level * tau
    assert rec["grew"] == [True, True] and rec["ell"] == 2
    np.testing.assert_allclose(rec["lam"][:2], [2 * g * g, g * g], rtol=1e-12)
    assert st.ranks == (3, 3, 4)
    x = np.concatenate([x0, yb], axis=-1)
    assert np.linalg.norm(x - st.reconstruct()) <= 1e-12


@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_block_tolerance_keeps_residuals_below_tau_over_sqrt_d(core_update):
    """The converse: parts of 0.55 tau ||Y_B|| (below tau ||Y_B|| / sqrt(3))
    grow nothing and the bound adds the three squared parts. A smaller block
    tolerance (tau ||Y_B|| / sqrt(d b), or one from a single slice's norm
    ||Y_B|| / sqrt(2) here) would grow all three."""
    x0, yb, tau = _block_threshold_case(0.55)
    st = StreamingTucker(x0, tau, core_update=core_update)
    rec = st.update_block(yb)
    assert rec["grew"] == [False, False] and rec["ell"] == 0
    assert st.ranks == (2, 2, 2)
    bound = st.recon_error_bound() * np.sqrt(st.xnorm2)
    assert bound == pytest.approx(np.sqrt(3.0) * 0.55 * tau, rel=1e-9)
    x = np.concatenate([x0, yb], axis=-1)
    assert np.linalg.norm(x - st.reconstruct()) <= bound * (1 + 1e-12)
