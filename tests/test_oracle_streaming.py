"""Pins for Alg. 4 / Alg. 5 (the streaming update) on small inputs.

The harness keeps every slice, so the true error of the streamed
decomposition is measured directly and checked against the guarantee of
Alg. 5 (App. D) after every slice, together with Assumption 1, the Alg. 4
post-conditions, the exact error split of Prop. 3, exact recovery of exactly
low-rank streams and the batch ST-HOSVD at the same ranks.
"""

import math

import numpy as np
import pytest

from oracle import (StreamingTucker, multi_ttm, non_streaming_update,
                    reconstruct, sthosvd, ttm, unfold, vec)
from synth import BlobStream, LowRankStream


def _lowrank_stream(shape, ranks, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    core = rng.standard_normal(ranks)
    mats = [np.linalg.qr(rng.standard_normal((n, r)))[0] for n, r in zip(shape, ranks)]
    x = multi_ttm(core, mats)
    if noise:
        x = x + noise * np.linalg.norm(x) / math.sqrt(x.size) * rng.standard_normal(shape)
    return x


def _check_assumption1(st, tol=1e-12):
    for u in st.U:
        np.testing.assert_allclose(u.T @ u, np.eye(u.shape[1]), atol=tol)
    v = st.vmat()
    np.testing.assert_allclose(v.T @ v, np.eye(v.shape[1]), atol=tol)
    assert np.all(st.S > 0) and np.all(np.diff(st.S) <= 0)
    assert st.C.shape == tuple(u.shape[1] for u in st.U)


CASES = [
    # (name, full tensor builder, n_init, tau)
    ("lowrank3_noisy", lambda: LowRankStream((12, 10), 40, (3, 2, 4), 1e-3, seed=3).full, 6, 1e-2),
    ("lowrank4_noisy", lambda: _lowrank_stream((6, 5, 4, 30), (2, 3, 2, 4), 4, 1e-2), 3, 5e-2),
    ("blobs_small", lambda: np.stack([BlobStream((10, 9, 8), 3, 4, (1.5, 3.0), 0.5,
                                                 n_slices=25, seed=5).slice(t)
                                      for t in range(25)], axis=-1), 4, 1e-2),
    ("matrix_d2", lambda: _lowrank_stream((15, 40), (5, 5), 6, 1e-2), 5, 5e-2),
]


@pytest.mark.parametrize("name,build,n_init,tau", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_guarantee_after_every_slice(name, build, n_init, tau, core_update):
    x = build()
    d = x.ndim
    st = StreamingTucker(x[..., :n_init], tau, core_update=core_update)
    _check_assumption1(st)
    n = x.shape[-1]
    for t in range(n_init, n):
        st.update(x[..., t])
        seen = x[..., :t + 1]
        xhat = st.reconstruct()
        err = np.linalg.norm(seen - xhat)
        nrm = np.linalg.norm(seen)
        assert err <= tau * nrm * (1 + 1e-10), (t, err / nrm)
        # the accumulated bound is certified and within tau
        assert err <= st.recon_error_bound() * nrm * (1 + 1e-9) + 1e-13
        assert st.recon_error_bound() <= tau * (1 + 1e-12)
        _check_assumption1(st)
        assert st.U[-1].shape[0] == t + 1
        np.testing.assert_allclose(st.xnorm2, nrm ** 2, rtol=1e-12)
        if core_update == "factored":
            np.testing.assert_allclose(st.C, ttm(st.V, np.diag(st.S), d - 1),
                                       atol=1e-12 * nrm)


@pytest.mark.parametrize("grow", [True, False])
def test_literal_core_vs_factored_core(grow):
    """Last step of Alg. 5 against the Ensure clause C~ = V~ x_d S~.

    When the ISVD keeps e (q > eps) the two cores coincide; when e is ignored
    the literal core is the projection of the data onto U~_d, so its model of
    the augmented tensor is never worse than V~ x_d S~.
    """
    x = _lowrank_stream((6, 5, 20), (2, 3, 3), 7, 1e-2)
    st = StreamingTucker(x[..., :6], 5e-2)
    np.testing.assert_allclose(st.C, ttm(st.V, np.diag(st.S), 2), atol=1e-12)
    rng = np.random.default_rng(8)
    y = x[..., 6] + (0.2 * rng.standard_normal(x.shape[:-1]) if grow else 0.0)
    y = multi_ttm(y, [u @ u.T for u in st.U[:-1]]) if not grow else y
    rec = st.update(y)
    assert rec["ignored"] == (not grow)
    factored = ttm(st.V, np.diag(st.S), 2)
    seen = np.concatenate([x[..., :6], y[..., None]], axis=-1)
    if grow:
        np.testing.assert_allclose(st.C, factored, atol=1e-12 * np.linalg.norm(seen))
    else:
        err_lit = np.linalg.norm(seen - reconstruct(st.C, st.U))
        err_fac = np.linalg.norm(seen - reconstruct(factored, st.U))
        assert err_lit <= err_fac * (1 + 1e-12)


def _one_nonstreaming_step(seed, grow):
    rng = np.random.default_rng(seed)
    x = _lowrank_stream((7, 6, 5, 12), (2, 2, 2, 3), seed, 1e-3)
    st = StreamingTucker(x[..., :5], 1e-2)
    y = x[..., 5] + (0.3 if grow else 0.0) * rng.standard_normal(x.shape[:-1])
    return st, y


@pytest.mark.parametrize("grow", [False, True])
def test_alg4_postconditions_and_prop3(grow):
    st, y = _one_nonstreaming_step(11, grow)
    d = st.d
    ynorm = np.linalg.norm(y)
    eps = st.tau * ynorm / math.sqrt(d)
    c, dk, v = st.C, y, st.V
    u_list = list(st.U)
    deltas = []
    grew_any = False
    x_old_model = reconstruct(st.C, st.U)
    for k in range(d - 1):
        u_new, c_new, d_new, v_new, info = non_streaming_update(k, u_list[k], c, dk, v, eps)
        grew_any |= info["grew"]
        # C_k x_k U~_k = C_{k-1} x_k U_k (exact)
        np.testing.assert_allclose(ttm(c_new, u_new, k), ttm(c, u_list[k], k), atol=1e-12)
        # ||D*_{k-1} - D*_k x_k U~_k|| <= eps, and equals the reported delta
        resid2 = np.sum((dk - ttm(d_new, u_new, k)) ** 2)
        assert math.sqrt(resid2) <= eps * (1 + 1e-10)
        # (the Gram route resolves eigenvalues to about u ||E||^2, Sec. 2.3)
        np.testing.assert_allclose(resid2, info["delta2"], rtol=1e-8, atol=1e-13 * ynorm ** 2)
        deltas.append(info["delta2"])
        # V padding keeps the mode-d matricization row-orthonormal
        vm = unfold(v_new, d - 1)
        np.testing.assert_allclose(vm @ vm.T, np.eye(vm.shape[0]), atol=1e-12)
        u_list[k] = u_new
        c, dk, v = c_new, d_new, v_new
    assert grew_any == grow
    # Prop. 3: the model of the old data is unchanged ...
    np.testing.assert_allclose(reconstruct(c, u_list), x_old_model, atol=1e-12)
    # ... and the new-slice error is the exact sum of the per-mode errors
    yhat = multi_ttm(dk, u_list[:-1])
    np.testing.assert_allclose(np.sum((y - yhat) ** 2), sum(deltas), rtol=1e-8,
                               atol=1e-13 * ynorm ** 2)


def test_exact_low_rank_stream_no_growth_and_exact_recovery():
    x = LowRankStream((32, 32), 100, (4, 4, 6), noise_rel=0.0, seed=1000).full
    st = StreamingTucker(x[..., :10], 1e-3)
    assert st.ranks == (4, 4, 6)
    for t in range(10, 100):
        rec = st.update(x[..., t])
        assert not any(rec["grew"]) and rec["ignored"]
    assert st.ranks == (4, 4, 6)
    assert np.linalg.norm(x - st.reconstruct()) <= 1e-12 * np.linalg.norm(x)


def test_low_rank_stream_small_init_ranks_stay_below_true_ranks():
    x = _lowrank_stream((9, 8, 7, 40), (3, 3, 2, 6), 13, 0.0)
    st = StreamingTucker(x[..., :2], 1e-4)
    for t in range(2, 40):
        st.update(x[..., t])
        assert all(r <= rt for r, rt in zip(st.ranks[:-1], (3, 3, 2)))
    assert st.ranks[:-1] == (3, 3, 2)
    assert np.linalg.norm(x - st.reconstruct()) <= 1e-10 * np.linalg.norm(x)


def test_matches_batch_sthosvd_at_the_same_ranks():
    x = _lowrank_stream((8, 7, 6, 30), (3, 2, 3, 4), 17, 0.0)
    st = StreamingTucker(x[..., :8], 1e-6)
    for t in range(8, 30):
        st.update(x[..., t])
    batch = sthosvd(x, 0.0, ranks=st.ranks)
    for u_s, u_b in zip(st.U, batch["factors"]):
        np.testing.assert_allclose(u_s @ u_s.T, u_b @ u_b.T, atol=1e-10)
    np.testing.assert_allclose(st.reconstruct(), reconstruct(batch["core"], batch["factors"]),
                               atol=1e-10 * np.linalg.norm(x))


def test_noisy_stream_and_batch_both_meet_tau():
    x = _lowrank_stream((8, 7, 6, 30), (3, 2, 3, 4), 19, 5e-3)
    tau = 2e-2
    st = StreamingTucker(x[..., :6], tau)
    for t in range(6, 30):
        st.update(x[..., t])
    batch = sthosvd(x, tau)
    nrm = np.linalg.norm(x)
    assert np.linalg.norm(x - st.reconstruct()) <= tau * nrm
    assert np.linalg.norm(x - reconstruct(batch["core"], batch["factors"])) <= tau * nrm


def test_zero_slice_changes_no_rank():
    x = _lowrank_stream((6, 5, 12), (2, 2, 3), 21, 1e-3)
    st = StreamingTucker(x[..., :6], 1e-2)
    ranks, bound, xn = st.ranks, st.recon_error_bound(), st.xnorm2
    rec = st.update(np.zeros(x.shape[:-1]))
    assert st.ranks == ranks and rec["ignored"] and not any(rec["grew"])
    assert st.xnorm2 == xn and st.recon_error_bound() == bound
    assert st.U[-1].shape[0] == 7
    np.testing.assert_allclose(st.reconstruct_slice(6), 0.0, atol=1e-14)


def test_invalid_inputs_raise():
    x = _lowrank_stream((6, 5, 8), (2, 2, 3), 23, 1e-3)
    with pytest.raises(ValueError):
        StreamingTucker(np.zeros_like(x), 1e-2)
    st = StreamingTucker(x[..., :4], 1e-2)
    bad = x[..., 4].copy()
    bad[0, 0] = np.nan
    with pytest.raises(ValueError):
        st.update(bad)
    with pytest.raises(ValueError):
        st.update(np.zeros((5, 6)))
    assert st.U[-1].shape[0] == 4


def _threshold_case(level, alpha=0.1, n=8, tau=0.1):
    """Old data: two rank-one slices of norm alpha (ranks (2, 2, 2), no
    truncation). New slice: a part inside the old span plus three orthogonal
    parts of norm level * tau * ||Y|| each, one outside the mode-1 span, one
    outside the mode-2 span, and one inside both spans but outside the span of
    the streaming-mode auxiliary matrix V (core coordinate (1, 2))."""
    q_, _ = np.linalg.qr(np.random.default_rng(31).standard_normal((n, 3)))
    a1, a2, a3 = q_.T
    q_, _ = np.linalg.qr(np.random.default_rng(32).standard_normal((n, 3)))
    b1, b2, b3 = q_.T
    x0 = np.stack([alpha * np.outer(a1, b1), alpha * np.outer(a2, b2)], axis=-1)
    g = level * tau
    mu = math.sqrt(1.0 - 3.0 * g * g)  # ||Y|| = 1
    y = (mu * np.outer(a1, b1) + g * np.outer(a1, b2) + g * np.outer(a3, b1)
         + g * np.outer(a1, b3))
    return x0, y, tau


@pytest.mark.parametrize("level", [0.60, 0.80])
def test_alg5_tolerance_splits_the_slice_budget_over_d(level):
    """Alg. 5 gives every one of the d steps of a slice the tolerance
    eps = tau ||Y|| / sqrt(d), so the d squared errors sum to at most
    tau^2 ||Y||^2 (App. D). Residuals of level * tau ||Y|| with
    1/sqrt(3) < level must therefore grow both slice modes and the streaming
    rank, and the guarantee ||X - X^|| <= tau ||X|| holds after the slice. A
    tolerance of tau ||Y|| (or tau ||Y|| / sqrt(d - 1) at level 0.6) would keep
    all three parts and break the guarantee: the three squared residuals add
    up to 3 level^2 tau^2 ||Y||^2 > tau^2 (||Y||^2 + ||X_old||^2)."""
    x0, y, tau = _threshold_case(level)
    st = StreamingTucker(x0, tau)
    assert st.ranks == (2, 2, 2) and st.disc < 1e-14
    rec = st.update(y)
    assert rec["grew"] == [True, True]
    assert not rec["ignored"]
    assert st.ranks == (3, 3, 3)
    x = np.concatenate([x0, y[..., None]], axis=-1)
    err = np.linalg.norm(x - st.reconstruct())
    assert err <= tau * np.linalg.norm(x)
    # the three parts lie inside the grown spans: nothing is lost
    assert err <= 1e-12


@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_alg5_tolerance_keeps_residuals_below_tau_over_sqrt_d(core_update):
    """The converse side of the same tolerance: residuals of 0.55 tau ||Y||
    (below tau ||Y|| / sqrt(3) = 0.577 tau ||Y||) grow nothing, and the slice
    adds the three squared residuals to the error bound (Prop. 3 for the slice
    modes, Prop. 1 for the ignored ISVD residual). With the core kept as
    C = V x_d S the error equals that bound (Prop. 1 is an equality); the
    literal core update of Alg. 5 keeps part of the ignored residual, so its
    error is at most the bound. A smaller tolerance such as tau ||Y|| / d would
    grow all three."""
    x0, y, tau = _threshold_case(0.55)
    st = StreamingTucker(x0, tau, core_update=core_update)
    rec = st.update(y)
    assert rec["grew"] == [False, False] and rec["ignored"]
    assert st.ranks == (2, 2, 2)
    x = np.concatenate([x0, y[..., None]], axis=-1)
    err = np.linalg.norm(x - st.reconstruct())
    bound = st.recon_error_bound() * math.sqrt(st.xnorm2)
    assert bound == pytest.approx(math.sqrt(3.0) * 0.55 * tau, rel=1e-9)
    if core_update == "factored":
        assert err == pytest.approx(bound, rel=1e-9)
    else:
        # the two slice-mode residuals are lost in any case
        assert math.sqrt(2.0) * 0.55 * tau * (1 - 1e-9) <= err <= bound * (1 + 1e-12)
    assert err <= tau * np.linalg.norm(x)


@pytest.mark.parametrize("core_update", ["literal", "factored"])
def test_reconstruct_slice_is_a_slice_of_the_reconstruction(core_update):
    """reconstruct_slice(t) is slice t of C x_1 U_1 ... x_d U_d (Sec. 2.2) for
    every t, initial and streamed slices alike."""
    x = _lowrank_stream((7, 6, 5, 18), (3, 2, 2, 5), 41, 1e-2)
    st = StreamingTucker(x[..., :4], 5e-2, core_update=core_update)
    for t in range(4, x.shape[-1]):
        st.update(x[..., t])
    full = st.reconstruct()
    assert full.shape == x.shape
    for t in range(x.shape[-1]):
        np.testing.assert_allclose(st.reconstruct_slice(t), full[..., t], rtol=0, atol=1e-13)
    # and the slices differ from each other (a reversed or shifted row of U_d
    # would be caught)
    assert np.linalg.norm(full[..., 0] - full[..., -1]) > 1e-3
