"""Plain FP64 streaming ST-HOSVD, step by step (test infrastructure only).

What this file is: the oracle. It follows the paper's algorithms in their
order and notation, in float64 NumPy, with no blocking or fusion. Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may use it.

Conventions (paper Sec. 2.1): tensors are NumPy arrays indexed (i_1, ..., i_d);
the mode-k matricization puts mode k on the rows and orders the columns with
the first remaining index fastest (column-major). ``vec`` is the column-major
vectorisation, the same order as the columns of a mode-d matricization.

Readings taken where the paper is silent or self-contradictory (each is a
named argument with the default used everywhere):

* Alg. 1 writes S = diag(lambda(1:r)); the core factorization of Sec. 3.2 needs
  singular values, so S = diag(sqrt(lambda_1..r)) and V = A^T U S^{-1}.
* Eigenvalues are sorted descending, negative round-off eigenvalues are
  clamped to 0, and the rank rule keeps the smallest r whose tail sum is
  <= eps^2 (equality truncates).
* One eps = tau ||Y|| / sqrt(d) per slice is used by every NonStreamingUpdate
  and by the ISVD (Alg. 5, App. D).
* ``<=`` in the branch tests of Alg. 3 and Alg. 4 means "keep": a zero slice
  changes no rank.
* ISVD: the complement e is computed with two Gram-Schmidt passes (``cgs2``),
  and the orthogonality check of Alg. 3 is applied to every column of V, with
  ``eps_m`` = 1e-12.
* TruncatedSVD(S', 0) in Alg. 3 is an exact compact SVD: S' has full column
  rank (S > 0, and q > eps >= 0 when the new direction is kept), so the
  streaming rank grows by one exactly when q > eps.
* New columns W_k of Alg. 4 are re-orthogonalised against U_k (two passes,
  then a QR of W_k) so that the factors stay orthonormal to about 1e-15.
* The core update is the literal last step of Alg. 5 (``core_update =
  "literal"``); ``"factored"`` keeps C = V x_d S instead (the Ensure clause).
"""

from __future__ import annotations

import math

import numpy as np


# ----------------------------------------------------------------------------
# Sec. 2.1: matricization, TTM, multi-TTM
# ----------------------------------------------------------------------------

def unfold(x, k):
    """Mode-k matricization X_(k) (Sec. 2.1): n_k x prod_{l != k} n_l,
    columns ordered with the first remaining index fastest."""
    x = np.asarray(x)
    return np.reshape(np.moveaxis(x, k, 0), (x.shape[k], -1), order="F")


def fold(m, k, shape):
    """Inverse of ``unfold`` for a tensor of the given shape."""
    shape = tuple(shape)
    rest = shape[:k] + shape[k + 1:]
    t = np.reshape(m, (shape[k],) + rest, order="F")
    return np.moveaxis(t, 0, k)


def vec(x):
    """Column-major vectorisation (first index fastest)."""
    return np.reshape(np.asarray(x), (-1,), order="F")


def ttm(x, a, k):
    """Y = X x_k A, defined by Y_(k) = A X_(k) (Sec. 2.1)."""
    a = np.asarray(a, dtype=np.float64)
    shape = list(np.shape(x))
    shape[k] = a.shape[0]
    return fold(a @ unfold(x, k), k, shape)


def multi_ttm(x, mats, transpose=False, skip=None):
    """X x_1 A_1 ... x_d A_d (A_k^T if ``transpose``), skipping mode ``skip``."""
    y = x
    for k, a in enumerate(mats):
        if k == skip or a is None:
            continue
        y = ttm(y, a.T if transpose else a, k)
    return y


def reconstruct(core, factors):
    """Tucker reconstruction C x_1 U_1 ... x_d U_d (Sec. 2.2, eq. tucker_def)."""
    return multi_ttm(core, factors)


# ----------------------------------------------------------------------------
# Alg. 1: truncated Gram SVD
# ----------------------------------------------------------------------------

def tsvd_gram(a, eps, rank=None, max_rank=None):
    """TruncatedSVD(A, eps) of Alg. 1.

    Returns ``(r, U, s, tail_r, lam)``: the rank r, the leading r eigenvectors
    U of the Gram A A^T, s = sqrt(lambda_1..r), the discarded tail
    lambda_{r+1} + ... + lambda_m, and all eigenvalues (descending).
    ``rank`` fixes r instead of applying the tolerance (batch comparison at
    given ranks); ``max_rank`` caps r.
    """
    a = np.asarray(a, dtype=np.float64)
    g = a @ a.T
    lam, p = np.linalg.eigh(g)
    order = np.argsort(lam)[::-1]
    lam = np.maximum(lam[order], 0.0)
    p = p[:, order]
    m = lam.shape[0]
    # tail[l] = lambda_{l+1} + ... + lambda_m, summed from the smallest upward
    tail = np.zeros(m + 1)
    tail[:m] = np.cumsum(lam[::-1])[::-1]
    if rank is None:
        r = int(np.argmax(tail <= eps * eps))  # tail[m] = 0 always qualifies
    else:
        r = int(rank)
    if max_rank is not None:
        r = min(r, int(max_rank))
    return r, p[:, :r], np.sqrt(lam[:r]), float(tail[r]), lam


# ----------------------------------------------------------------------------
# Alg. 2: ST-HOSVD
# ----------------------------------------------------------------------------

def sthosvd(x, tau, ranks=None):
    """ST-HOSVD(X, tau) of Alg. 2, modes processed in the order 1..d.

    Returns a dict with the core, the factors, the per-mode discarded tails
    (whose sum is the squared error, Sec. 2.3), eps, and for the last mode
    the singular values ``s_last`` and the Gram-SVD right factor
    ``v_last`` = A^T U_d S^{-1} with A = C*_{d-1,(d)} (Alg. 1, optional rows).
    ``ranks`` fixes the ranks instead of the tolerance.
    """
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    eps = tau * np.linalg.norm(x) / math.sqrt(d)
    c = x
    factors, tails = [], []
    s_last = v_last = None
    for k in range(d):
        a = unfold(c, k)
        r, u, s, t, _ = tsvd_gram(a, eps, rank=None if ranks is None else ranks[k])
        if k == d - 1:
            s_last = s
            v_last = (a.T @ u) / s[None, :] if r > 0 else np.zeros((a.shape[1], 0))
        c = ttm(c, u.T, k)
        factors.append(u)
        tails.append(t)
    return dict(core=c, factors=factors, tails=tails, eps=eps,
                s_last=s_last, v_last=v_last)


# ----------------------------------------------------------------------------
# Alg. 3: incremental SVD
# ----------------------------------------------------------------------------

def isvd(u, s, v, b, eps, eps_m=1e-12, cgs2=True):
    """IncrementalSVD(U, S, V, b, eps) of Alg. 3 for a new row b.

    U is m x r, S holds the r singular values, V is n x r. Returns
    ``(U~, S~, V~, info)``; info has p, q, ``ignored`` (q <= eps), ``qr``
    (whether the orthogonality check fired) and U'', V''.
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = s.shape[0]
    p = v.T @ b
    e = b - v @ p
    # diagnostic only: Alg. 3's orthogonality measure taken on the single-pass
    # complement, max_j |V(:,j)^T e| / ||e|| (no effect on the result)
    e1n = float(np.linalg.norm(e))
    single = float(np.max(np.abs(v.T @ e)) / e1n) if r > 0 and e1n > 0 else 0.0
    if cgs2:
        p2 = v.T @ e
        e = e - v @ p2
        p = p + p2
    q = float(np.linalg.norm(e))
    fired = False
    orth = 0.0
    if q <= eps:
        s_prime = np.vstack([np.diag(s), p[None, :]])
        v_prime = v
    else:
        vnew = e / q
        s_prime = np.zeros((r + 1, r + 1))
        s_prime[:r, :r] = np.diag(s)
        s_prime[r, :r] = p
        s_prime[r, r] = q
        v_prime = np.hstack([v, vnew[:, None]])
        orth = float(np.max(np.abs(v.T @ vnew))) if r > 0 else 0.0
        if r > 0 and orth > eps_m:
            fired = True
            qm, rm = np.linalg.qr(v_prime)
            v_prime = qm
            s_prime = s_prime @ rm.T
    # exact compact SVD of the small middle matrix
    u2, s_new, v2t = np.linalg.svd(s_prime, full_matrices=False)
    v2 = v2t.T
    u_new = np.vstack([u @ u2[:r, :], u2[r:r + 1, :]])
    v_new = v_prime @ v2
    info = dict(p=p, q=q, ignored=q <= eps, qr=fired, u2=u2, v2=v2, orth_single_pass=single,
                orth_check=orth)
    return u_new, s_new, v_new, info


def block_isvd(u, s, v, bmat, eps, eps_m=1e-12):
    """Alg. 3 for a block of b new rows at once (the columns of ``bmat``, R x b).

    The paper processes one slice per update and names several slices at once
    as future work (Sec. 6); this is the block form the single-row steps
    generalise to. Each new row is split against the span of V by the same two
    Gram-Schmidt passes; the residual block E (R x b) takes the place of e, and
    which of its directions to keep is the TruncatedSVD of Alg. 1 applied to E:
    the eigenpairs (lambda_i, w_i) of the Gram E^T E, and the smallest l whose
    tail lambda_{l+1} + ... + lambda_b is at most eps^2 (for b = 1 this keeps e
    exactly when ||e|| > eps). The kept directions Q = E W_l Lambda_l^{-1/2}
    extend V, and the middle matrix becomes

        S' = [[diag(S), 0], [P^T, W_l Lambda_l^{1/2}]]     ((r + b) x (r + l)),

    since row j of the block is p_j^T V^T + sum_i sqrt(lambda_i) W[j, i] Q_i^T
    up to the discarded tail. The orthogonality check covers V^T Q and
    Q^T Q - I; when it exceeds eps_m, [V Q] = Q' R' and S' -> S' R'^T as in
    Alg. 3. Returns ``(U~, S~, V~, info)`` with U~ = blockdiag(U, I_b) U''.
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    bmat = np.asarray(bmat, dtype=np.float64)
    r, b = s.shape[0], bmat.shape[1]
    p = v.T @ bmat
    e = bmat - v @ p
    p2 = v.T @ e
    e = e - v @ p2
    p = p + p2
    ell, w, sq, tail, lam = tsvd_gram(e.T, eps)
    q = e @ w / sq[None, :] if ell > 0 else np.zeros((v.shape[0], 0))
    k_mat = np.zeros((r + b, r + ell))
    k_mat[:r, :r] = np.diag(s)
    k_mat[r:, :r] = p.T
    k_mat[r:, r:] = w * sq[None, :]
    v_prime = np.hstack([v, q])
    orth = 0.0
    if ell > 0:
        orth = float(np.max(np.abs(q.T @ q - np.eye(ell))))
        if r > 0:
            orth = max(orth, float(np.max(np.abs(v.T @ q))))
    fired = ell > 0 and orth > eps_m
    if fired:
        qm, rm = np.linalg.qr(v_prime)
        v_prime = qm
        k_mat = k_mat @ rm.T
    u2, s_new, v2t = np.linalg.svd(k_mat, full_matrices=False)
    n = u.shape[0]
    u_new = np.vstack([u @ u2[:r, :], u2[r:, :]])
    v_new = v_prime @ v2t.T
    assert u_new.shape == (n + b, r + ell)
    info = dict(p=p, ell=ell, lam=lam, tail=tail, qr=fired, orth_check=orth, u2=u2)
    return u_new, s_new, v_new, info


# ----------------------------------------------------------------------------
# Alg. 4: non-streaming mode update
# ----------------------------------------------------------------------------

def _pad(x, k, extra):
    widths = [(0, 0)] * x.ndim
    widths[k] = (0, extra)
    return np.pad(x, widths)


def _reorth(w, u, passes=2):
    """Remove the span of U from W (two passes) and re-orthonormalise W."""
    for _ in range(passes):
        w = w - u @ (u.T @ w)
    if w.shape[1] > 0:
        w, rr = np.linalg.qr(w)
        w = w * np.sign(np.where(np.diag(rr) == 0, 1.0, np.diag(rr)))[None, :]
    return w


def non_streaming_update(k, u, c, d, v, eps, reorth=True):
    """NonStreamingUpdate(k, U_k, C_{k-1}, D*_{k-1}, V_{k-1}, eps) of Alg. 4.

    ``c`` and ``v`` are the d-way core and auxiliary tensors, ``d`` the
    (d-1)-way partial core of the new slice. Returns
    ``(U~_k, C_k, D*_k, V_k, info)``; info has ``e_norm`` (||E_k||), ``grew``,
    ``r_new`` (r'_k) and ``delta2``, the squared error this mode adds to the
    slice, ||D*_{k-1} - D*_k x_k U~_k||^2 (Prop. 3).
    """
    p_k = ttm(d, u.T, k)
    e_k = d - ttm(p_k, u, k)
    e_norm = float(np.linalg.norm(e_k))
    if e_norm <= eps:
        return u, c, p_k, v, dict(e_norm=e_norm, grew=False, r_new=0,
                                  delta2=e_norm * e_norm)
    n_k, r_k = u.shape
    r_new, w, _, tail, _ = tsvd_gram(unfold(e_k, k), eps, max_rank=n_k - r_k)
    if reorth:
        w = _reorth(w, u)
    l_k = ttm(e_k, w.T, k)
    u_new = np.hstack([u, w])
    c_k = _pad(c, k, r_new)
    d_k = np.concatenate([p_k, l_k], axis=k)
    v_k = _pad(v, k, r_new)
    return u_new, c_k, d_k, v_k, dict(e_norm=e_norm, grew=r_new > 0,
                                      r_new=r_new, delta2=tail)


# ----------------------------------------------------------------------------
# Alg. 5: streaming ST-HOSVD update, with the Alg. 2 initialisation
# ----------------------------------------------------------------------------

class StreamingTucker:
    """Streaming Tucker state (Assumption 1) and its per-slice update (Alg. 5).

    State: the core C (r_1 x ... x r_d), the factors U_1..U_d, the diagonal S
    and the auxiliary tensor V with C = V x_d S right after initialisation.
    ``xnorm2`` is ||X||^2 of all data seen and ``disc`` the accumulated bound on
    the squared reconstruction error (App. D): the initial ST-HOSVD error is the
    sum of the per-mode tails (Sec. 2.3), and each slice adds the per-mode
    residuals of Prop. 3 plus q^2 when the ISVD ignores e (Prop. 1).
    """

    def __init__(self, x0, tau, eps_m=1e-12, reorth=True, cgs2=True,
                 core_update="literal"):
        x0 = np.asarray(x0, dtype=np.float64)
        if not np.all(np.isfinite(x0)):
            raise ValueError("non-finite initial data")
        self.tau = float(tau)
        self.d = x0.ndim
        self.eps_m = eps_m
        self.reorth = reorth
        self.cgs2 = cgs2
        if core_update not in ("literal", "factored"):
            raise ValueError(core_update)
        self.core_update = core_update
        xnorm = float(np.linalg.norm(x0))
        if xnorm == 0.0:
            raise ValueError("degenerate initial data: ||X|| = 0")
        res = sthosvd(x0, tau)  # the streaming mode is processed last
        self.C = res["core"]
        self.U = list(res["factors"])
        self.S = res["s_last"]
        r = self.C.shape
        # V_(d) = V^T with V = A^T U_d S^{-1} (Sec. 3.2, core factorization)
        self.V = fold(res["v_last"].T, self.d - 1, r)
        self.xnorm2 = xnorm * xnorm
        self.disc = float(sum(res["tails"]))
        self.init_tails = list(res["tails"])
        self.history = []

    # -- accessors -------------------------------------------------------------
    @property
    def ranks(self):
        return tuple(self.C.shape)

    @property
    def n_slices(self):
        return self.U[-1].shape[0]

    def vmat(self):
        """V = V_(d)^T, rows indexed like vec() of a partial core."""
        return unfold(self.V, self.d - 1).T

    def recon_error_bound(self):
        return math.sqrt(self.disc / self.xnorm2)

    def reconstruct(self):
        return reconstruct(self.C, self.U)

    def reconstruct_slice(self, t):
        c = ttm(self.C, self.U[-1][t:t + 1, :], self.d - 1)
        return multi_ttm(c[..., 0], self.U[:-1])

    # -- Alg. 5 ----------------------------------------------------------------
    def update(self, y):
        y = np.asarray(y, dtype=np.float64)
        d = self.d
        if y.shape != tuple(u.shape[0] for u in self.U[:-1]):
            raise ValueError("slice shape mismatch")
        ynorm = float(np.linalg.norm(y))
        if not math.isfinite(ynorm):
            raise ValueError("non-finite slice")
        eps = self.tau * ynorm / math.sqrt(d)
        c_k, d_k, v_k = self.C, y, self.V
        rec = dict(eps=eps, ynorm=ynorm, e_norm=[], grew=[], r_new=[])
        delta2 = 0.0
        for k in range(d - 1):
            u_new, c_k, d_k, v_k, info = non_streaming_update(
                k, self.U[k], c_k, d_k, v_k, eps, reorth=self.reorth)
            self.U[k] = u_new
            delta2 += info["delta2"]
            rec["e_norm"].append(info["e_norm"])
            rec["grew"].append(info["grew"])
            rec["r_new"].append(info["r_new"])
        dvec = vec(d_k)
        r_sp = c_k.shape[:-1]
        vmat = unfold(v_k, d - 1).T
        ud_old = self.U[-1]
        n_d = ud_old.shape[0]
        ud_new, s_new, v_new, info = isvd(ud_old, self.S, vmat, dvec, eps,
                                          eps_m=self.eps_m, cgs2=self.cgs2)
        r_d_new = s_new.shape[0]
        v_tensor = fold(v_new.T, d - 1, r_sp + (r_d_new,))
        if self.core_update == "literal":
            # C~ = C_{d-1} x_d (U~_d(1:n_d,:)^T U_d) + D*_{d-1} x_d U~_d(n_d+1,:)^T
            m = ud_new[:n_d, :].T @ ud_old
            c_new = ttm(c_k, m, d - 1)
            c_new = c_new + ttm(d_k[..., None], ud_new[n_d:n_d + 1, :].T, d - 1)
        else:
            c_new = ttm(v_tensor, np.diag(s_new), d - 1)
        if info["ignored"]:
            delta2 += info["q"] ** 2
        self.C, self.V, self.S = c_new, v_tensor, s_new
        self.U[-1] = ud_new
        self.xnorm2 += ynorm * ynorm
        self.disc += delta2
        rec.update(q=info["q"], ignored=bool(info["ignored"]), qr=info["qr"],
                   orth_single_pass=info["orth_single_pass"], orth_check=info["orth_check"],
                   delta2=delta2, ranks=self.ranks)
        self.history.append(rec)
        return rec

    def update_block(self, yb):
        """Alg. 5 for b slices at once: ``yb`` has the slice shape plus a last
        mode of size b (the slices in stream order).

        The per-update tolerance is that of the block, eps = tau ||Y_B|| / sqrt(d):
        each update then discards at most d eps^2 = tau^2 ||Y_B||^2, and over a
        stream cut into blocks the squared error stays within tau^2 ||X||^2, the
        argument of App. D with the block in place of the slice. Alg. 4 runs on
        the block tensor (its block mode is carried along like the slice modes,
        so the residual Gram of mode k sums over all b slices), and the streaming
        mode takes block_isvd. With b = 1 this is update().
        """
        yb = np.asarray(yb, dtype=np.float64)
        d = self.d
        shape = tuple(u.shape[0] for u in self.U[:-1])
        if yb.ndim != d or yb.shape[:-1] != shape or yb.shape[-1] < 1:
            raise ValueError("block shape mismatch")
        b = yb.shape[-1]
        ynorm = float(np.linalg.norm(yb))
        if not math.isfinite(ynorm):
            raise ValueError("non-finite block")
        eps = self.tau * ynorm / math.sqrt(d)
        c_k, d_k, v_k = self.C, yb, self.V
        rec = dict(eps=eps, ynorm=ynorm, b=b, e_norm=[], grew=[], r_new=[])
        delta2 = 0.0
        for k in range(d - 1):
            u_new, c_k, d_k, v_k, info = non_streaming_update(
                k, self.U[k], c_k, d_k, v_k, eps, reorth=self.reorth)
            self.U[k] = u_new
            delta2 += info["delta2"]
            rec["e_norm"].append(info["e_norm"])
            rec["grew"].append(info["grew"])
            rec["r_new"].append(info["r_new"])
        r_sp = c_k.shape[:-1]
        bmat = unfold(d_k, d - 1).T  # R x b: column j is vec of slice j's partial core
        vmat = unfold(v_k, d - 1).T
        ud_old = self.U[-1]
        n_d = ud_old.shape[0]
        ud_new, s_new, v_new, info = block_isvd(ud_old, self.S, vmat, bmat, eps,
                                                eps_m=self.eps_m)
        r_d_new = s_new.shape[0]
        v_tensor = fold(v_new.T, d - 1, r_sp + (r_d_new,))
        if self.core_update == "literal":
            m = ud_new[:n_d, :].T @ ud_old
            c_new = ttm(c_k, m, d - 1) + ttm(d_k, ud_new[n_d:n_d + b, :].T, d - 1)
        else:
            c_new = ttm(v_tensor, np.diag(s_new), d - 1)
        delta2 += info["tail"]
        self.C, self.V, self.S = c_new, v_tensor, s_new
        self.U[-1] = ud_new
        self.xnorm2 += ynorm * ynorm
        self.disc += delta2
        rec.update(ell=info["ell"], lam=info["lam"], tail=info["tail"], qr=info["qr"],
                   orth_check=info["orth_check"], delta2=delta2, ranks=self.ranks)
        self.history.append(rec)
        return rec
