// Streaming Tucker engine: device state, the initial ST-HOSVD (Alg. 2) and the
// per-slice update (Alg. 5 = Alg. 4 on every slice mode, then Alg. 3 on the
// streaming mode and the core update), behind the C ABI of stucker.h.
//
// Host code only orchestrates: every arithmetic step of the update runs in the
// kernels of k_fiber.hip / k_isvd.hip, except the small symmetric
// eigendecompositions of the Gram matrices, which run on the device through
// rocSOLVER (FP64). The host reads back the scalars that decide the branches
// (norms, eigenvalues for the rank rule) and the new ranks.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stucker.h"
#include "common.hpp"
#include "kernels.hpp"
#include "secular.hpp"

using namespace st;

namespace {

template <class T>
struct DBuf {
  T *p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t n) {
    if (n <= cap && p) return hipSuccess;
    size_t want = std::max(n, cap + cap / 2);
    if (want == 0) want = 1;
    T *q = nullptr;
    hipError_t e = hipMalloc((void **)&q, want * sizeof(T));
    if (e != hipSuccess) {
      want = n > 0 ? n : 1;
      e = hipMalloc((void **)&q, want * sizeof(T));
      if (e != hipSuccess) return e;
    }
    if (p) (void)hipFree(p);
    p = q;
    cap = want;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

thread_local std::string g_create_error;  // st_create and the stateless calls

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Rank rule of Alg. 1 on eigenvalues given in ascending order: descending
// order, negative round-off clamped to zero, tail sums from the smallest up,
// r = min{l : tail(l) <= eps^2}. Returns r and tail(r).
void rank_rule(const double *lam_asc, int64_t n, double eps, int64_t &r, double &tail_r,
               std::vector<double> &desc) {
  desc.resize(n);
  for (int64_t i = 0; i < n; ++i) desc[i] = std::max(lam_asc[n - 1 - i], 0.0);
  std::vector<double> tail(n + 1, 0.0);
  for (int64_t l = n - 1; l >= 0; --l) tail[l] = tail[l + 1] + desc[l];
  const double e2 = eps * eps;
  r = n;
  for (int64_t l = 0; l <= n; ++l)
    if (tail[l] <= e2) {
      r = l;
      break;
    }
  tail_r = tail[r];
}

}  // namespace

namespace st {
void set_stateless_error(const char *msg) { g_create_error = msg ? msg : ""; }
}  // namespace st

struct st_handle {
  // configuration
  int m = 0;  // slice modes
  int64_t n[ST_MAX_MODES] = {};
  int64_t NY = 0;
  double tau = 0.0;
  Prec prec = Prec::FP32;
  double orth_tol = 1e-12;
  int64_t qr_total = 0;  // QR fixes applied since init
  int64_t blk = 1;       // slices in the update being processed (block updates)
  int cus = 0;           // compute units of the device (cached)
  int device_cus() {
    if (cus <= 0) {
      int c = 0;
      cus = (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) ==
                 hipSuccess &&
             c > 0)
                ? c
                : 256;
    }
    return cus;
  }
  double guard_rel = 0.0;
  int64_t max_rank_d = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  rocblas_handle rb = nullptr;
  std::string err;

  // decomposition
  bool inited = false;
  bool factored = false;  // ST_CORE_FACTORED: V = V0 M, C = V x_d S
  int64_t r[ST_MAX_MODES] = {};
  int64_t rd = 0, nd = 0;
  double xnorm2 = 0.0, disc = 0.0;
  std::vector<double> S_host;
  st_slice_stats stats{};

  // factors of the slice modes (capacity n_k columns)
  double *U64[ST_MAX_MODES] = {};
  float *Uf[ST_MAX_MODES] = {};
  float *Ut[ST_MAX_MODES] = {};
  __bf16 *Uh[ST_MAX_MODES] = {};
  __bf16 *Ul[ST_MAX_MODES] = {};
  int64_t ldb[ST_MAX_MODES] = {};

  // streaming-mode state (ping-pong)
  DBuf<double> Ud[2];
  int64_t ud_ld[2] = {0, 0};
  DBuf<double> S[2];
  DBuf<double> V[2];  // auxiliary matrix (FP64 in every form: it decides the ISVD test)
  DBuf<float> C[2];   // core, mode-d unfolding transposed
  int cur = 0;
  // factored form: V[v0cur] holds V0 (rows at the current ranks, ld = R);
  // Mf[cur] holds M (r_d x r_d, ld r_d)
  int v0cur = 0;
  DBuf<double> Mf[2], Gf[2];  // M and G0 = V0^T V0 (r_d x r_d)
  DBuf<double> tvec, wvec, e1buf, tmp64, qrw, qrg, qvte;
  DBuf<double> bV, bE, bQ, bC, bsm;  // block updates: V at new rows, E, Q, FP64 core, small
  DBuf<double> bsec;  // block updates: the middle-matrix SVD by row appends
  DBuf<int> qstat;
  DBuf<float> tmp32;

  // work buffers
  DBuf<double> D[2];   // partial cores D*_k of the update (FP64)
  DBuf<double> Dspec[ST_MAX_MODES], specpart, specsums;  // the no-growth pass over all modes
  DBuf<float> RB[2], wrow;  // reconstruction work
  DBuf<double> part, sums;
  DBuf<double> gram_part;
  DBuf<double> G, eigval, eigwork, Wnew, coef;
  DBuf<double> eigtri;  // tridiagonal form and reflections of the last small Gram
  bool eig_lazy = false;  // its eigenvectors are computed on demand (eig_top)
  DBuf<int> info;
  DBuf<double> colpart, q2part, p1, p2, p;
  DBuf<double> U2, V2;
  DBuf<double> Wv;
  DBuf<float> Wc;
  DBuf<double> dlt, pref;  // ISVD refinement: delta = d_exact - d, V^T delta and p
  // secular scratch
  DBuf<double> sd, sz, szh, smu, srot_cs, szz;
  DBuf<int> sact, sK, sdefl, sorg, srot_t, scounts;
  double *hpin = nullptr;  // pinned host scratch
  double *hpin_dev = nullptr;  // device view of hpin (kernels publish results there)
  // Singular values of the last update, published to pinned memory (hS) without
  // a synchronisation; taken into S_host by finish_pending() after the next one.
  double *hS = nullptr, *hS_dev = nullptr;
  size_t hS_cap = 0;
  int64_t s_pending = 0;
  size_t hpin_cap = 0, hpin_cap_prev = 0;

  // optional per-group timing with HIP events on `stream`
  bool profile = false;
  st_kernel_profile prof[ST_K_GROUPS] = {};
  struct Pending {
    int group;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Bracket a launch sequence: tic() before, toc(group, flops, bytes) after.
  hipEvent_t tic_ev = nullptr;
  void tic() {
    if (!profile) return;
    tic_ev = get_event();
    if (tic_ev) (void)hipEventRecord(tic_ev, stream);
  }
  void toc(int group, double flops, double bytes) {
    if (!profile || !tic_ev) return;
    hipEvent_t b = get_event();
    if (!b) return;
    (void)hipEventRecord(b, stream);
    pending.push_back(Pending{group, tic_ev, b, flops, bytes});
    tic_ev = nullptr;
  }
  // After a stream synchronisation: fold finished intervals into the counters.
  void settle() {
    for (auto &pd : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
        prof[pd.group].launches += 1;
        prof[pd.group].ms += ms;
        prof[pd.group].flops += pd.flops;
        prof[pd.group].bytes += pd.bytes;
      }
      event_pool.push_back(pd.a);
      event_pool.push_back(pd.b);
    }
    pending.clear();
  }

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }

  int hipfail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory)
      return fail(ST_ENOMEM, "%s: out of device memory", what);
    return fail(ST_EHIP, "%s: %s", what, hipGetErrorString(e));
  }

  FiberW wmat(int k) const {
    FiberW w{};
    w.w = Uf[k];
    w.ldw = n[k];
    w.w_hi = Uh[k];
    w.w_lo = Ul[k];
    w.ldw_bf = ldb[k];
    w.w64 = U64[k];
    return w;
  }

  int64_t rprod(const int64_t *rr, int upto) const {
    int64_t p_ = 1;
    for (int k = 0; k < upto; ++k) p_ *= rr[k];
    return p_;
  }
  // product of the slice dims from mode `from` on, times the number of slices
  // in the update being processed (blk = 1 except inside a block update, whose
  // block mode is carried along the slice-mode chain like another slice mode)
  int64_t nprod(int from) const {
    int64_t p_ = blk;
    for (int k = from; k < m; ++k) p_ *= n[k];
    return p_;
  }

  // (only while no publication into hS is pending)
  hipError_t ensure_hS(size_t count) {
    if (count <= hS_cap) return hipSuccess;
    if (hS) (void)hipHostFree(hS);
    hS = hS_dev = nullptr;
    hS_cap = 0;
    const size_t want = std::max<size_t>(count, 2 * count + 64);
    hipError_t e = hipHostMalloc((void **)&hS, want * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&hS_dev, hS, 0);
    if (e == hipSuccess) hS_cap = want;
    return e;
  }
  // After a stream synchronisation: take the last update's singular values.
  // The host state an update changes at its commit. Device state needs no copy:
  // an update writes its new V / C / M / G0 / U_d / S into the other half of
  // each ping-pong pair and its new factor or V0 columns past the committed
  // ranks, and the next update overwrites neither before it has validated the
  // pending singular values (its first synchronisation).
  struct Committed {
    int64_t r[ST_MAX_MODES];
    int64_t rd, nd;
    int cur, v0cur;
    double xnorm2, disc;
    st_slice_stats stats;
    int64_t qr_total;
  } prev{};
  void snapshot() {
    std::copy(r, r + ST_MAX_MODES, prev.r);
    prev.rd = rd;
    prev.nd = nd;
    prev.cur = cur;
    prev.v0cur = v0cur;
    prev.xnorm2 = xnorm2;
    prev.disc = disc;
    prev.stats = stats;
    prev.qr_total = qr_total;
  }
  void rollback() {
    std::copy(prev.r, prev.r + ST_MAX_MODES, r);
    rd = prev.rd;
    nd = prev.nd;
    cur = prev.cur;
    v0cur = prev.v0cur;
    xnorm2 = prev.xnorm2;
    disc = prev.disc;
    stats = prev.stats;
    qr_total = prev.qr_total;
  }
  // Validates the singular values the last update published without a
  // synchronisation (call after one). If one is not positive, that update is
  // undone and the error is reported by this call: the state is the one before
  // it, as if it had failed.
  int finish_pending() {
    if (!s_pending) return ST_OK;
    const int64_t c = s_pending;
    s_pending = 0;
    for (int64_t i = 0; i < c; ++i)
      if (!std::isfinite(hS[i]) || hS[i] <= 0.0) {
        rollback();
        return fail(ST_ESOLVER,
                    "the last update was rolled back: its small SVD produced a non-positive "
                    "singular value");
      }
    S_host.assign(hS, hS + c);
    return ST_OK;
  }
  // Synchronises and validates a pending publication (readers of the state).
  int take_pending() {
    if (!s_pending) return ST_OK;
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "pending update");
    settle();
    return finish_pending();
  }

  // Pinned scratch for the scalars and short vectors the host reads back. It is
  // separate from hS (a pending publication of the last update's singular
  // values stays valid across a regrowth) and grows geometrically.
  hipError_t ensure_pinned(size_t count) {
    if (count <= hpin_cap) return hipSuccess;
    // work queued by earlier calls may still read or write the old buffer
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    if (hpin) (void)hipHostFree(hpin);
    hpin = hpin_dev = nullptr;
    hpin_cap = 0;
    const size_t want = std::max(count, 2 * hpin_cap_prev);
    e = hipHostMalloc((void **)&hpin, want * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&hpin_dev, hpin, 0);
    if (e != hipSuccess) {
      if (hpin) (void)hipHostFree(hpin);
      hpin = hpin_dev = nullptr;
      return e;
    }
    hpin_cap = want;
    hpin_cap_prev = want;
    return hipSuccess;
  }

  // Norms of E and X for mode k into hpin[0..1].
  int project_resid(const FiberIn &in, const FiberW &w, int rows, const FiberOut &out, Prec pr,
                    int group) {
    hipError_t e = part.ensure(2 * (size_t)fiber_max_blocks(in.F));
    if (e != hipSuccess) return hipfail(e, "partials");
    int nb = 0;
    tic();
    e = launch_fiber_project(in, w, 0, rows, out, part.p, pr, stream, &nb);
    if (e != hipSuccess) return hipfail(e, "fiber projection + residual");
    // P = D x_k U^T and E = D - P x_k U: 4 F n r flops; D read once, P written once
    toc(group, 4.0 * in.F * in.n * rows, 4.0 * in.F * (in.n + rows));
    e = launch_reduce_pairs(part.p, nb, sums.p, stream);
    if (e != hipSuccess) return hipfail(e, "reduce");
    e = hipMemcpyAsync(hpin, sums.p, 2 * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "residual norms");
    settle();
    return ST_OK;
  }

  // Gram of the residual (rows > 0) or of the tensor (rows == 0) for fibres of
  // length nk, then its eigendecomposition; eigenvalues (ascending) land in
  // hpin[0..nk), eigenvectors in G.
  // P (optional): the FP64-product projection of the same fibres, which lets the
  // mode-1 Gram of the slice form E from it (gram_contig) instead of projecting again
  int gram_eig(const FiberIn &in, const FiberW &w, int rows, int64_t nk, GramPrec pr,
               bool e64, const double *P = nullptr) {
    const int gnb = gram_blocks(in.F, nk, pr);
    hipError_t e = gram_part.ensure(gram_partial_elems(nk, gnb, pr));
    if (e == hipSuccess) e = G.ensure((size_t)nk * nk);
    if (e == hipSuccess) e = eigval.ensure(nk);
    if (e == hipSuccess) e = eigwork.ensure(nk);
    if (e == hipSuccess) e = info.ensure(1);
    if (e == hipSuccess) e = ensure_pinned(nk + 8);
    if (e != hipSuccess) return hipfail(e, "gram buffers");
    tic();
    if (P != nullptr && e64 && w.w64 != nullptr && gram_contig_eligible(in, rows, pr)) {
      // one block per CU (one wave per SIMD; each wave walks its fibre tiles)
      const int nbc = std::min(gnb, device_cus());
      e = launch_gram_contig(in, w.w64, nk, rows, P, gram_part.p, nbc, stream);
      if (e == hipSuccess) e = launch_gram_reduce(gram_part.p, nbc, nk, G.p, stream);
      if (e != hipSuccess) return hipfail(e, "gram");
      // E = X - U P (2 F n r) and the lower triangle of E E^T (F n^2); X and P read
      toc(ST_K_GRAM, 2.0 * in.F * nk * rows + 1.0 * in.F * nk * nk,
          4.0 * in.F * nk + 8.0 * in.F * rows);
    } else {
      e = launch_gram(in, w, rows, gram_part.p, gnb, pr, e64, stream, G.p);
      if (e != hipSuccess) return hipfail(e, "gram");
      // recompute E (4 F n r) and form the lower triangle of E E^T (F n^2)
      toc(ST_K_GRAM, 4.0 * in.F * nk * rows + 1.0 * in.F * nk * nk,
          (in.x64 ? 8.0 : 4.0) * in.F * nk);
    }
    tic();
    int hinfo = 0;
    eig_lazy = eig_small_supported((int)nk);
    if (eig_lazy) {
      // own kernels: eigenvalues now, eigenvectors of the kept ones in eig_top
      e = eigtri.ensure(eig_work_elems((int)nk));
      if (e == hipSuccess) e = launch_eig_tridiag(G.p, (int)nk, eigtri.p, stream);
      if (e == hipSuccess) e = launch_eig_values(eigtri.p, (int)nk, eigval.p, stream);
      toc(ST_K_EIG, (4.0 / 3.0) * nk * nk * nk + 10.0 * 64.0 * 3.0 * nk * nk, 8.0 * nk * nk);
      if (e != hipSuccess) return hipfail(e, "eigenvalues");
      e = hipMemcpyAsync(hpin, eigval.p, nk * sizeof(double), hipMemcpyDeviceToHost, stream);
    } else {
      rocblas_status rs = rocsolver_dsyevd(rb, rocblas_evect_original, rocblas_fill_lower,
                                           (rocblas_int)nk, G.p, (rocblas_int)nk, eigval.p,
                                           eigwork.p, info.p);
      toc(ST_K_EIG, 9.0 * nk * nk * nk, 16.0 * nk * nk);
      if (rs != rocblas_status_success) return fail(ST_ESOLVER, "rocsolver_dsyevd status %d", rs);
      e = hipMemcpyAsync(hpin, eigval.p, nk * sizeof(double), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "eigenvalues");
    settle();
    if (hinfo != 0) return fail(ST_ESOLVER, "rocsolver_dsyevd info %d", hinfo);
    for (int64_t i = 0; i < nk; ++i)
      if (!std::isfinite(hpin[i])) return fail(ST_ENONFINITE, "non-finite Gram eigenvalue");
    return ST_OK;
  }

  // Eigenvectors of the cnt largest eigenvalues of the last gram_eig into the
  // last cnt columns of G (column nk-1-c for the c-th largest), where the
  // library solver has not already written every eigenvector there.
  int eig_top(int64_t nk, int64_t cnt) {
    if (!eig_lazy || cnt <= 0) return ST_OK;
    tic();
    const hipError_t e =
        launch_eig_vectors(eigtri.p, (int)nk, eigval.p, (int)cnt, G.p, nk, 0, stream);
    toc(ST_K_EIG, 4.0 * cnt * nk * nk + 40.0 * cnt * nk, 8.0 * cnt * nk * 2.0);
    if (e != hipSuccess) return hipfail(e, "eigenvectors");
    return ST_OK;
  }

  int append_columns(int k, int64_t c0, int64_t cnt) {
    const int rc = eig_top(n[k], cnt);
    if (rc != ST_OK) return rc;
    const int64_t nk = n[k];
    hipError_t e = Wnew.ensure((size_t)nk * cnt);
    if (e == hipSuccess) e = coef.ensure((size_t)std::max<int64_t>(c0, 1) * cnt);
    if (e != hipSuccess) return hipfail(e, "new columns");
    e = launch_new_columns(G.p, nk, U64[k], (int)c0, (int)cnt, Wnew.p, coef.p, stream);
    if (e != hipSuccess) return hipfail(e, "reorthogonalise new columns");
    e = launch_append_cols(Wnew.p, nk, (int)c0, (int)cnt, U64[k], Uf[k], Ut[k], Uh[k], Ul[k],
                           ldb[k], stream);
    if (e != hipSuccess) return hipfail(e, "append columns");
    return ST_OK;
  }

  SecData secdata(int rr) {
    SecData s{};
    s.n = rr + 1;
    s.r = rr;
    s.d = sd.p;
    s.z = sz.p;
    s.zh = szh.p;
    s.active = sact.p;
    s.K = sK.p;
    s.defl = sdefl.p;
    s.org = sorg.p;
    s.mu = smu.p;
    s.rot_t = srot_t.p;
    s.rot_cs = srot_cs.p;
    s.counts = scounts.p;
    s.zz = szz.p;
    return s;
  }

  hipError_t ensure_secular(int64_t nn) {
    hipError_t e = sd.ensure(nn);
    if (e == hipSuccess) e = sz.ensure(nn);
    if (e == hipSuccess) e = szh.ensure(nn);
    if (e == hipSuccess) e = smu.ensure(nn);
    if (e == hipSuccess) e = srot_cs.ensure(2 * nn);
    if (e == hipSuccess) e = szz.ensure(1);
    if (e == hipSuccess) e = sact.ensure(nn);
    if (e == hipSuccess) e = sK.ensure(nn);
    if (e == hipSuccess) e = sdefl.ensure(nn);
    if (e == hipSuccess) e = sorg.ensure(nn);
    if (e == hipSuccess) e = srot_t.ensure(2 * nn);
    if (e == hipSuccess) e = scounts.ensure(4);
    return e;
  }

  // Tail band of the rank rule of Alg. 1 for a reduced-precision Gram, as a
  // fraction of the Gram's trace: a tail sum within this band of eps^2 is
  // decided again on the FP64 Gram.
  double tail_band(GramPrec gp) const {
    return gp == GramPrec::FP64 ? 0.0 : (gp == GramPrec::BF16X3 ? 1e-3 : 1e-5);
  }
  static bool tail_in_band(const std::vector<double> &desc, double eps, double band) {
    if (band <= 0.0) return false;
    double trace = 0.0;
    for (double v : desc) trace += v;
    const double e2 = eps * eps, w = band * std::max(trace, e2);
    double tail = 0.0;
    for (int64_t l = (int64_t)desc.size(); l >= 0; --l) {
      if (std::fabs(tail - e2) <= w) return true;
      if (l > 0) tail += desc[l - 1];
    }
    return false;
  }
  int exact_coords(const float *y, const double **dout);
  int do_init(const float *x0, int64_t n_init);
  int do_update(const float *y, int64_t b = 1);
  hipError_t block_rows_svd(const double *K, int n2, int rdi, int bi, int c, double tol,
                            double *Uo, double *Vo, double *So);
  int stream_block(const RowMap &map, const double *Dm, int64_t b, int64_t Rold, int64_t Rnew,
                   double eps, st_slice_stats &stt, const int64_t *rn, double delta2,
                   double ynorm2, double ms_modes, clk::time_point t0);
  hipError_t chunk_tn(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t R,
                      int p, int q, double *out);
  int stream_factored(const RowMap &map, const double *dvec, int64_t Rold, int64_t Rnew,
                      double eps, st_slice_stats &stt, int &grow, double &q2, int64_t &c,
                      int &v0next, bool exact_d, const float *y);
  hipError_t factored_product(const double *S_or_null, double *out64);
  hipError_t init_g0(int64_t R, int rk);
  hipError_t chunk_gram(const double *X, int64_t R, int r, double *out);
  int qr_fix(const double *Gtop, int rdi, const double *vte, const double *ee, const double *pv,
             double tol, int nxt);
  int do_reconstruct_slice(int64_t t, float *out);
  void destroy();
};

// ---------------------------------------------------------------------------
// Alg. 2 with the streaming mode processed last.
// ---------------------------------------------------------------------------
int st_handle::do_init(const float *x0, int64_t n_init) {
  const auto t0 = clk::now();
  if (inited) return fail(ST_ESTATE, "already initialised");
  if (x0 == nullptr || n_init < 1) return fail(ST_EINVAL, "bad initial data");
  const int d = m + 1;
  const int64_t N0 = NY * n_init;
  hipError_t e = ensure_pinned(256);
  if (e != hipSuccess) return hipfail(e, "pinned buffer");

  // ||X0||^2 in FP64
  {
    const int nb = 1024;
    e = part.ensure(2 * nb);
    if (e != hipSuccess) return hipfail(e, "partials");
    e = launch_sumsq(x0, N0, part.p, nb, stream);
    if (e == hipSuccess) e = launch_reduce_pairs(part.p, nb, sums.p, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hpin, sums.p, 2 * sizeof(double), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "norm of initial data");
  }
  const double xn2 = hpin[0];
  if (!std::isfinite(xn2)) return fail(ST_ENONFINITE, "initial data is not finite");
  if (xn2 == 0.0) return fail(ST_EDEGENERATE, "initial data is zero");
  const double eps = tau * std::sqrt(xn2 / d);

  int64_t rr[ST_MAX_MODES] = {};
  double tails = 0.0;
  std::vector<double> desc;
  DBuf<double> T[2];
  const void *Din = x0;
  int din64 = 0;
  int sel = 0;
  int rc = ST_OK;
  for (int k = 0; k <= m && rc == ST_OK; ++k) {
    const int64_t a = rprod(rr, k);
    const int64_t nk = (k < m) ? n[k] : n_init;
    const int64_t b = (k < m) ? nprod(k + 1) * n_init : 1;
    FiberIn in{};
    in.x = Din;
    in.x64 = din64;
    in.a = a;
    in.n = nk;
    in.F = a * b;
    // Gram of the data itself: eigenvalues near eps^2 = tau^2 ||X||^2 / d must
    // be resolved, so the products are accumulated exactly in FP64.
    rc = gram_eig(in, FiberW{}, 0, nk, GramPrec::FP64, false);
    if (rc != ST_OK) break;
    int64_t rk;
    double tail;
    rank_rule(hpin, nk, eps, rk, tail, desc);
    if (k == m && max_rank_d > 0 && rk > max_rank_d) {
      rc = fail(ST_ECAPACITY, "initial streaming rank %lld exceeds the cap", (long long)rk);
      break;
    }
    if (rk == 0) {
      rc = fail(ST_EDEGENERATE, "rank 0 in mode %d", k + 1);
      break;
    }
    // the discarded tail with the chosen rank
    tail = 0.0;
    for (int64_t i = rk; i < nk; ++i) tail += desc[i];
    tails += tail;
    if (k < m) {
      rc = append_columns(k, 0, rk);
      if (rc != ST_OK) break;
      rr[k] = rk;
      e = T[sel].ensure((size_t)(a * rk * b));
      if (e != hipSuccess) {
        rc = hipfail(e, "init partial core");
        break;
      }
      // the initial chain runs once: exact FP64 products in every form (with
      // FP32 products, V = A^T U_d S^-1 would carry u s_1 / s_k in its columns
      // of small singular value and start out non-orthonormal)
      FiberOut out{T[sel].p, 1, a, rk};
      e = launch_fiber_project(in, wmat(k), 0, (int)rk, out, nullptr, Prec::FP64, stream);
      if (e != hipSuccess) {
        rc = hipfail(e, "init projection");
        break;
      }
      Din = T[sel].p;
      din64 = 1;
      sel ^= 1;
    } else {
      const int64_t R = a;
      rd = rk;
      nd = n_init;
      const int64_t ldu = round_up(std::max<int64_t>(2 * n_init, 64), 64);
      e = Ud[cur].ensure((size_t)ldu * std::max<int64_t>(rk, 1));
      if (e == hipSuccess) e = Wnew.ensure((size_t)nk * rk);
      if (e == hipSuccess) e = S[cur].ensure(rk);
      if (e != hipSuccess) {
        rc = hipfail(e, "streaming factor");
        break;
      }
      ud_ld[cur] = ldu;
      rc = eig_top(nk, rk);
      if (rc != ST_OK) break;
      e = launch_new_columns(G.p, nk, nullptr, 0, (int)rk, Wnew.p, nullptr, stream);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(Ud[cur].p, ldu * sizeof(double), Wnew.p, nk * sizeof(double),
                             nk * sizeof(double), rk, hipMemcpyDeviceToDevice, stream);
      S_host.assign(rk, 0.0);
      for (int64_t i = 0; i < rk; ++i) S_host[i] = std::sqrt(desc[i]);
      if (e == hipSuccess)
        e = hipMemcpyAsync(S[cur].p, S_host.data(), rk * sizeof(double), hipMemcpyHostToDevice,
                           stream);
      // factored form: room for later appended columns of V0; M = I
      if (e == hipSuccess)
        e = V[cur].ensure(factored ? (size_t)R * (rk + 16) : (size_t)(R * rk));
      if (e == hipSuccess && !factored) e = C[cur].ensure((size_t)(R * rk));
      if (e == hipSuccess && factored) e = Mf[cur].ensure((size_t)(rk * rk));
      if (e == hipSuccess && factored) e = launch_identity(Mf[cur].p, (int)rk, stream);
      if (e == hipSuccess && factored) e = Gf[cur].ensure((size_t)(rk * rk));
      v0cur = cur;
      // V = A^T U_d S^-1 and C_(d)^T = A^T U_d, A = C*_{d-1,(d)} (FP64 accumulation)
      if (e == hipSuccess && !din64) e = hipErrorInvalidValue;  // d >= 2: A is a partial core
      if (e == hipSuccess)
        e = launch_init_vc(static_cast<const double *>(Din), R, n_init, Ud[cur].p, ldu, (int)rk,
                           S[cur].p, V[cur].p, factored ? nullptr : C[cur].p, stream);
      if (e == hipSuccess && factored) e = init_g0(R, (int)rk);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) {
        rc = hipfail(e, "init core");
        break;
      }
    }
  }
  T[0].release();
  T[1].release();
  if (rc != ST_OK) {
    for (int k = 0; k < m; ++k) r[k] = 0;
    rd = nd = 0;
    return rc;
  }
  for (int k = 0; k < m; ++k) r[k] = rr[k];
  xnorm2 = xn2;
  disc = tails;
  inited = true;
  stats = st_slice_stats{};
  stats.ynorm = std::sqrt(xn2);
  stats.eps = eps;
  stats.delta2 = tails;
  stats.ms_total = ms_since(t0);
  return ST_OK;
}

// ---------------------------------------------------------------------------
// d = vec(Y x_1 U_1^T ... x_{d-1} U_{d-1}^T) at the current ranks with FP64
// products (the exact coordinates of a slice whose slice modes all kept their
// factors), into one of the two partial-core buffers.
// ---------------------------------------------------------------------------
int st_handle::exact_coords(const float *y, const double **dout) {
  const void *x = y;
  int x64 = 0, sel = 0;
  for (int k = 0; k < m; ++k) {
    const int64_t a = rprod(r, k), b = nprod(k + 1);
    FiberIn in{};
    in.x = x;
    in.x64 = x64;
    in.a = a;
    in.n = n[k];
    in.F = a * b;
    tic();
    hipError_t e = launch_fiber_project(in, wmat(k), 0, (int)r[k], FiberOut{D[sel].p, 1, a, r[k]},
                                        nullptr, Prec::FP64, stream);
    toc(ST_K_REFINE, 2.0 * in.F * n[k] * r[k], (x64 ? 8.0 : 4.0) * in.F * n[k] + 8.0 * in.F * r[k]);
    if (e != hipSuccess) return hipfail(e, "FP64 slice coordinates");
    x = D[sel].p;
    x64 = 1;
    sel ^= 1;
  }
  *dout = static_cast<const double *>(x);
  return ST_OK;
}

// ---------------------------------------------------------------------------
// Alg. 5.
// ---------------------------------------------------------------------------
int st_handle::do_update(const float *y, int64_t bsz) {
  const auto t0 = clk::now();
  if (!inited) return fail(ST_ESTATE, "update before init");
  if (y == nullptr) return fail(ST_EINVAL, "null slice");
  if (bsz < 1) return fail(ST_EINVAL, "block of %lld slices", (long long)bsz);
  const int d = m + 1;
  st_slice_stats stt{};
  int64_t rn[ST_MAX_MODES];
  for (int k = 0; k < m; ++k) rn[k] = r[k];
  // (a block update also reads back b eigenvalues and V^T Q, Q^T Q: b (r_d + b))
  hipError_t e = ensure_pinned(2 * (size_t)std::max<int64_t>(rd + 2, 64) + 64 +
                               (size_t)(bsz * (rd + bsz) + 4 * bsz));
  if (e != hipSuccess) return hipfail(e, "pinned buffer");
  // the slice-mode chain below runs on all bsz slices at once (nprod includes blk)
  struct BlkScope {
    int64_t &b;
    ~BlkScope() { b = 1; }
  } blk_scope{blk};
  blk = bsz;
  if (bsz > 1) {
    e = D[0].ensure((size_t)(NY * bsz));
    if (e == hipSuccess) e = D[1].ensure((size_t)(NY * bsz));
    if (e != hipSuccess) return hipfail(e, "block buffers");
  }

  std::vector<double> desc;
  const void *Din = y;
  int din64 = 0;
  int dsel = 0;
  double delta2 = 0.0, eps = 0.0, ynorm2 = 0.0;
  int rc;
  // reduced-precision products (FP32, bf16x3) decide only clear of the guard band
  const bool fast = prec != Prec::FP64;
  Prec mp = prec;             // product precision of the per-mode loop below
  bool exact_d = !fast;       // d = vec(D*_{d-1}) carries FP64 products
  // Every mode is first projected at the current ranks, the case of no growth
  // (Alg. 4 keeping U_k for every k), and the residual norms of all modes come
  // back with one synchronisation. From the first mode whose test fails or
  // falls in the guard band, the modes are redone one at a time below.
  int k0 = 0;
  {
    size_t poff[ST_MAX_MODES + 1];
    poff[0] = 0;
    for (int k = 0; k < m; ++k)
      poff[k + 1] = poff[k] + 2 * (size_t)fiber_max_blocks(rprod(r, k) * nprod(k + 1));
    e = specpart.ensure(poff[m]);
    if (e == hipSuccess) e = specsums.ensure(2 * (size_t)m);
    for (int k = 0; k < m && e == hipSuccess; ++k)
      e = Dspec[k].ensure((size_t)(rprod(r, k) * nprod(k + 1) * r[k]));
    if (e != hipSuccess) return hipfail(e, "mode buffers");
    const void *x = y;
    int x64 = 0;
    for (int k = 0; k < m; ++k) {
      const int64_t a = rprod(r, k), nk = n[k], b = nprod(k + 1);
      FiberIn in{};
      in.x = x;
      in.x64 = x64;
      in.a = a;
      in.n = nk;
      in.F = a * b;
      int nb = 0;
      tic();
      e = launch_fiber_project(in, wmat(k), 0, (int)r[k], FiberOut{Dspec[k].p, 1, a, r[k]},
                               specpart.p + poff[k], prec, stream, &nb);
      toc(k == 0 ? ST_K_TTM1 : ST_K_TTM, 4.0 * in.F * nk * r[k], 4.0 * in.F * (nk + r[k]));
      if (e == hipSuccess) e = launch_reduce_pairs(specpart.p + poff[k], nb, specsums.p + 2 * k,
                                                   stream);
      if (e != hipSuccess) return hipfail(e, "fiber projection + residual");
      x = Dspec[k].p;
      x64 = 1;
    }
    e = launch_gather3(hpin_dev, specsums.p, 2 * m, 0, nullptr, 0, 0, nullptr, 0, 0, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "residual norms");
    settle();
    rc = finish_pending();
    if (rc != ST_OK) return rc;
    ynorm2 = hpin[1];
    if (!std::isfinite(ynorm2)) return fail(ST_ENONFINITE, "slice is not finite");
    eps = tau * std::sqrt(ynorm2 / d);
    for (int k = 0; k < m; ++k) stt.e_norm_fast[k] = std::sqrt(std::max(hpin[2 * k], 0.0));
    for (k0 = 0; k0 < m; ++k0) {
      const double e2 = hpin[2 * k0];
      if (!std::isfinite(e2)) return fail(ST_ENONFINITE, "non-finite residual in mode %d", k0 + 1);
      const double en = std::sqrt(e2);
      // keep U_k only when the test passes clear of the guard band (R9); the
      // FP64 form decides on its own products
      if (fast ? en > (1.0 - guard_rel) * eps : en > eps) break;
      stt.e_norm[k0] = en;
      delta2 += e2;
    }
    if (fast && k0 < m) {
      // A slice mode grows or lies near its threshold: the decisions of this
      // slice and the new factor columns must not depend on reduced-precision
      // products, so every slice mode is redone from Y with FP64 products.
      k0 = 0;
      delta2 = 0.0;
      for (int k = 0; k < m; ++k) stt.e_norm[k] = 0.0;
      mp = Prec::FP64;
      exact_d = true;
      stt.refined_modes = 1;
      ++stt.guard_hits;
    } else if (k0 > 0) {
      Din = Dspec[k0 - 1].p;
      din64 = 1;
    }
  }
  for (int k = k0; k < m; ++k) {
    const int64_t a = rprod(rn, k);
    const int64_t nk = n[k];
    const int64_t b = nprod(k + 1);
    FiberIn in{};
    in.x = Din;
    in.x64 = din64;
    in.a = a;
    in.n = nk;
    in.F = a * b;
    double *Dout = D[dsel].p;
    const int tgroup = k == 0 ? ST_K_TTM1 : ST_K_TTM;
    // (this loop only runs with FP64 products: the FP64 form, or a refined slice)
    rc = project_resid(in, wmat(k), (int)r[k], FiberOut{Dout, 1, a, r[k]}, mp,
                       fast ? ST_K_REFINE : tgroup);
    if (rc != ST_OK) return rc;
    double e2 = hpin[0];
    if (k == 0) {
      ynorm2 = hpin[1];
      if (!std::isfinite(ynorm2)) return fail(ST_ENONFINITE, "slice is not finite");
      eps = tau * std::sqrt(ynorm2 / d);
    }
    if (!std::isfinite(e2)) return fail(ST_ENONFINITE, "non-finite residual in mode %d", k + 1);
    stt.e_norm[k] = std::sqrt(e2);
    if (std::sqrt(e2) <= eps) {  // Alg. 4: keep U_k, D*_k = P_k
      delta2 += e2;
      Din = Dout;
      din64 = 1;
      dsel ^= 1;
      continue;
    }
    // Alg. 4 growth: TruncatedSVD of E_(k) via its Gram (Alg. 1). E is
    // recomputed with FP64 products; the Gram's own products take the form's
    // precision, and a tail sum within the band of eps^2 is decided again on
    // the FP64 Gram.
    const GramPrec gp = prec == Prec::FP64 ? GramPrec::FP64
                        : (prec == Prec::BF16X3 ? GramPrec::BF16X3 : GramPrec::FP32);
    // (Dout holds P_k from FP64 products: this loop runs with mp = FP64)
    rc = gram_eig(in, wmat(k), (int)r[k], nk, gp, true, mp == Prec::FP64 ? Dout : nullptr);
    if (rc != ST_OK) return rc;
    int64_t rp;
    double tail;
    rank_rule(hpin, nk, eps, rp, tail, desc);
    if (tail_in_band(desc, eps, tail_band(gp))) {
      rc = gram_eig(in, wmat(k), (int)r[k], nk, GramPrec::FP64, true);
      if (rc != ST_OK) return rc;
      rank_rule(hpin, nk, eps, rp, tail, desc);
      ++stt.refined_gram;
      ++stt.guard_hits;
    }
    rp = std::min<int64_t>(rp, nk - r[k]);
    if (rp <= 0) {  // the Gram resolves nothing above the tolerance
      delta2 += e2;
      Din = Dout;
      din64 = 1;
      dsel ^= 1;
      continue;
    }
    tail = 0.0;
    for (int64_t i = rp; i < nk; ++i) tail += desc[i];
    delta2 += tail;
    rc = append_columns(k, r[k], rp);
    if (rc != ST_OK) return rc;
    rn[k] = r[k] + rp;
    stt.grew[k] = (int32_t)rp;
    // D*_k = D*_{k-1} x_k [U_k W_k]^T
    tic();
    e = launch_fiber_project(in, wmat(k), 0, (int)rn[k], FiberOut{Dout, 1, a, rn[k]}, nullptr,
                             mp, stream);
    toc(ST_K_TTM_EXT, 2.0 * in.F * nk * rn[k],
        (din64 ? 8.0 : 4.0) * in.F * nk + 8.0 * in.F * rn[k]);
    if (e != hipSuccess) return hipfail(e, "extended projection");
    Din = Dout;
    din64 = 1;
    dsel ^= 1;
  }
  const double ms_modes = ms_since(t0);

  // ---- streaming mode: Alg. 3 on d = vec(D*_{d-1}) ----
  const int64_t Rold = rprod(r, m), Rnew = rprod(rn, m);
  RowMap map{};
  map.nm = m;
  map.identity = 1;
  for (int k = 0; k < m; ++k) {
    map.r_old[k] = (int32_t)r[k];
    map.r_new[k] = (int32_t)rn[k];
    if (rn[k] != r[k]) map.identity = 0;
  }
  if (!din64) return fail(ST_EINVAL, "slice has no slice modes");
  const double *dvec = static_cast<const double *>(Din);  // (replaced by exact coordinates
                                                          // when the ISVD is refined)
  if (bsz > 1) {
    // the block form of Alg. 3 decides on FP64-product coordinates only
    if (!exact_d) {
      const double *dex = nullptr;
      rc = exact_coords(y, &dex);
      if (rc != ST_OK) return rc;
      dvec = dex;
      stt.refined_isvd = 1;
    }
    return stream_block(map, dvec, bsz, Rold, Rnew, eps, stt, rn, delta2, ynorm2, ms_modes, t0);
  }
  if (factored) {
    int growf = 0, v0next = v0cur;
    double q2f = 0.0;
    int64_t cf = 0;
    rc = stream_factored(map, dvec, Rold, Rnew, eps, stt, growf, q2f, cf, v0next, exact_d, y);
    if (rc != ST_OK) return rc;
    // ---- commit (the singular values follow through hS) ----
    snapshot();
    s_pending = cf;
    for (int k = 0; k < m; ++k) r[k] = rn[k];
    rd = cf;
    nd += 1;
    cur ^= 1;
    v0cur = v0next;
    xnorm2 += ynorm2;
    if (!growf) delta2 += q2f;
    disc += delta2;
    stt.ynorm = std::sqrt(ynorm2);
    stt.eps = eps;
    stt.delta2 = delta2;
    stt.ms_modes = ms_modes;
    stt.ms_total = ms_since(t0);
    stt.ms_isvd = stt.ms_total - ms_modes;
    qr_total += stt.qr_fired;
    stt.qr_total = qr_total;
    stats = stt;
    return ST_OK;
  }
  const int rdi = (int)rd;
  // Alg. 3's two Gram-Schmidt passes: p1 = V^T d by a coalesced GEMV (V read
  // through the row map), then one sweep forming e1 = d - V p1 with ||e1||^2 and
  // p2 = V^T e1; p = p1 + p2 and q^2 = ||e1||^2 - ||p2||^2
  const int nbg = gemv_t_blocks(Rnew);
  const int nbp = isvd_blocks(Rnew, rdi);
  e = colpart.ensure((size_t)(rdi + 1) * std::max(nbg, nbp));
  if (e == hipSuccess) e = q2part.ensure(nbp);
  if (e == hipSuccess) e = p1.ensure(rdi);
  if (e == hipSuccess) e = p2.ensure(rdi);
  if (e == hipSuccess) e = p.ensure(rdi);
  if (e == hipSuccess) e = e1buf.ensure((size_t)Rnew);
  if (e != hipSuccess) return hipfail(e, "isvd buffers");
  IsvdArgs ia{};
  ia.e1out = e1buf.p;  // e1 = d - V p1, kept for the second projection step
  ia.V = V[cur].p;
  ia.ldv = Rold;
  ia.r = rdi;
  ia.R = Rnew;
  ia.map = map;
  ia.d = dvec;
  ia.p1 = p1.p;
  ia.colpart = colpart.p;
  ia.q2part = q2part.p;
  tic();
  e = launch_gemv_t_mapped(V[cur].p, Rold, map, Rnew, rdi, dvec, colpart.p, nbg, stream);
  if (e == hipSuccess)
    e = launch_colsum(colpart.p, nbg, rdi, p1.p, nullptr, nullptr, nullptr, nullptr, stream);
  if (e == hipSuccess) e = launch_isvd_pass(2, ia, nbp, stream);
  if (e == hipSuccess)
    e = launch_colsum(colpart.p, nbp, rdi, p2.p, p1.p, p.p, q2part.p, sums.p, stream);
  // 4 R r flops (two products with V^T) + 2 R r (row dots); V (FP64) read twice, d twice
  toc(ST_K_ISVD, 6.0 * Rnew * rdi, 2.0 * 8.0 * Rold * rdi + 2.0 * 8.0 * Rnew);
  if (e == hipSuccess)
    e = launch_gather3(hpin_dev, sums.p, 1, 0, p.p, rdi, 3, p2.p, rdi, 3 + rdi, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "isvd projections");
  settle();
  // q^2 = ||e1 - V p2||^2 = ||e1||^2 - ||p2||^2 (V orthonormal; p2 ~ u ||d||)
  const double e1sq = hpin[0];
  double p2sq = 0.0, p2max = 0.0;
  for (int j = 0; j < rdi; ++j) {
    p2sq += hpin[3 + rdi + j] * hpin[3 + rdi + j];
    p2max = std::max(p2max, std::fabs(hpin[3 + rdi + j]));
  }
  double q2 = std::max(e1sq - p2sq, 0.0);
  double q = std::sqrt(q2);
  if (!std::isfinite(q)) return fail(ST_ENONFINITE, "non-finite ISVD residual");
  const double *pvec = p.p;    // p of Alg. 3 on the device
  const double *p2vec = p2.p;  // second projection: e = e1 - V p2 (the CGS2 order)
  std::vector<double> ph(hpin + 3, hpin + 3 + rdi);
  stt.q_fast = q;
  if (!exact_d && q > (1.0 - guard_rel) * eps) {
    // The slice may grow V (or lies near the threshold): q, p and the new
    // column must come from FP64 products. With d' = d + delta the exact
    // coordinates, p' = p + V^T delta and, since e = d - V p is orthogonal to
    // V, ||e'||^2 = q^2 + 2 (d.delta - p.V^T delta) + ||delta||^2
    // - ||V^T delta||^2: one sweep over V instead of both passes again.
    const double *dex = nullptr;
    rc = exact_coords(y, &dex);
    if (rc != ST_OK) return rc;
    const int nbd = 1024;
    e = dlt.ensure((size_t)Rnew);
    if (e == hipSuccess) e = pref.ensure(3 * (size_t)rdi + 2);
    if (e == hipSuccess) e = part.ensure(2 * (size_t)nbd);
    if (e != hipSuccess) return hipfail(e, "isvd refinement buffers");
    double *vtd = pref.p, *pnew = pref.p + rdi;
    tic();
    e = launch_delta(dex, dvec, Rnew, dlt.p, part.p, nbd, stream);
    if (e == hipSuccess) e = launch_reduce_pairs(part.p, nbd, sums.p + 16, stream);
    if (e == hipSuccess)
      e = launch_gemv_t_mapped(V[cur].p, Rold, map, Rnew, rdi, dlt.p, colpart.p, nbg, stream);
    if (e == hipSuccess && rdi > 0)
      e = launch_colsum(colpart.p, nbg, rdi, vtd, p.p, pnew, nullptr, nullptr, stream);
    // e1' = e1 + delta and p2' = p2 + V^T delta: the same two steps on d'
    double *p2new = pref.p + 2 * rdi;
    if (e == hipSuccess) e = launch_vadd(e1buf.p, dlt.p, Rnew, e1buf.p, stream);
    if (e == hipSuccess) e = launch_vadd(p2.p, vtd, rdi, p2new, stream);
    toc(ST_K_REFINE, 2.0 * Rnew * rdi + 5.0 * Rnew, 8.0 * Rold * rdi + 48.0 * Rnew);
    if (e == hipSuccess)
      e = launch_gather3(hpin_dev, sums.p + 16, 2, 0, vtd, rdi, 2, pnew, rdi, 2 + rdi, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "isvd refinement");
    settle();
    double pv = 0.0, vv = 0.0;
    for (int j = 0; j < rdi; ++j) {
      pv += ph[j] * hpin[2 + j];
      vv += hpin[2 + j] * hpin[2 + j];
    }
    q2 = std::max(q2 + 2.0 * (hpin[0] - pv) + hpin[1] - vv, 0.0);
    q = std::sqrt(q2);
    if (!std::isfinite(q)) return fail(ST_ENONFINITE, "non-finite ISVD residual");
    ph.assign(hpin + 2 + rdi, hpin + 2 + 2 * rdi);
    dvec = dex;
    pvec = pnew;
    p2vec = p2new;
    exact_d = true;
    stt.refined_isvd = 1;
    ++stt.guard_hits;
  }
  double pmax = 0.0;
  for (int j = 0; j < rdi; ++j) pmax = std::max(pmax, std::fabs(ph[j]));
  const double tol = 8.0 * 0x1p-53 * std::max({S_host.empty() ? 0.0 : S_host[0], pmax, q});
  const int grow = (q > eps && q > tol) ? 1 : 0;
  const int64_t c = rd + grow;
  stt.q = q;
  stt.isvd_ignored = grow ? 0 : 1;
  stt.orth_check = 0.0;
  stt.qr_fired = 0;
  (void)e1sq;
  (void)p2max;
  if (max_rank_d > 0 && c > max_rank_d)
    return fail(ST_ECAPACITY, "streaming rank %lld exceeds the cap", (long long)c);
  // q of S' and of v = e / q: on a growing slice the norm of e itself
  double qv = q;
  double *vte = nullptr, *eev = sums.p + 20;
  if (grow) {
    // Alg. 3's orthogonality check on the new direction, over all columns:
    // e = e1 - V p2, V^T e and ||e||^2 in one more sweep over V
    e = qvte.ensure((size_t)rdi + 1);
    if (e != hipSuccess) return hipfail(e, "orthogonality check buffers");
    vte = qvte.p;
    IsvdArgs ic = ia;
    ic.d = e1buf.p;
    ic.p1 = p2vec;
    ic.e1out = nullptr;
    tic();
    e = launch_isvd_pass(2, ic, nbp, stream);
    if (e == hipSuccess)
      e = launch_colsum(colpart.p, nbp, rdi, vte, nullptr, nullptr, q2part.p, eev, stream);
    toc(ST_K_ORTH, 4.0 * Rnew * rdi, 8.0 * Rold * rdi + 8.0 * Rnew);
    if (e == hipSuccess)
      e = launch_gather3(hpin_dev, eev, 1, 0, vte, rdi, 1, nullptr, 0, 0, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "orthogonality check");
    settle();
    const double ee = hpin[0];
    if (!(ee > 0.0) || !std::isfinite(ee)) return fail(ST_ENONFINITE, "non-finite ISVD residual");
    double vmax = 0.0;
    for (int j = 0; j < rdi; ++j) vmax = std::max(vmax, std::fabs(hpin[1 + j]));
    qv = std::sqrt(ee);
    stt.orth_check = vmax / qv;
    stt.qr_fired = stt.orth_check > orth_tol ? 1 : 0;
  }

  const int nxt = cur ^ 1;
  const int64_t nn = rd + 1;
  const int64_t kv = rd + grow;
  const int64_t ldwv = round_up(kv, 4), ldwc = round_up(rd + 1, 4);
  e = ensure_secular(nn);
  if (e == hipSuccess) e = U2.ensure((size_t)nn * c);
  if (e == hipSuccess) e = V2.ensure((size_t)nn * c);
  if (e == hipSuccess) e = S[nxt].ensure(c);
  if (e == hipSuccess) e = Wv.ensure((size_t)c * ldwv);
  if (e == hipSuccess) e = Wc.ensure((size_t)c * ldwc);
  if (e == hipSuccess) e = V[nxt].ensure((size_t)(Rnew * c));
  if (e == hipSuccess) e = C[nxt].ensure((size_t)(Rnew * c));
  int64_t ldn = ud_ld[nxt];
  if (e == hipSuccess && (ldn < nd + 1 || Ud[nxt].cap < (size_t)ldn * c)) {
    ldn = std::max<int64_t>(ud_ld[cur], round_up(nd + 1, 64));
    if (ldn < nd + 1 + 0) ldn = round_up(2 * (nd + 1), 64);
    e = Ud[nxt].ensure((size_t)ldn * c);
  }
  if (e != hipSuccess) return hipfail(e, "streaming buffers");
  ud_ld[nxt] = ldn;

  if (stt.qr_fired) {
    // [V v] = Q R through the Gram of [V v]; V^T V over the old layout (padded
    // rows are zero)
    tic();
    e = qrg.ensure((size_t)rdi * rdi);
    if (e == hipSuccess) e = chunk_gram(V[cur].p, Rold, rdi, qrg.p);
    if (e != hipSuccess) return hipfail(e, "V^T V");
    rc = qr_fix(qrg.p, rdi, vte, eev, pvec, tol, nxt);
    toc(ST_K_ORTH, 2.0 * Rold * rdi * rdi + 40.0 * (double)nn * nn * nn, 8.0 * Rold * rdi);
    if (rc != ST_OK) return rc;
    settle();
  } else {
    tic();
    e = launch_secular_svd(secdata(rdi), S[cur].p, pvec, qv, nullptr, grow, tol, (int)c, U2.p,
                           V2.p, S[nxt].p, stream);
    toc(ST_K_SVD, 60.0 * (double)nn * nn, 8.0 * 4.0 * nn * c);
    if (e != hipSuccess) return hipfail(e, "small SVD");
  }
  e = launch_build_rot_w(U2.p, V2.p, rdi, (int)c, (int)kv, grow ? 1.0 / qv : 0.0, Wv.p, ldwv,
                         Wc.p, ldwc, stream);
  if (e != hipSuccess) return hipfail(e, "rotation matrices");
  // V~ = [V v] V''  (mode-d TTM of V with the padded rows mapped)
  FiberIn vin{};
  vin.x = V[cur].p;
  vin.x64 = 1;
  vin.a = Rold;
  vin.n = rd;
  vin.F = Rnew;
  vin.mapped = 1;
  vin.map = map;
  vin.extra = grow ? e1buf.p : nullptr;
  tic();
  // V~ = [V v] V'' with v = e / q, e = e1 - V p2 formed per row in FP64
  e = launch_rot64(vin, Wv.p, 1, ldwv, 0, (int)c, FiberOut{V[nxt].p, 1, Rnew, c}, grow ? 2 : 0,
                   p2vec, stream);
  // read V (R_old x r_d, FP64) and d, write V~ (R_new x c, FP64): 2 R_new K c flops
  toc(ST_K_ROT_V, 2.0 * Rnew * (double)kv * c + (grow ? 2.0 * Rnew * rd : 0.0),
      8.0 * ((double)Rold * rd + (grow ? Rnew : 0) + (double)Rnew * c));
  if (e != hipSuccess) return hipfail(e, "V rotation");
  // C~_(d) = U~_d(1:n_d,:)^T U_d C_(d) + U~_d(n_d+1,:)^T d^T = U''^T [C_(d); d^T]
  FiberIn cin = vin;
  cin.x = C[cur].p;
  cin.x64 = 0;
  cin.extra = dvec;
  tic();
  // the FP32 and bf16x3 forms take the FP32 MFMA with FP64 sums across K blocks
  // (the core never enters a rank test); the FP64 form keeps exact products
  e = launch_rot64(cin, Wc.p, 0, ldwc, 0, (int)c, FiberOut{C[nxt].p, 0, Rnew, c}, 1, nullptr,
                   stream, prec == Prec::FP64 ? 0 : 1);
  // read C (FP32) and d (FP64), write C~ (FP32)
  toc(ST_K_ROT_C, 2.0 * Rnew * (double)(rd + 1) * c,
      4.0 * ((double)Rold * rd + (double)Rnew * c) + 8.0 * Rnew);
  if (e != hipSuccess) return hipfail(e, "core rotation");
  tic();
  e = launch_ud_update(Ud[cur].p, ud_ld[cur], nd, rdi, U2.p, (int)c, Ud[nxt].p, ldn, stream);
  toc(ST_K_UD, 2.0 * nd * (double)rd * c, 8.0 * ((double)nd * rd + (nd + 1.0) * c));
  if (e != hipSuccess) return hipfail(e, "streaming factor update");
  // The new singular values go to pinned memory without a synchronisation: the
  // device work of this update may still run when the call returns, and the
  // next call that needs them (the next update's first synchronisation, st_sv)
  // takes them (finish_pending).
  e = ensure_hS((size_t)c);
  if (e == hipSuccess)
    e = launch_gather3(hS_dev, S[nxt].p, (int)c, 0, nullptr, 0, 0, nullptr, 0, 0, stream);
  if (e != hipSuccess) return hipfail(e, "streaming update");

  // ---- commit ----
  snapshot();
  s_pending = c;
  for (int k = 0; k < m; ++k) r[k] = rn[k];
  rd = c;
  nd += 1;
  cur = nxt;
  xnorm2 += ynorm2;
  if (!grow) delta2 += q2;
  disc += delta2;
  stt.ynorm = std::sqrt(ynorm2);
  stt.eps = eps;
  stt.delta2 = delta2;
  stt.ms_modes = ms_modes;
  stt.ms_total = ms_since(t0);
  stt.ms_isvd = stt.ms_total - ms_modes;
  qr_total += stt.qr_fired;
  stt.qr_total = qr_total;
  stats = stt;
  return ST_OK;
}

// ---------------------------------------------------------------------------
// Alg. 3 in the factored form V = V0 M, with G0 = V0^T V0 kept alongside.
// V0 is brought to the row layout of the new slice-mode ranks (only when one of
// them grew). One sweep over V0 gives t1 = V0^T d and ||d||^2; the rest of the
// two Gram-Schmidt passes is r x r work through G0 (isvd_gram_kernel). When q
// lands within the rounding bound of that formula of eps, the second pass is
// redone exactly by a sweep over V0. A growing slice forms e1 = d - V0 w1 and
// then e = e1 - V0 w2 in two sweeps (each with V0^T of its result), checks the
// orthogonality of v = e / ||e|| to V (Alg. 3, with the QR fix when it fails),
// appends v as a new column of V0 and extends G0; in every case
// M~ = blockdiag(M, 1) V'' and U_d, S are updated as in the literal form. On
// success hpin[0 .. c) holds the new singular values.
// ---------------------------------------------------------------------------
int st_handle::stream_factored(const RowMap &map, const double *dvec, int64_t Rold, int64_t Rnew,
                               double eps, st_slice_stats &stt, int &grow, double &q2,
                               int64_t &c, int &v0next, bool exact_d, const float *y) {
  const int rdi = (int)rd;
  const int nxt = cur ^ 1;
  hipError_t e = hipSuccess;
  int w0 = v0cur;
  const size_t need = (size_t)Rnew * (size_t)(rd + 1);
  if (!map.identity || V[v0cur].cap < need) {
    // relayout (or grow the column capacity) into the other buffer; the
    // committed V0 stays untouched until the commit. Zero rows leave G0 as is.
    w0 = v0cur ^ 1;
    e = V[w0].ensure(std::max(need, (size_t)Rnew * (size_t)(rd + 16)));
    if (e == hipSuccess) {
      if (!map.identity)
        e = launch_remap_rows(V[v0cur].p, Rold, map, Rnew, rdi, V[w0].p, stream);
      else
        e = hipMemcpyAsync(V[w0].p, V[v0cur].p, (size_t)Rold * rd * sizeof(double),
                           hipMemcpyDeviceToDevice, stream);
    }
    if (e != hipSuccess) return hipfail(e, "V0 relayout");
  }
  double *V0 = V[w0].p;
  const double *M = Mf[cur].p;
  const double *G0 = Gf[cur].p;
  const int nbg = gemv_t_blocks(Rnew);
  const int nbp = isvd_blocks(Rnew, rdi);
  e = colpart.ensure((size_t)(rdi + 1) * std::max(nbg, nbp));
  if (e == hipSuccess) e = q2part.ensure(nbp);
  if (e == hipSuccess) e = p1.ensure(rdi);
  if (e == hipSuccess) e = p2.ensure(rdi);
  if (e == hipSuccess) e = p.ensure(rdi);
  if (e == hipSuccess) e = tvec.ensure(3 * (size_t)rdi + 8);
  if (e == hipSuccess) e = wvec.ensure(4 * (size_t)rdi + 8);
  if (e != hipSuccess) return hipfail(e, "isvd buffers");
  double *t1 = tvec.p, *t2 = tvec.p + rdi, *ge = tvec.p + 2 * rdi;
  double *w1 = wvec.p, *w2 = wvec.p + rdi, *ws = wvec.p + 2 * rdi, *gv = wvec.p + 3 * rdi;
  double *sc = sums.p + 8;  // [0] ||e1||^2, [1] q^2, [2] cancelled magnitude
  double *dd = sums.p + 12, *ee = sums.p + 13;
  double e1sq = 0.0, q = 0.0;
  for (int attempt = 0;; ++attempt) {
    const int igroup = attempt ? ST_K_REFINE : ST_K_ISVD;
    tic();
    e = launch_gemv_t(V0, Rnew, rdi, dvec, colpart.p, nbg, stream);
    if (e == hipSuccess)
      e = launch_colsum(colpart.p, nbg, rdi, t1, nullptr, nullptr, colpart.p + (size_t)rdi * nbg,
                        dd, stream);
    if (e == hipSuccess)
      e = launch_isvd_gram(M, G0, rdi, t1, dd, 0, p1.p, w1, t2, p2.p, w2, p.p, ws, sc, gv, nullptr,
                           stream);
    // V0 and d read once (FP64); r x r products
    toc(igroup, 2.0 * Rnew * rdi + 10.0 * (double)rdi * rdi, 8.0 * Rnew * (rdi + 1.0));
    if (e == hipSuccess)
      e = launch_gather3(hpin_dev, sc, 3, 0, p.p, rdi, 3, p2.p, rdi, 3 + rdi, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "isvd projections");
    settle();
    e1sq = hpin[0];
    q2 = std::max(hpin[1], 0.0);
    q = std::sqrt(q2);
    if (attempt == 0) stt.q_fast = q;
    // rounding bound of the cancelled sum forming q^2, as a bound on q
    const double dq2 = 64.0 * 0x1p-53 * hpin[2];
    const double dq = q > 0.0 ? dq2 / (2.0 * q) : std::sqrt(dq2);
    if (!std::isfinite(q)) return fail(ST_ENONFINITE, "non-finite ISVD residual");
    if (std::fabs(q - eps) <= 4.0 * dq) {
      // too close to call from G0: redo the second pass exactly over V0
      RowMap ident{};
      ident.nm = m;
      ident.identity = 1;
      IsvdArgs ia{};
      ia.V = V0;
      ia.ldv = Rnew;
      ia.r = rdi;
      ia.R = Rnew;
      ia.map = ident;
      ia.d = dvec;
      ia.p1 = w1;
      ia.colpart = colpart.p;
      ia.q2part = q2part.p;
      tic();
      e = launch_isvd_pass(2, ia, nbp, stream);
      if (e == hipSuccess)
        e = launch_colsum(colpart.p, nbp, rdi, t2, nullptr, nullptr, q2part.p, sc, stream);
      if (e == hipSuccess)
        e = launch_isvd_gram(M, G0, rdi, t1, dd, 1, p1.p, w1, t2, p2.p, w2, p.p, ws, sc, gv,
                             nullptr, stream);
      toc(igroup, 4.0 * Rnew * rdi, 8.0 * Rnew * (rdi + 1.0));
      if (e == hipSuccess)
        e = launch_gather3(hpin_dev, sc, 3, 0, p.p, rdi, 3, p2.p, rdi, 3 + rdi, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hipfail(e, "exact second pass");
      settle();
      e1sq = hpin[0];
      q2 = std::max(hpin[1], 0.0);
      q = std::sqrt(q2);
      ++stt.guard_hits;
    }
    if (!exact_d && q > (1.0 - guard_rel) * eps) {
      // The slice may grow V (or lies near the threshold): redo the projection
      // from FP64-product coordinates, so the test and the appended column of V0
      // carry no reduced-precision rounding.
      const double *dex = nullptr;
      const int rc2 = exact_coords(y, &dex);
      if (rc2 != ST_OK) return rc2;
      dvec = dex;
      exact_d = true;
      stt.refined_isvd = 1;
      ++stt.guard_hits;
      continue;
    }
    break;
  }
  double pmax = 0.0, p2max = 0.0;
  for (int j = 0; j < rdi; ++j) {
    pmax = std::max(pmax, std::fabs(hpin[3 + j]));
    p2max = std::max(p2max, std::fabs(hpin[3 + rdi + j]));
  }
  const double tol = 8.0 * 0x1p-53 * std::max({S_host.empty() ? 0.0 : S_host[0], pmax, q});
  grow = (q > eps && q > tol) ? 1 : 0;
  c = rd + grow;
  stt.q = q;
  stt.isvd_ignored = grow ? 0 : 1;
  stt.orth_check = 0.0;
  stt.qr_fired = 0;
  (void)e1sq;
  (void)p2max;
  if (max_rank_d > 0 && c > max_rank_d)
    return fail(ST_ECAPACITY, "streaming rank %lld exceeds the cap", (long long)c);

  const int64_t nn = rd + 1;
  e = ensure_secular(nn);
  if (e == hipSuccess) e = U2.ensure((size_t)nn * c);
  if (e == hipSuccess) e = V2.ensure((size_t)nn * c);
  if (e == hipSuccess) e = S[nxt].ensure(c);
  if (e == hipSuccess) e = Mf[nxt].ensure((size_t)(c * c));
  if (e == hipSuccess) e = Gf[nxt].ensure((size_t)(c * c));
  int64_t ldn = ud_ld[nxt];
  if (e == hipSuccess && (ldn < nd + 1 || Ud[nxt].cap < (size_t)ldn * c)) {
    ldn = std::max<int64_t>(ud_ld[cur], round_up(nd + 1, 64));
    e = Ud[nxt].ensure((size_t)ldn * c);
  }
  if (e != hipSuccess) return hipfail(e, "streaming buffers");
  ud_ld[nxt] = ldn;
  tic();
  if (grow) {
    // The new direction in the order of the two Gram-Schmidt passes, so that
    // the rounding of the first step (about u ||d|| per row) is projected out by
    // the second: e1 = d - V0 w1 into column r_d of V0 with V0^T e1 and ||e1||^2,
    // the r x r part of the second pass on that exact V0^T e1 (p2, w2, p), then
    // e = e1 - V0 w2 in place with V0^T e and ||e||^2. S' takes ||e|| itself as
    // its q entry and v = e / ||e|| is appended, so that [V, v] stays
    // orthonormal: the q of the G0 formula decided the growth, but it carries
    // the rounding of a difference of terms of size ||d||^2 and is not accurate
    // enough to normalise v (its relative error grows as (||d|| / q)^2).
    RowMap ident{};
    ident.nm = m;
    ident.identity = 1;
    IsvdArgs ia{};
    ia.V = V0;
    ia.ldv = Rnew;
    ia.r = rdi;
    ia.R = Rnew;
    ia.map = ident;
    ia.d = dvec;
    ia.p1 = w1;
    ia.colpart = colpart.p;
    ia.q2part = q2part.p;
    ia.e1out = V0 + Rnew * rd;
    e = launch_isvd_pass(2, ia, nbp, stream);
    if (e == hipSuccess)
      e = launch_colsum(colpart.p, nbp, rdi, t2, nullptr, nullptr, q2part.p, sc, stream);
    if (e == hipSuccess)
      e = launch_isvd_gram(M, G0, rdi, t1, dd, 1, p1.p, w1, t2, p2.p, w2, p.p, ws, sc, gv,
                           nullptr, stream);
    ia.d = V0 + Rnew * rd;  // e1, overwritten row by row with e
    ia.p1 = w2;
    if (e == hipSuccess) e = launch_isvd_pass(2, ia, nbp, stream);
    if (e == hipSuccess)
      e = launch_colsum(colpart.p, nbp, rdi, ge, nullptr, nullptr, q2part.p, ee, stream);
    if (e == hipSuccess) e = launch_scale_rsqrt(V0 + Rnew * rd, Rnew, ee, stream);
  }
  // the appended column: V0 read twice, d read, the column written twice
  toc(ST_K_ROT_V, grow ? 8.0 * Rnew * rd : 0.0,
      grow ? 8.0 * (2.0 * Rnew * rd + 5.0 * Rnew) : 0.0);
  if (e != hipSuccess) return hipfail(e, "V0 append");
  if (grow) {
    // Alg. 3's orthogonality check on v = e / ||e|| over all columns of
    // V = V0 M: V^T e = M^T (V0^T e), r x r work on the sweep's V0^T e
    e = qvte.ensure((size_t)rdi + 1);
    if (e != hipSuccess) return hipfail(e, "orthogonality check buffers");
    tic();
    e = launch_small_gemv(M, rdi, ge, 1, qvte.p, nullptr, nullptr, stream);
    toc(ST_K_ORTH, 2.0 * (double)rdi * rdi, 8.0 * (double)rdi * rdi);
    if (e == hipSuccess)
      e = launch_gather3(hpin_dev, ee, 1, 0, qvte.p, rdi, 1, nullptr, 0, 0, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "orthogonality check");
    settle();
    const double eeh = hpin[0];
    if (!(eeh > 0.0) || !std::isfinite(eeh))
      return fail(ST_ENONFINITE, "non-finite ISVD residual");
    double vmax = 0.0;
    for (int j = 0; j < rdi; ++j) vmax = std::max(vmax, std::fabs(hpin[1 + j]));
    stt.orth_check = vmax / std::sqrt(eeh);
    stt.qr_fired = stt.orth_check > orth_tol ? 1 : 0;
  }
  if (stt.qr_fired) {
    // QR fix: V^T V = M^T G0 M (r x r products)
    tic();
    e = qrg.ensure(2 * (size_t)rdi * rdi);
    if (e == hipSuccess)
      e = launch_small_gemm(0, G0, rdi, M, rdi, qrg.p + (size_t)rdi * rdi, rdi, rdi, rdi, rdi,
                            stream);
    if (e == hipSuccess)
      e = launch_small_gemm(1, M, rdi, qrg.p + (size_t)rdi * rdi, rdi, qrg.p, rdi, rdi, rdi, rdi,
                            stream);
    if (e != hipSuccess) return hipfail(e, "V^T V");
    const int rc = qr_fix(qrg.p, rdi, qvte.p, ee, p.p, tol, nxt);
    toc(ST_K_ORTH, 4.0 * (double)rdi * rdi * rdi + 40.0 * (double)nn * nn * nn,
        8.0 * 3.0 * rdi * rdi);
    if (rc != ST_OK) return rc;
    settle();
  }
  // S' (unless the QR fix took its SVD), then M~ = blockdiag(M, 1) V'' and G0
  tic();
  if (!stt.qr_fired)
    e = launch_secular_svd(secdata(rdi), S[cur].p, p.p, q, grow ? ee : nullptr, grow, tol, (int)c,
                           U2.p, V2.p, S[nxt].p, stream);
  if (e == hipSuccess) e = launch_g0_update(G0, rdi, ge, ee, grow, Gf[nxt].p, stream);
  if (e == hipSuccess) e = launch_m_update(M, rdi, V2.p, (int)c, grow, Mf[nxt].p, stream);
  toc(ST_K_SVD, 60.0 * (double)nn * nn + 2.0 * (double)c * c * rd,
      8.0 * 4.0 * nn * c + 16.0 * (double)c * c);
  if (e != hipSuccess) return hipfail(e, "small SVD / M update");
  tic();
  e = launch_ud_update(Ud[cur].p, ud_ld[cur], nd, rdi, U2.p, (int)c, Ud[nxt].p, ldn, stream);
  toc(ST_K_UD, 2.0 * nd * (double)rd * c, 8.0 * ((double)nd * rd + (nd + 1.0) * c));
  if (e != hipSuccess) return hipfail(e, "streaming factor update");
  // published without a synchronisation, as in the literal form
  e = ensure_hS((size_t)c);
  if (e == hipSuccess)
    e = launch_gather3(hS_dev, S[nxt].p, (int)c, 0, nullptr, 0, 0, nullptr, 0, 0, stream);
  if (e != hipSuccess) return hipfail(e, "streaming update");
  v0next = w0;
  return ST_OK;
}

// G0 = V0^T V0 at initialisation: library GEMMs over row chunks into separate
// partial Grams, summed in a fixed order. One GEMM over all R rows would chain
// R products per entry; the factored ISVD test takes differences of terms of
// size ||d||^2 through G0, so its rounding must stay at the level of the other
// blocked sums over R rows (t1 = V0^T d, ||d||^2).
hipError_t st_handle::init_g0(int64_t R, int rk) { return chunk_gram(V[cur].p, R, rk, Gf[cur].p); }

// out (r x r) = X^T X for a column-major R x r X (ld R): library GEMMs over row
// chunks into separate partial Grams (in tmp64), summed in a fixed order.
hipError_t st_handle::chunk_gram(const double *X, int64_t R, int r, double *out) {
  const size_t rr = (size_t)r * r;
  if (rr == 0) return hipSuccess;
  const int64_t max_parts = std::max<int64_t>(1, std::min<int64_t>(1024, (8 << 20) / (int64_t)rr));
  const int64_t ch = std::max<int64_t>(2048, (R + max_parts - 1) / max_parts);
  const int64_t nfull = R / ch, tail = R - nfull * ch;
  const int64_t nb = nfull + (tail > 0 ? 1 : 0);
  if (nb == 0) return hipErrorInvalidValue;
  hipError_t e = tmp64.ensure((size_t)nb * rr);
  if (e != hipSuccess) return e;
  const double one = 1.0, zero = 0.0;
  rocblas_status bs = rocblas_status_success;
  if (nfull > 0)
    bs = rocblas_dgemm_strided_batched(
        rb, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)r, (rocblas_int)r,
        (rocblas_int)ch, &one, X, (rocblas_int)R, (rocblas_stride)ch, X, (rocblas_int)R,
        (rocblas_stride)ch, &zero, tmp64.p, (rocblas_int)r, (rocblas_stride)rr,
        (rocblas_int)nfull);
  if (bs == rocblas_status_success && tail > 0)
    bs = rocblas_dgemm(rb, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)r,
                       (rocblas_int)r, (rocblas_int)tail, &one, X + nfull * ch, (rocblas_int)R,
                       X + nfull * ch, (rocblas_int)R, &zero, tmp64.p + (size_t)nfull * rr,
                       (rocblas_int)r);
  if (bs != rocblas_status_success) return hipErrorUnknown;
  return launch_batch_sum(tmp64.p, (int)nb, (int64_t)rr, out, stream);
}

// The QR fix of Alg. 3, taken when the orthogonality check on the new v fires:
// [V v] = Q R and S' -> S' R^T (k_dense.hip). Gtop = V^T V (r x r), vte = V^T e,
// ee = ||e||^2 (v = e / ||e||) and pv = p are on the device; tol is the secular
// solve's deflation tolerance. Writes U'' (U2), V'' (V2, so that V~ = [V v] V''
// as without the fix) and S~ (S[nxt], descending); c = n = r + 1. The SVD of
// S' R^T starts from the secular SVD of S' = U_S diag(S_S) V_S^T: S' R^T =
// U_S A^T with A = R V_S diag(S_S), whose columns are orthogonal up to the
// deviation the check measured, so the one-sided Jacobi on A (A J = U_A
// diag(s')) ends in a sweep or two; U'' = U_S J and V'' = R^{-1} U_A =
// V_S diag(S_S) J diag(s')^{-1}. Past kQrOrderMax columns the dense Jacobi SVD
// of S' R^T and V'' = R^{-1} V_B by back substitution.
int st_handle::qr_fix(const double *Gtop, int rdi, const double *vte, const double *ee,
                      const double *pv, double tol, int nxt) {
  const int n = rdi + 1;
  const size_t nn2 = (size_t)n * n;
  hipError_t e = qrw.ensure(7 * nn2 + 2 * (size_t)n);
  if (e == hipSuccess) e = qstat.ensure(2);
  if (e != hipSuccess) return hipfail(e, "QR fix buffers");
  double *G = qrw.p, *A = G + nn2, *W = A + nn2, *Us = W + nn2, *Vs = Us + nn2, *Jp = Vs + nn2,
         *JpS = Jp + nn2, *Ss = JpS + nn2, *sig = Ss + n;
  e = launch_qr_gram_fill(Gtop, rdi, vte, ee, G, stream);
  if (e == hipSuccess) e = launch_chol_upper(G, n, qstat.p, stream);
  if (n <= kQrOrderMax) {
    if (e == hipSuccess)
      e = launch_secular_svd(secdata(rdi), S[cur].p, pv, 0.0, ee, 1, tol, n, Us, Vs, Ss, stream);
    if (e == hipSuccess) e = launch_form_rvs(G, n, Vs, n, Ss, A, stream);
    if (e == hipSuccess) e = launch_jacobi_svd(A, n, W, 60, qstat.p, stream);
    if (e == hipSuccess) e = launch_qr_order(A, W, n, Ss, S[nxt].p, Jp, JpS, stream);
    if (e == hipSuccess) e = launch_small_gemm(0, Us, n, Jp, n, U2.p, n, n, n, n, stream);
    if (e == hipSuccess) e = launch_small_gemm(0, Vs, n, JpS, n, V2.p, n, n, n, n, stream);
  } else {
    if (e == hipSuccess) e = launch_arrow_rt(S[cur].p, pv, ee, G, rdi, A, stream);
    if (e == hipSuccess) e = launch_jacobi_svd(A, n, W, 60, qstat.p, stream);
    if (e == hipSuccess)
      e = launch_jacobi_finish(A, W, G, n, U2.p, V2.p, S[nxt].p, sig, stream);
  }
  int st[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(st, qstat.p, sizeof(st), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "QR fix");
  if (st[0] == 1) return fail(ST_ESOLVER, "QR fix: the Gram of [V v] is not positive definite");
  if (st[0] == 2) return fail(ST_ESOLVER, "QR fix: Jacobi SVD did not converge");
  return ST_OK;
}

// out (p x q) = X^T Y for column-major X (R x p, ld ldx) and Y (R x q, ld ldy):
// library GEMMs over row chunks into separate partials, summed in a fixed order.
hipError_t st_handle::chunk_tn(const double *X, int64_t ldx, const double *Y, int64_t ldy,
                               int64_t R, int p_, int q_, double *out) {
  const size_t pq = (size_t)p_ * q_;
  if (pq == 0) return hipSuccess;
  const int64_t max_parts = std::max<int64_t>(1, std::min<int64_t>(1024, (8 << 20) / (int64_t)pq));
  const int64_t ch = std::max<int64_t>(2048, (R + max_parts - 1) / max_parts);
  const int64_t nfull = R / ch, tail = R - nfull * ch;
  const int64_t nb = nfull + (tail > 0 ? 1 : 0);
  if (nb == 0) return hipErrorInvalidValue;
  hipError_t e = tmp64.ensure((size_t)nb * pq);
  if (e != hipSuccess) return e;
  const double one = 1.0, zero = 0.0;
  rocblas_status bs = rocblas_status_success;
  if (nfull > 0)
    bs = rocblas_dgemm_strided_batched(
        rb, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)p_, (rocblas_int)q_,
        (rocblas_int)ch, &one, X, (rocblas_int)ldx, (rocblas_stride)ch, Y, (rocblas_int)ldy,
        (rocblas_stride)ch, &zero, tmp64.p, (rocblas_int)p_, (rocblas_stride)pq,
        (rocblas_int)nfull);
  if (bs == rocblas_status_success && tail > 0)
    bs = rocblas_dgemm(rb, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)p_,
                       (rocblas_int)q_, (rocblas_int)tail, &one, X + nfull * ch, (rocblas_int)ldx,
                       Y + nfull * ch, (rocblas_int)ldy, &zero, tmp64.p + (size_t)nfull * pq,
                       (rocblas_int)p_);
  if (bs != rocblas_status_success) return hipErrorUnknown;
  return launch_batch_sum(tmp64.p, (int)nb, (int64_t)pq, out, stream);
}

// ---------------------------------------------------------------------------
// Alg. 3 for a block of b slices (the paper's Sec. 6 future work), literal core.
// Dm (R_new x b, FP64) holds the slices' core coordinates. Both Gram-Schmidt
// passes run on all b columns (P1 = V^T Dm, E = Dm - V P1, P2 = V^T E,
// E -= V P2); the residual block's kept directions follow the TruncatedSVD of
// Alg. 1 on E (eigenpairs of E^T E, tail rule against eps^2); Q = E W_l L_l^-1/2
// extends V; the middle matrix [[diag S, 0], [P^T, W_l L_l^1/2]] is dense, so its
// SVD is one-sided Jacobi (k_dense.hip), after the QR fix of the orthogonality
// check when [V Q] is not orthonormal to eps_m. Then V~ = [V Q] V'',
// C~ = [C, Dm] U'' and U~_d = blockdiag(U_d, I_b) U''; commits like the
// single-slice form.
// ---------------------------------------------------------------------------
// SVD of the block middle matrix K (rows 0..rd+b-1, columns 0..c-1 of the
// n2 x n2 array, ld n2) as b row appends to [diag(S), 0]: each appended row,
// rotated into the current right singular vectors (z = VK^T k_j), makes a
// diagonal matrix plus one row whose SVD is the secular solve of the
// single-slice update with no new column; VK and UK take its factors
// (VK <- VK V'', UK <- [[UK, 0], [0, 1]] U''). The l zero columns of [diag(S), 0]
// are poles at zero, deflated while their weights vanish. Writes U'' and V''
// into Uo ((rd + b) x c) and Vo (c x c), both ld n2, and So (c).
hipError_t st_handle::block_rows_svd(const double *K, int n2, int rdi, int bi, int c, double tol,
                                     double *Uo, double *Vo, double *So) {
  const int ldv = c + 1, ldu = c + bi;
  const size_t nv = (size_t)ldv * c, nu = (size_t)ldu * c;
  hipError_t e = bsec.ensure(4 * nv + 2 * nu + 3 * (size_t)c);
  if (e == hipSuccess) e = ensure_secular(c + 1);
  if (e != hipSuccess) return e;
  double *VK[2] = {bsec.p, bsec.p + nv};
  double *U2s = bsec.p + 2 * nv, *V2s = bsec.p + 3 * nv;
  double *UK[2] = {bsec.p + 4 * nv, bsec.p + 4 * nv + nu};
  double *sg[2] = {bsec.p + 4 * nv + 2 * nu, bsec.p + 4 * nv + 2 * nu + c};
  double *z = sg[1] + c;
  e = launch_block_rows_init(S[cur].p, rdi, c, VK[0], ldv, UK[0], ldu, sg[0], stream);
  int k = 0;
  for (int j = 0; j < bi && e == hipSuccess; ++j) {
    e = launch_block_row_z(VK[k], ldv, c, K, n2, rdi + j, z, stream);
    if (e == hipSuccess)
      e = launch_secular_svd(secdata(c), sg[k], z, 0.0, nullptr, 0, tol, c, U2s, V2s, sg[k ^ 1],
                             stream);
    // VK (c x c) <- VK V''(0:c, :); UK ((c + j) x c) <- [UK U''(0:c, :); U''(c, :)]
    if (e == hipSuccess) e = launch_ud_update(VK[k], ldv, c, c, V2s, c, VK[k ^ 1], ldv, stream);
    if (e == hipSuccess)
      e = launch_ud_update(UK[k], ldu, c + j, c, U2s, c, UK[k ^ 1], ldu, stream);
    k ^= 1;
  }
  if (e == hipSuccess)
    e = launch_block_rows_finish(VK[k], ldv, UK[k], ldu, sg[k], rdi, bi, c, Vo, Uo, So, stream);
  return e;
}

int st_handle::stream_block(const RowMap &map, const double *Dm, int64_t b, int64_t Rold,
                            int64_t Rnew, double eps, st_slice_stats &stt, const int64_t *rn,
                            double delta2, double ynorm2, double ms_modes,
                            clk::time_point t0) {
  const int rdi = (int)rd, bi = (int)b;
  const int n2 = rdi + bi;  // rows of the middle matrix (and its padded order)
  const int nxt = cur ^ 1;
  const size_t nn2 = (size_t)n2 * n2;
  hipError_t e = hipSuccess;
  tic();
  // V at the new row layout (the padded rows are zero). In the factored form
  // this is V0 (V = V0 M), relaid into the other V buffer, with room for the b
  // columns a block may append, whenever the committed one cannot take them in
  // place (the committed V0 is only ever written past its r_d columns).
  const double *Vn = V[cur].p;
  int w0 = v0cur;
  double *V0n = nullptr;
  if (factored) {
    const size_t need = (size_t)Rnew * (size_t)(rd + b);
    if (!map.identity || V[v0cur].cap < need) {
      w0 = v0cur ^ 1;
      e = V[w0].ensure(std::max(need, (size_t)Rnew * (size_t)(rd + 16)));
      if (e == hipSuccess) {
        if (!map.identity)
          e = launch_remap_rows(V[v0cur].p, Rold, map, Rnew, rdi, V[w0].p, stream);
        else
          e = hipMemcpyAsync(V[w0].p, V[v0cur].p, (size_t)Rold * rd * sizeof(double),
                             hipMemcpyDeviceToDevice, stream);
      }
    }
    V0n = V[w0].p;
    Vn = V0n;
  } else if (!map.identity) {
    e = bV.ensure((size_t)Rnew * std::max(rdi, 1));
    if (e == hipSuccess) e = launch_remap_rows(V[cur].p, Rold, map, Rnew, rdi, bV.p, stream);
    Vn = bV.p;
  }
  const double *Mc = factored ? Mf[cur].p : nullptr;
  // small buffers: P1, P2, P (rd x b each), GE (b x b), Wsc (b x b), VQ (rd x b),
  // QQ (b x b), VtV (rd x rd), then G, K, W, Rpad, sig for the dense part
  const size_t rb_ = (size_t)rdi * bi, bb = (size_t)bi * bi;
  const size_t off_p2 = rb_, off_p = 2 * rb_, off_ge = 3 * rb_, off_wsc = off_ge + bb,
               off_vq = off_wsc + bb, off_qq = off_vq + rb_, off_vtv = off_qq + bb,
               off_g = off_vtv + (size_t)rdi * rdi, off_k = off_g + nn2, off_w = off_k + nn2,
               off_r = off_w + nn2, off_sig = off_r + nn2, off_ge2 = off_sig + n2 + bi,
               off_gw = off_ge2 + bb, off_tt = off_gw + bb, off_tw = off_tt + rb_,
               off_tq = off_tw + rb_, off_x1 = off_tq + rb_, off_x2 = off_x1 + nn2,
               off_jp = off_x2 + nn2, off_jps = off_jp + nn2, off_sk = off_jps + nn2,
               nsmall = off_sk + n2;
  if (e == hipSuccess) e = bsm.ensure(nsmall);
  if (e == hipSuccess) e = bE.ensure((size_t)Rnew * bi);
  if (e == hipSuccess) e = qstat.ensure(2);
  if (e != hipSuccess) return hipfail(e, "block buffers");
  double *P1 = bsm.p, *P2 = bsm.p + off_p2, *Pv = bsm.p + off_p, *GE = bsm.p + off_ge,
         *Wsc = bsm.p + off_wsc, *VQ = bsm.p + off_vq, *QQ = bsm.p + off_qq,
         *VtV = bsm.p + off_vtv, *G = bsm.p + off_g, *K = bsm.p + off_k, *Wj = bsm.p + off_w,
         *Rp = bsm.p + off_r, *sig = bsm.p + off_sig, *GE2 = bsm.p + off_ge2,
         *GW = bsm.p + off_gw, *TT = bsm.p + off_tt, *TW = bsm.p + off_tw, *TQ = bsm.p + off_tq,
         *X1 = bsm.p + off_x1, *X2 = bsm.p + off_x2, *Jp = bsm.p + off_jp, *JpS = bsm.p + off_jps,
         *sK = bsm.p + off_sk;
  const double one = 1.0, mone = -1.0, zero = 0.0;
  rocblas_status bs = rocblas_status_success;
  // two Gram-Schmidt passes on all b columns
  // V^T X and V P: directly, or as M^T (V0^T X) and V0 (M P) in the factored form
  auto vt_times = [&](const double *X, int cols, double *out) -> hipError_t {
    if (!factored) return chunk_tn(Vn, Rnew, X, Rnew, Rnew, rdi, cols, out);
    hipError_t ee = chunk_tn(V0n, Rnew, X, Rnew, Rnew, rdi, cols, TT);
    if (ee == hipSuccess) ee = launch_small_gemm(1, Mc, rdi, TT, rdi, out, rdi, rdi, cols, rdi, stream);
    return ee;
  };
  auto sub_v_times = [&](const double *Pm, double *X) -> rocblas_status {
    const double *F = Pm;
    if (factored) {
      if (launch_small_gemm(0, Mc, rdi, Pm, rdi, TW, rdi, rdi, bi, rdi, stream) != hipSuccess)
        return rocblas_status_internal_error;
      F = TW;
    }
    return rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew,
                         bi, rdi, &mone, Vn, (rocblas_int)Rnew, F, rdi, &one, X,
                         (rocblas_int)Rnew);
  };
  if (rdi > 0) {
    e = vt_times(Dm, bi, P1);
    if (e == hipSuccess)
      e = hipMemcpyAsync(bE.p, Dm, (size_t)Rnew * bi * sizeof(double), hipMemcpyDeviceToDevice,
                         stream);
    if (e == hipSuccess) bs = sub_v_times(P1, bE.p);
    if (e == hipSuccess && bs == rocblas_status_success) e = vt_times(bE.p, bi, P2);
    if (e == hipSuccess && bs == rocblas_status_success) bs = sub_v_times(P2, bE.p);
    if (e == hipSuccess) e = launch_vadd(P1, P2, (int64_t)rb_, Pv, stream);
  } else {
    e = hipMemcpyAsync(bE.p, Dm, (size_t)Rnew * bi * sizeof(double), hipMemcpyDeviceToDevice,
                       stream);
  }
  if (bs != rocblas_status_success) return fail(ST_EHIP, "block projection GEMM failed");
  // TruncatedSVD of the residual block (Alg. 1 on E^T): eigenpairs of E^T E by
  // one-sided Jacobi (E^T E is positive semidefinite: its singular values are
  // its eigenvalues, its right singular vectors the eigenvectors)
  if (e == hipSuccess) e = chunk_tn(bE.p, Rnew, bE.p, Rnew, Rnew, bi, bi, GE);
  if (e == hipSuccess) e = hipMemsetAsync(qstat.p, 0, 2 * sizeof(int), stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(GE2, GE, bb * sizeof(double), hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess) e = launch_pad_upper(nullptr, 0, bi, Rp, stream);
  if (e == hipSuccess) e = launch_jacobi_svd(GE2, bi, Wj, 60, qstat.p, stream);
  // (sorted eigenvectors into GW; the left vectors, unused, into K)
  if (e == hipSuccess) e = launch_jacobi_finish(GE2, Wj, Rp, bi, K, GW, sig, sig + bi, stream);
  toc(ST_K_ISVD, 6.0 * Rnew * rdi * b + 2.0 * Rnew * b * b,
      8.0 * (2.0 * Rnew * rdi + 4.0 * Rnew * b));
  if (e == hipSuccess) e = launch_gather3(hpin_dev, sig, bi, 0, nullptr, 0, 0, nullptr, 0, 0, stream);
  int st2[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(st2, qstat.p, sizeof(st2), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "block residual");
  settle();
  if (st2[0] != 0) return fail(ST_ESOLVER, "block residual eigensolver did not converge");
  std::vector<double> lam_asc(bi), desc;
  for (int i = 0; i < bi; ++i) {
    if (!std::isfinite(hpin[i])) return fail(ST_ENONFINITE, "non-finite block residual");
    lam_asc[bi - 1 - i] = hpin[i];
  }
  int64_t ell64 = 0;
  double tail = 0.0;
  rank_rule(lam_asc.data(), bi, eps, ell64, tail, desc);
  const int ell = (int)ell64;
  const int c = rdi + ell;
  stt.q = std::sqrt(std::max(tail, 0.0));
  stt.isvd_ignored = ell < bi ? 1 : 0;
  stt.orth_check = 0.0;
  stt.qr_fired = 0;
  if (max_rank_d > 0 && c > max_rank_d)
    return fail(ST_ECAPACITY, "streaming rank %lld exceeds the cap", (long long)c);
  // buffers of the new state
  e = U2.ensure(nn2);
  if (e == hipSuccess) e = V2.ensure(nn2);
  if (e == hipSuccess) e = S[nxt].ensure((size_t)n2);
  // (the factored form keeps V0 in V[w0] and no core: its V buffers follow
  // v0cur, not cur, and must not be reallocated here)
  if (e == hipSuccess && !factored) e = V[nxt].ensure((size_t)Rnew * std::max(c, 1));
  if (e == hipSuccess && !factored) e = C[nxt].ensure((size_t)Rnew * std::max(c, 1));
  if (e == hipSuccess && factored) e = Mf[nxt].ensure((size_t)c * c);
  if (e == hipSuccess && factored) e = Gf[nxt].ensure((size_t)c * c);
  if (e == hipSuccess) e = bQ.ensure((size_t)Rnew * std::max(ell, 1));
  int64_t ldn = ud_ld[nxt];
  if (e == hipSuccess && (ldn < nd + b || Ud[nxt].cap < (size_t)ldn * c)) {
    ldn = std::max<int64_t>(ud_ld[cur], round_up(nd + b, 64));
    e = Ud[nxt].ensure((size_t)ldn * std::max(c, 1));
  }
  if (e != hipSuccess) return hipfail(e, "streaming buffers");
  ud_ld[nxt] = ldn;
  tic();
  if (ell > 0) {
    // Q = E W_l L_l^{-1/2}, and the orthogonality of [V Q]: V^T Q and Q^T Q - I
    e = launch_scale_cols_rsqrt(GW, bi, bi, ell, sig, Wsc, stream);
    if (e == hipSuccess)
      bs = rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew,
                         ell, bi, &one, bE.p, (rocblas_int)Rnew, Wsc, bi, &zero, bQ.p,
                         (rocblas_int)Rnew);
    if (bs != rocblas_status_success) return fail(ST_EHIP, "block basis GEMM failed");
    if (e == hipSuccess && rdi > 0) {
      if (factored) {
        // V0^T Q also extends G0 at the commit
        e = chunk_tn(V0n, Rnew, bQ.p, Rnew, Rnew, rdi, ell, TQ);
        if (e == hipSuccess)
          e = launch_small_gemm(1, Mc, rdi, TQ, rdi, VQ, rdi, rdi, ell, rdi, stream);
      } else {
        e = chunk_tn(Vn, Rnew, bQ.p, Rnew, Rnew, rdi, ell, VQ);
      }
    }
    if (e == hipSuccess) e = chunk_tn(bQ.p, Rnew, bQ.p, Rnew, Rnew, ell, ell, QQ);
    if (e == hipSuccess)
      e = launch_gather3(hpin_dev, VQ, rdi * ell, 0, QQ, ell * ell, rdi * ell, nullptr, 0, 0,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hipfail(e, "block orthogonality check");
    settle();
    double orth = 0.0;
    for (int i = 0; i < rdi * ell; ++i) orth = std::max(orth, std::fabs(hpin[i]));
    for (int j = 0; j < ell; ++j)
      for (int i = 0; i < ell; ++i)
        orth = std::max(orth, std::fabs(hpin[rdi * ell + i + ell * j] - (i == j ? 1.0 : 0.0)));
    stt.orth_check = orth;
    stt.qr_fired = orth > orth_tol ? 1 : 0;
  }
  // middle matrix (zero-padded to n2 x n2), with the QR fix when the check fired
  e = launch_block_k(S[cur].p, Pv, rdi, bi, GW, bi, sig, ell, K, stream);
  // With an old basis K keeps its structure (diag(S) over b rows) and its SVD
  // comes from the row appends; the QR fix then rotates those factors (K R^T =
  // U_K (R V_K diag(S_K))^T, whose right factor has columns orthogonal up to the
  // deviation the check measured, so the Jacobi on it ends in a sweep or two).
  // An empty old basis takes the dense one-sided Jacobi SVD of K (R^T).
  const bool by_rows = rdi > 0 && c <= kQrOrderMax;
  if (e == hipSuccess && stt.qr_fired) {
    if (rdi > 0 && factored) {
      // V^T V = M^T G0 M
      e = qrg.ensure((size_t)rdi * rdi);
      if (e == hipSuccess)
        e = launch_small_gemm(0, Gf[cur].p, rdi, Mc, rdi, qrg.p, rdi, rdi, rdi, rdi, stream);
      if (e == hipSuccess)
        e = launch_small_gemm(1, Mc, rdi, qrg.p, rdi, VtV, rdi, rdi, rdi, rdi, stream);
    } else if (rdi > 0) {
      e = chunk_tn(Vn, Rnew, Vn, Rnew, Rnew, rdi, rdi, VtV);
    }
    if (e == hipSuccess) e = launch_gram_block_fill(VtV, rdi, VQ, QQ, ell, G, stream);
    if (e == hipSuccess) e = launch_chol_upper(G, c, qstat.p, stream);
    if (e == hipSuccess && !by_rows) e = launch_right_mul_rt(K, n2, G, c, stream);
    if (e == hipSuccess && !by_rows) e = launch_pad_upper(G, c, n2, Rp, stream);
  } else if (e == hipSuccess) {
    e = hipMemsetAsync(qstat.p, 0, 2 * sizeof(int), stream);
  }
  if (by_rows) {
    const double tol =
        8.0 * 0x1p-53 * std::max(S_host.empty() ? 0.0 : S_host[0], std::sqrt(ynorm2));
    if (!stt.qr_fired) {
      if (e == hipSuccess) e = block_rows_svd(K, n2, rdi, bi, c, tol, U2.p, V2.p, S[nxt].p);
    } else {
      // U_K, V_K, S_K into X1, X2, sK; A = R V_K diag(S_K) over K (read by then)
      if (e == hipSuccess) e = block_rows_svd(K, n2, rdi, bi, c, tol, X1, X2, sK);
      if (e == hipSuccess) e = launch_form_rvs(G, c, X2, n2, sK, K, stream);
      if (e == hipSuccess) e = launch_jacobi_svd(K, c, Wj, 60, qstat.p, stream);
      if (e == hipSuccess) e = launch_qr_order(K, Wj, c, sK, S[nxt].p, Jp, JpS, stream);
      if (e == hipSuccess)
        e = launch_small_gemm(0, X1, n2, Jp, c, U2.p, n2, n2, c, c, stream);
      if (e == hipSuccess)
        e = launch_small_gemm(0, X2, n2, JpS, c, V2.p, n2, c, c, c, stream);
    }
    toc(ST_K_SVD, b * (60.0 * (double)c * c + 4.0 * (double)c * c * c + 2.0 * (double)c * c * b),
        8.0 * b * (4.0 * (double)c * c + (double)c * (c + b)));
  } else {
    if (e == hipSuccess && !stt.qr_fired) e = launch_pad_upper(nullptr, 0, n2, Rp, stream);
    if (e == hipSuccess) e = launch_jacobi_svd(K, n2, Wj, 60, qstat.p, stream);
    if (e == hipSuccess)
      e = launch_jacobi_finish(K, Wj, Rp, n2, U2.p, V2.p, S[nxt].p, sig, stream);
    toc(ST_K_SVD, 40.0 * (double)n2 * n2 * n2, 8.0 * 4.0 * nn2);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(st2, qstat.p, sizeof(st2), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "block middle matrix");
  settle();
  if (st2[0] == 1) return fail(ST_ESOLVER, "QR fix: the Gram of [V Q] is not positive definite");
  if (st2[0] == 2) return fail(ST_ESOLVER, "block middle matrix: Jacobi SVD did not converge");
  if (factored) {
    // [V Q] V'' = [V0 Q] diag(M, I) V'': Q becomes columns rd..c-1 of V0,
    // M~ = [M V''(0:rd, :); V''(rd:c, :)] and G0~ = [[G0, V0^T Q], [Q^T V0, Q^T Q]]
    tic();
    if (ell > 0)
      e = hipMemcpyAsync(V0n + (size_t)Rnew * rdi, bQ.p, (size_t)Rnew * ell * sizeof(double),
                         hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && rdi > 0)
      e = launch_small_gemm(0, Mc, rdi, V2.p, n2, Mf[nxt].p, c, rdi, c, rdi, stream);
    if (e == hipSuccess && ell > 0)
      e = hipMemcpy2DAsync(Mf[nxt].p + rdi, (size_t)c * sizeof(double), V2.p + rdi,
                           (size_t)n2 * sizeof(double), (size_t)ell * sizeof(double), c,
                           hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = launch_gram_block_fill(Gf[cur].p, rdi, TQ, QQ, ell, Gf[nxt].p, stream);
    toc(ST_K_SVD, 2.0 * (double)rdi * rdi * c, 8.0 * (Rnew * (double)ell + 2.0 * c * c));
    if (e != hipSuccess) return hipfail(e, "block factored update");
  } else {
  // V~ = V V''(0:rd, :) + Q V''(rd:c, :)
  tic();
  if (rdi > 0)
    bs = rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew, c,
                       rdi, &one, Vn, (rocblas_int)Rnew, V2.p, n2, &zero, V[nxt].p,
                       (rocblas_int)Rnew);
  if (bs == rocblas_status_success && ell > 0)
    bs = rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew, c,
                       ell, &one, bQ.p, (rocblas_int)Rnew, V2.p + rdi, n2,
                       rdi > 0 ? &one : &zero, V[nxt].p, (rocblas_int)Rnew);
  toc(ST_K_ROT_V, 2.0 * Rnew * (double)c * c, 8.0 * Rnew * (rdi + ell + c));
  if (bs != rocblas_status_success) return fail(ST_EHIP, "block V rotation failed");
  // C~ = C U''(0:rd, :) + Dm U''(rd:rd+b, :), formed in FP64 and rounded once
  tic();
  e = bC.ensure((size_t)Rnew * std::max(c, std::max(rdi, 1)) * 2);
  if (e != hipSuccess) return hipfail(e, "block core buffer");
  double *Cd = bC.p, *Cn = bC.p + (size_t)Rnew * std::max(c, std::max(rdi, 1));
  if (rdi > 0) e = launch_remap_rows_f32(C[cur].p, Rold, map, Rnew, rdi, Cd, stream);
  if (e == hipSuccess && rdi > 0)
    bs = rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew, c,
                       rdi, &one, Cd, (rocblas_int)Rnew, U2.p, n2, &zero, Cn, (rocblas_int)Rnew);
  if (e == hipSuccess && bs == rocblas_status_success)
    bs = rocblas_dgemm(rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)Rnew, c,
                       bi, &one, Dm, (rocblas_int)Rnew, U2.p + rdi, n2, rdi > 0 ? &one : &zero,
                       Cn, (rocblas_int)Rnew);
  if (e == hipSuccess && bs == rocblas_status_success)
    e = launch_f64_to_f32(Cn, Rnew * c, C[nxt].p, stream);
  toc(ST_K_ROT_C, 2.0 * Rnew * (double)(rdi + b) * c, 4.0 * Rold * rdi + 8.0 * Rnew * b + 4.0 * Rnew * c);
  if (bs != rocblas_status_success) return fail(ST_EHIP, "block core GEMM failed");
  if (e != hipSuccess) return hipfail(e, "block core update");
  }
  tic();
  e = launch_ud_update_block(Ud[cur].p, ud_ld[cur], nd, rdi, bi, U2.p, n2, c, Ud[nxt].p, ldn,
                             stream);
  toc(ST_K_UD, 2.0 * nd * (double)rd * c, 8.0 * ((double)nd * rd + (nd + b) * c));
  if (e == hipSuccess) e = ensure_hS((size_t)c);
  if (e == hipSuccess)
    e = launch_gather3(hS_dev, S[nxt].p, c, 0, nullptr, 0, 0, nullptr, 0, 0, stream);
  if (e != hipSuccess) return hipfail(e, "streaming factor update");
  // ---- commit ----
  snapshot();
  s_pending = c;
  for (int k = 0; k < m; ++k) r[k] = rn[k];
  rd = c;
  nd += b;
  cur = nxt;
  if (factored) v0cur = w0;
  xnorm2 += ynorm2;
  delta2 += tail;
  disc += delta2;
  stt.ynorm = std::sqrt(ynorm2);
  stt.eps = eps;
  stt.delta2 = delta2;
  stt.ms_modes = ms_modes;
  stt.ms_total = ms_since(t0);
  stt.ms_isvd = stt.ms_total - ms_modes;
  qr_total += stt.qr_fired;
  stt.qr_total = qr_total;
  stats = stt;
  return ST_OK;
}

// V0 M diag(S) (S not null: the core C_(d)^T) or V0 M (V) into out64 (R x r_d).
hipError_t st_handle::factored_product(const double *S_or_null, double *out64) {
  const int64_t R = rprod(r, m);
  const int rdi = (int)rd;
  hipError_t e = wvec.ensure((size_t)rdi * rdi + 2 * (size_t)rdi);
  if (e != hipSuccess) return e;
  double *W = wvec.p;
  e = launch_mt_rows(Mf[cur].p, rdi, S_or_null, W, rdi, stream);
  if (e != hipSuccess) return e;
  FiberIn in{};
  in.x = V[v0cur].p;
  in.x64 = 1;
  in.a = R;
  in.n = rd;
  in.F = R;
  in.mapped = 1;
  in.map.nm = m;
  in.map.identity = 1;
  return launch_rot64(in, W, 1, rdi, 0, rdi, FiberOut{out64, 1, R, rd}, 0, nullptr, stream);
}

// Slice t of C x_1 U_1 ... x_d U_d.
int st_handle::do_reconstruct_slice(int64_t t, float *out) {
  if (!inited) return fail(ST_ESTATE, "not initialised");
  if (t < 0 || t >= nd || out == nullptr) return fail(ST_EINVAL, "slice index out of range");
  const int64_t R = rprod(r, m);
  hipError_t e = wrow.ensure(round_up(rd, 4));
  if (e == hipSuccess) e = RB[0].ensure(NY);
  if (e == hipSuccess) e = RB[1].ensure(NY);
  if (e != hipSuccess) return hipfail(e, "reconstruct buffers");
  float *cur_buf = RB[0].p;
  if (factored) {
    // C x_d U_d(t,:) = V0 (M (S o U_d(t,:))), formed in FP64 and rounded once
    e = wvec.ensure(2 * (size_t)rd);
    if (e == hipSuccess)
      e = launch_ud_row64(Ud[cur].p, ud_ld[cur], t, (int)rd, S[cur].p, wvec.p, stream);
    if (e == hipSuccess)
      e = launch_small_gemv(Mf[cur].p, (int)rd, wvec.p, 0, wvec.p + rd, nullptr, nullptr, stream);
    if (e == hipSuccess)
      e = launch_vcol(V[v0cur].p, R, (int)rd, wvec.p + rd, nullptr, -1.0, nullptr, cur_buf,
                      stream);
  } else {
    e = launch_ud_row(Ud[cur].p, ud_ld[cur], t, (int)rd, wrow.p, stream);
    FiberIn in{};
    in.x = C[cur].p;
    in.a = R;
    in.n = rd;
    in.F = R;
    FiberW w{};
    w.w = wrow.p;
    w.ldw = rd;
    if (e == hipSuccess)
      e = launch_fiber_project(in, w, 0, 1, FiberOut{cur_buf, 0, R, 1}, nullptr, Prec::FP32,
                               stream);
  }
  int sel = 1;
  int64_t shape[ST_MAX_MODES];
  for (int k = 0; k < m; ++k) shape[k] = r[k];
  for (int k = m - 1; k >= 0 && e == hipSuccess; --k) {
    int64_t a = 1, b = 1;
    for (int l = 0; l < k; ++l) a *= shape[l];
    for (int l = k + 1; l < m; ++l) b *= shape[l];
    FiberIn ein{};
    ein.x = cur_buf;
    ein.a = a;
    ein.n = shape[k];
    ein.F = a * b;
    FiberW uw{};
    uw.w = Ut[k];
    uw.ldw = n[k];
    float *dst = (k == 0) ? out : RB[sel].p;
    e = launch_fiber_project(ein, uw, 0, (int)n[k], FiberOut{dst, 0, a, n[k]}, nullptr,
                             Prec::FP32, stream);
    shape[k] = n[k];
    cur_buf = dst;
    sel ^= 1;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hipfail(e, "reconstruct slice");
  return ST_OK;
}

void st_handle::destroy() {
  (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  for (int k = 0; k < m; ++k) {
    if (U64[k]) (void)hipFree(U64[k]);
    if (Uf[k]) (void)hipFree(Uf[k]);
    if (Ut[k]) (void)hipFree(Ut[k]);
    if (Uh[k]) (void)hipFree(Uh[k]);
    if (Ul[k]) (void)hipFree(Ul[k]);
  }
  for (int i = 0; i < 2; ++i) {
    Ud[i].release();
    S[i].release();
    V[i].release();
    Mf[i].release();
    Gf[i].release();
    C[i].release();
    D[i].release();
    RB[i].release();
  }
  for (int k = 0; k < ST_MAX_MODES; ++k) Dspec[k].release();
  specpart.release();
  specsums.release();
  wrow.release();
  tvec.release();
  wvec.release();
  e1buf.release();
  tmp64.release();
  qrw.release();
  bV.release();
  bE.release();
  bQ.release();
  bC.release();
  bsm.release();
  qrg.release();
  qvte.release();
  qstat.release();
  tmp32.release();
  part.release();
  sums.release();
  gram_part.release();
  G.release();
  eigval.release();
  eigtri.release();
  eigwork.release();
  Wnew.release();
  coef.release();
  info.release();
  colpart.release();
  q2part.release();
  p1.release();
  p2.release();
  p.release();
  U2.release();
  V2.release();
  Wv.release();
  Wc.release();
  sd.release();
  sz.release();
  szh.release();
  smu.release();
  srot_cs.release();
  szz.release();
  sact.release();
  sK.release();
  sdefl.release();
  sorg.release();
  srot_t.release();
  scounts.release();
  if (hpin) (void)hipHostFree(hpin);
  if (hS) (void)hipHostFree(hS);
  hpin = hpin_dev = hS = hS_dev = nullptr;
  hpin_cap = hS_cap = 0;
  for (auto &pd : pending) {
    event_pool.push_back(pd.a);
    event_pool.push_back(pd.b);
  }
  pending.clear();
  for (hipEvent_t ev : event_pool) (void)hipEventDestroy(ev);
  event_pool.clear();
  if (tic_ev) (void)hipEventDestroy(tic_ev);
  if (rb) rocblas_destroy_handle(rb);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int st_create(const st_config *cfg, st_handle **out) {
  g_create_error.clear();
  if (out == nullptr || cfg == nullptr) {
    g_create_error = "null argument";
    return ST_EINVAL;
  }
  *out = nullptr;
  if (cfg->nmodes < 1 || cfg->nmodes > ST_MAX_MODES || !(cfg->tau > 0.0) ||
      !std::isfinite(cfg->tau) || cfg->precision < ST_FP32 || cfg->precision > ST_FP64 ||
      cfg->max_rank_d < 0 ||
      (cfg->core_update != ST_CORE_LITERAL && cfg->core_update != ST_CORE_FACTORED)) {
    g_create_error = "invalid configuration";
    return ST_EINVAL;
  }
  int64_t ny = 1;
  for (int k = 0; k < cfg->nmodes; ++k) {
    if (cfg->dims[k] < 1 || cfg->dims[k] > (1 << 20)) {
      g_create_error = "invalid slice dimension";
      return ST_EINVAL;
    }
    ny *= cfg->dims[k];
  }
  if (ny > ((int64_t)1 << 34)) {
    g_create_error = "slice too large";
    return ST_EINVAL;
  }
  st_handle *h = new (std::nothrow) st_handle();
  if (!h) {
    g_create_error = "host allocation failed";
    return ST_ENOMEM;
  }
  h->m = cfg->nmodes;
  for (int k = 0; k < h->m; ++k) h->n[k] = cfg->dims[k];
  h->NY = ny;
  h->tau = cfg->tau;
  h->prec = cfg->precision == ST_BF16X3 ? Prec::BF16X3
                                        : (cfg->precision == ST_FP64 ? Prec::FP64 : Prec::FP32);
  h->orth_tol = cfg->orth_tol > 0.0 ? cfg->orth_tol : 1e-12;
  h->guard_rel = cfg->guard_rel > 0.0
                     ? cfg->guard_rel
                     : (h->prec == Prec::BF16X3 ? 5e-2 : (h->prec == Prec::FP32 ? 1e-2 : 0.0));
  h->max_rank_d = cfg->max_rank_d;
  h->profile = cfg->profile != 0;
  h->factored = cfg->core_update == ST_CORE_FACTORED;
  hipError_t e = hipGetDevice(&h->device);
  // the caller's stream, or the null stream (never a private non-blocking one:
  // inputs produced on the default stream must be complete before we read them)
  h->stream = (hipStream_t)cfg->stream;
  h->own_stream = false;
  for (int k = 0; k < h->m && e == hipSuccess; ++k) {
    const int64_t nk = h->n[k];
    h->ldb[k] = round_up(nk, 8);
    e = hipMalloc((void **)&h->U64[k], nk * nk * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->Uf[k], nk * nk * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&h->Ut[k], nk * nk * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&h->Uh[k], nk * h->ldb[k] * sizeof(__bf16));
    if (e == hipSuccess) e = hipMalloc((void **)&h->Ul[k], nk * h->ldb[k] * sizeof(__bf16));
    if (e == hipSuccess) e = hipMemsetAsync(h->Ut[k], 0, nk * nk * sizeof(float), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->Uf[k], 0, nk * nk * sizeof(float), h->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(h->Uh[k], 0, nk * h->ldb[k] * sizeof(__bf16), h->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(h->Ul[k], 0, nk * h->ldb[k] * sizeof(__bf16), h->stream);
  }
  if (e == hipSuccess) e = h->D[0].ensure(ny);
  if (e == hipSuccess) e = h->D[1].ensure(ny);
  if (e == hipSuccess) e = h->sums.ensure(64);
  if (e == hipSuccess) e = h->ensure_pinned(1024);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("device setup failed: ") + hipGetErrorString(e);
    h->destroy();
    delete h;
    return e == hipErrorOutOfMemory ? ST_ENOMEM : ST_EHIP;
  }
  if (rocblas_create_handle(&h->rb) != rocblas_status_success ||
      rocblas_set_stream(h->rb, h->stream) != rocblas_status_success) {
    g_create_error = "rocblas handle setup failed";
    h->destroy();
    delete h;
    return ST_EHIP;
  }
  *out = h;
  return ST_OK;
}

int st_init(st_handle *h, const float *x0, int64_t n_init) {
  if (!h) return ST_EINVAL;
  (void)hipSetDevice(h->device);
  return h->do_init(x0, n_init);
}

int st_update(st_handle *h, const float *y) {
  if (!h) return ST_EINVAL;
  (void)hipSetDevice(h->device);
  return h->do_update(y, 1);
}

int st_update_block(st_handle *h, const float *y, int64_t b) {
  if (!h) return ST_EINVAL;
  (void)hipSetDevice(h->device);
  return h->do_update(y, b);
}

int st_ranks(const st_handle *h, int64_t *ranks, int64_t *n_d) {
  if (!h || !ranks) return ST_EINVAL;
  for (int k = 0; k < h->m; ++k) ranks[k] = h->r[k];
  ranks[h->m] = h->rd;
  if (n_d) *n_d = h->nd;
  return ST_OK;
}

int st_core(const st_handle *hc, float *out, int64_t cap, int64_t *need, int where) {
  st_handle *h = const_cast<st_handle *>(hc);
  if (!h) return ST_EINVAL;
  if (!h->inited) return h->fail(ST_ESTATE, "not initialised");
  (void)hipSetDevice(h->device);
  if (const int rc = h->take_pending(); rc != ST_OK) return rc;
  const int64_t cnt = h->rprod(h->r, h->m) * h->rd;
  if (need) *need = cnt;
  if (!out) return ST_OK;
  if (cap < cnt) return h->fail(ST_ESMALL, "core buffer too small");
  (void)hipSetDevice(h->device);
  const float *src = h->C[h->cur].p;
  hipError_t e = hipSuccess;
  if (h->factored) {
    // C_(d)^T = V0 M diag(S), formed in FP64 and rounded once
    e = h->tmp64.ensure(cnt);
    if (e == hipSuccess) e = h->tmp32.ensure(cnt);
    if (e == hipSuccess) e = h->factored_product(h->S[h->cur].p, h->tmp64.p);
    if (e == hipSuccess) e = launch_f64_to_f32(h->tmp64.p, cnt, h->tmp32.p, h->stream);
    src = h->tmp32.p;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, src, cnt * sizeof(float),
                       where == ST_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hipfail(e, "core copy");
  return ST_OK;
}

int st_aux_v(const st_handle *hc, double *out, int64_t cap, int64_t *need, int where) {
  st_handle *h = const_cast<st_handle *>(hc);
  if (!h) return ST_EINVAL;
  if (!h->inited) return h->fail(ST_ESTATE, "not initialised");
  (void)hipSetDevice(h->device);
  if (const int rc = h->take_pending(); rc != ST_OK) return rc;
  const int64_t cnt = h->rprod(h->r, h->m) * h->rd;
  if (need) *need = cnt;
  if (!out) return ST_OK;
  if (cap < cnt) return h->fail(ST_ESMALL, "buffer too small");
  (void)hipSetDevice(h->device);
  const double *src = h->V[h->cur].p;
  hipError_t e = hipSuccess;
  if (h->factored) {  // V = V0 M
    e = h->tmp64.ensure(cnt);
    if (e == hipSuccess) e = h->factored_product(nullptr, h->tmp64.p);
    src = h->tmp64.p;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, src, cnt * sizeof(double),
                       where == ST_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hipfail(e, "V copy");
  return ST_OK;
}

int st_factor(const st_handle *hc, int mode, double *out, int64_t cap, int64_t *rows,
              int64_t *cols, int where) {
  st_handle *h = const_cast<st_handle *>(hc);
  if (!h) return ST_EINVAL;
  if (!h->inited) return h->fail(ST_ESTATE, "not initialised");
  (void)hipSetDevice(h->device);
  if (const int rc = h->take_pending(); rc != ST_OK) return rc;
  if (mode < 0 || mode > h->m) return h->fail(ST_EINVAL, "mode out of range");
  const int64_t nr = (mode < h->m) ? h->n[mode] : h->nd;
  const int64_t nc = (mode < h->m) ? h->r[mode] : h->rd;
  if (rows) *rows = nr;
  if (cols) *cols = nc;
  if (!out) return ST_OK;
  if (cap < nr * nc) return h->fail(ST_ESMALL, "factor buffer too small");
  (void)hipSetDevice(h->device);
  const hipMemcpyKind kind = where == ST_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  hipError_t e;
  if (mode < h->m) {
    e = hipMemcpyAsync(out, h->U64[mode], nr * nc * sizeof(double), kind, h->stream);
  } else {
    e = hipMemcpy2DAsync(out, nr * sizeof(double), h->Ud[h->cur].p,
                         h->ud_ld[h->cur] * sizeof(double), nr * sizeof(double), nc, kind,
                         h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return h->hipfail(e, "factor copy");
  return ST_OK;
}

int st_sv(const st_handle *hc, double *s, int64_t cap, int64_t *count) {
  if (!hc) return ST_EINVAL;
  st_handle *h = const_cast<st_handle *>(hc);  // takes a pending publication
  const int rc = h->take_pending();
  if (rc != ST_OK) return rc;
  if (count) *count = (int64_t)h->S_host.size();
  if (!s) return ST_OK;
  if (cap < (int64_t)h->S_host.size()) return ST_ESMALL;
  std::copy(h->S_host.begin(), h->S_host.end(), s);
  return ST_OK;
}

int st_recon_error(const st_handle *hc, double *rel_bound, double *norm_x) {
  st_handle *h = const_cast<st_handle *>(hc);
  if (!h) return ST_EINVAL;
  if (!h->inited) return ST_ESTATE;
  (void)hipSetDevice(h->device);
  if (const int rc = h->take_pending(); rc != ST_OK) return rc;
  if (rel_bound) *rel_bound = h->xnorm2 > 0 ? std::sqrt(h->disc / h->xnorm2) : 0.0;
  if (norm_x) *norm_x = std::sqrt(h->xnorm2);
  return ST_OK;
}

int st_stats(const st_handle *h, st_slice_stats *out) {
  if (!h || !out) return ST_EINVAL;
  *out = h->stats;
  return ST_OK;
}

int st_reconstruct_slice(const st_handle *hc, int64_t t, float *out) {
  st_handle *h = const_cast<st_handle *>(hc);
  if (!h) return ST_EINVAL;
  (void)hipSetDevice(h->device);
  if (const int rc = h->take_pending(); rc != ST_OK) return rc;
  return h->do_reconstruct_slice(t, out);
}

}  // extern "C"

namespace {

// Shape checks shared by st_ttm and st_ttm_noalloc; fills the fibre layout.
int ttm_args(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode, const float *a,
             int64_t rows, const float *out, const double *norms, int32_t precision,
             FiberIn &in, Prec &pr) {
  if (!x || !dims || !a || !out || nmodes < 1 || nmodes > ST_MAX_MODES || mode < 0 ||
      mode >= nmodes || rows < 1 || precision < ST_FP32 || precision > ST_FP64)
    return ST_EINVAL;
  int64_t lo = 1, hi = 1;
  for (int k = 0; k < nmodes; ++k) {
    if (dims[k] < 1) return ST_EINVAL;
    if (k < mode) lo *= dims[k];
    if (k > mode) hi *= dims[k];
  }
  if (norms && rows > 384) return ST_EINVAL;
  in = FiberIn{};
  in.x = x;
  in.a = lo;
  in.n = dims[mode];
  in.F = lo * hi;
  pr = precision == ST_BF16X3 ? Prec::BF16X3 : (precision == ST_FP64 ? Prec::FP64 : Prec::FP32);
  return ST_OK;
}

// Device buffers of one stateless TTM: the FP64 or split-bf16 copy of A (by
// precision) and the partial and total residual norms (with norms only).
struct TtmScratch {
  double *a64 = nullptr;
  __bf16 *bh = nullptr, *bl = nullptr;
  double *part = nullptr, *sum = nullptr;
};

size_t ttm_scratch_bytes(const FiberIn &in, int64_t rows, Prec pr, bool norms, size_t *off) {
  // offsets (256-byte aligned): [0] sum, [1] part, [2] a64 or bh, [3] bl
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const int64_t ldb = round_up(in.n, 8);
  size_t o = 0;
  off[0] = o;
  o += norms ? up(2 * sizeof(double)) : 0;
  off[1] = o;
  o += norms ? up(2 * (size_t)fiber_max_blocks(in.F) * sizeof(double)) : 0;
  off[2] = o;
  if (pr == Prec::FP64) o += up((size_t)rows * in.n * sizeof(double));
  if (pr == Prec::BF16X3) o += up((size_t)rows * ldb * sizeof(__bf16));
  off[3] = o;
  if (pr == Prec::BF16X3) o += up((size_t)rows * ldb * sizeof(__bf16));
  return o;
}

// The TTM itself on caller-provided scratch; waits for its work on s.
hipError_t ttm_run(const FiberIn &in, const float *a, int64_t rows, float *out, double *norms,
                   Prec pr, const TtmScratch &sc, hipStream_t s) {
  FiberW w{};
  w.w = a;
  w.ldw = in.n;
  hipError_t e = hipSuccess;
  if (pr == Prec::FP64) {
    e = launch_f32_to_f64(a, rows * in.n, sc.a64, s);
    w.w64 = sc.a64;
  }
  if (pr == Prec::BF16X3) {
    const int64_t ldb = round_up(in.n, 8);
    e = launch_split_rows(a, rows, in.n, in.n, sc.bh, sc.bl, ldb, s);
    w.w_hi = sc.bh;
    w.w_lo = sc.bl;
    w.ldw_bf = ldb;
  }
  int nb = 0;
  if (e == hipSuccess)
    e = launch_fiber_project(in, w, 0, (int)rows, FiberOut{out, 0, in.a, rows},
                             norms ? sc.part : nullptr, pr, s, &nb);
  if (e == hipSuccess && norms) e = launch_reduce_pairs(sc.part, nb, sc.sum, s);
  if (e == hipSuccess && norms)
    e = hipMemcpyAsync(norms, sc.sum, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// Fixed device scratch of st_ttm_noalloc (each GPU the library runs on holds
// its own copy until the process ends). Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int st_ttm(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode, const float *a,
           int64_t rows, float *out, double *norms, int32_t precision, void *stream) {
  FiberIn in{};
  Prec pr;
  int rc = ttm_args(x, nmodes, dims, mode, a, rows, out, norms, precision, in, pr);
  if (rc != ST_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ST_EHIP;  // initialises the runtime
  size_t off[4];
  const size_t bytes = ttm_scratch_bytes(in, rows, pr, norms != nullptr, off);
  unsigned char *buf = nullptr;
  hipError_t e = bytes ? hipMalloc((void **)&buf, bytes) : hipSuccess;
  if (e == hipSuccess) {
    TtmScratch sc;
    sc.sum = reinterpret_cast<double *>(buf + off[0]);
    sc.part = reinterpret_cast<double *>(buf + off[1]);
    sc.a64 = reinterpret_cast<double *>(buf + off[2]);
    sc.bh = reinterpret_cast<__bf16 *>(buf + off[2]);
    sc.bl = reinterpret_cast<__bf16 *>(buf + off[3]);
    e = ttm_run(in, a, rows, out, norms, pr, sc, s);
  }
  if (buf) (void)hipFree(buf);
  if (e == hipErrorOutOfMemory) return ST_ENOMEM;
  return e == hipSuccess ? ST_OK : ST_EHIP;
}

int st_ttm_noalloc(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode,
                   const float *a, int64_t rows, float *out, double *norms, int32_t precision,
                   void *stream) {
  FiberIn in{};
  Prec pr;
  int rc = ttm_args(x, nmodes, dims, mode, a, rows, out, norms, precision, in, pr);
  if (rc != ST_OK) {
    set_stateless_error("st_ttm_noalloc: invalid arguments");
    return rc;
  }
  size_t off[4];
  const size_t bytes = ttm_scratch_bytes(in, rows, pr, norms != nullptr, off);
  if (bytes > kNoAllocScratchBytes) {
    set_stateless_error("st_ttm_noalloc: the call needs more scratch than the fixed 8 MiB "
                        "(fibre count or rows x dims[mode] too large)");
    return ST_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ST_EHIP;
  void *base = nullptr;
  if (scratch_address(dev, &base) != hipSuccess) {
    set_stateless_error("st_ttm_noalloc: no device address for the scratch array");
    return ST_EHIP;
  }
  unsigned char *buf = static_cast<unsigned char *>(base);
  TtmScratch sc;
  sc.sum = reinterpret_cast<double *>(buf + off[0]);
  sc.part = reinterpret_cast<double *>(buf + off[1]);
  sc.a64 = reinterpret_cast<double *>(buf + off[2]);
  sc.bh = reinterpret_cast<__bf16 *>(buf + off[2]);
  sc.bl = reinterpret_cast<__bf16 *>(buf + off[3]);
  const hipError_t e = ttm_run(in, a, rows, out, norms, pr, sc, (hipStream_t)stream);
  return e == hipSuccess ? ST_OK : ST_EHIP;
}

int st_gram(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode, const float *a,
            int64_t rows, double *g, int32_t gram_precision, void *stream) {
  if (!x || !dims || !g || nmodes < 1 || nmodes > ST_MAX_MODES || mode < 0 || mode >= nmodes ||
      rows < 0 || rows > 256 || (rows > 0 && !a) || gram_precision < 0 || gram_precision > 2)
    return ST_EINVAL;
  int64_t lo = 1, hi = 1;
  for (int k = 0; k < nmodes; ++k) {
    if (dims[k] < 1) return ST_EINVAL;
    if (k < mode) lo *= dims[k];
    if (k > mode) hi *= dims[k];
  }
  const int64_t nk = dims[mode];
  if (nk > 512 || rows > nk) return ST_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ST_EHIP;  // initialises the runtime
  FiberIn in{};
  in.x = x;
  in.a = lo;
  in.n = nk;
  in.F = lo * hi;
  FiberW w{};
  w.w = a;
  w.ldw = nk;
  const GramPrec gp = (GramPrec)gram_precision;
  const int nb = gram_blocks(in.F, nk, gp);
  double *part = nullptr, *G = nullptr, *a64 = nullptr;
  // the FP64 Gram also forms the residual with FP64 products
  const bool e64 = gram_precision == 2 && rows > 0;
  hipError_t e = hipMalloc((void **)&part, gram_partial_elems(nk, nb, gp) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&G, nk * nk * sizeof(double));
  if (e == hipSuccess && e64) {
    e = hipMalloc((void **)&a64, rows * nk * sizeof(double));
    if (e == hipSuccess) e = launch_f32_to_f64(a, rows * nk, a64, s);
    w.w64 = a64;
  }
  if (e == hipSuccess) e = launch_gram(in, w, (int)rows, part, nb, gp, e64, s, G);
  if (e == hipSuccess) e = hipMemcpyAsync(g, G, nk * nk * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (part) (void)hipFree(part);
  if (G) (void)hipFree(G);
  if (a64) (void)hipFree(a64);
  if (e == hipErrorOutOfMemory) return ST_ENOMEM;
  return e == hipSuccess ? ST_OK : ST_EHIP;
}

int st_symeig(const double *a, int64_t n, double *w, double *q, int64_t k, void *stream) {
  if (!a || !w || n < 1 || n > kEigMaxN || k < 0 || k > n || (k > 0 && !q)) return ST_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ST_EHIP;  // initialises the runtime
  if (!eig_small_supported((int)n)) return ST_EINVAL;
  double *work = nullptr;
  hipError_t e = hipMalloc((void **)&work, eig_work_elems((int)n) * sizeof(double));
  if (e == hipSuccess) e = launch_eig_tridiag(a, (int)n, work, s);
  if (e == hipSuccess) e = launch_eig_values(work, (int)n, w, s);
  if (e == hipSuccess) e = launch_eig_vectors(work, (int)n, w, (int)k, q, n, 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (work) (void)hipFree(work);
  if (e == hipErrorOutOfMemory) return ST_ENOMEM;
  return e == hipSuccess ? ST_OK : ST_EHIP;
}

int st_profile(st_handle *h, st_kernel_profile *out, int32_t count, int32_t reset) {
  if (!h || (out == nullptr && count > 0) || count < 0) return ST_EINVAL;
  // the last update's device work may still be running: fold its intervals in
  if (hipStreamSynchronize(h->stream) == hipSuccess) h->settle();
  for (int i = 0; i < count && i < ST_K_GROUPS; ++i) out[i] = h->prof[i];
  if (reset)
    for (int i = 0; i < ST_K_GROUPS; ++i) h->prof[i] = st_kernel_profile{};
  return ST_OK;
}

void st_destroy(st_handle *h) {
  if (!h) return;
  h->destroy();
  delete h;
}

const char *st_last_error(const st_handle *h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
