// Symmetric eigendecomposition of the small FP64 Gram matrices of Alg. 1
// (TruncatedSVD through the Gram), order n <= kEigMaxN: every eigenvalue, and
// eigenvectors only for the k largest, the ones the rank rule keeps.
//
//   1. Householder tridiagonalisation in one block with the whole matrix in
//      registers. Step j reflects column j below the diagonal onto its first entry
//      (H_j = I - beta v v^T, the sign chosen against cancellation) and updates
//      the trailing block as B <- B - v w^T - w v^T with p = beta B v and
//      w = p - (beta / 2)(p^T v) v. The vectors v and the beta are kept.
//   2. Every eigenvalue of the tridiagonal T by multisection: one wave per
//      eigenvalue, each lane evaluating the Sturm count (the number of negative
//      pivots of the LDL^T factorisation of T - x I, which is the number of
//      eigenvalues below x) at one of 64 points of the current interval, so
//      each step shrinks it 65-fold; tiny pivots are replaced by -pivmin.
//   3. For each kept eigenvalue, inverse iteration on T in one wave (vectors
//      spread over the lanes, the recurrences stepping across them): three
//      solves with T - lambda I factored by Gaussian elimination with partial
//      pivoting (a zero or tiny last pivot replaced by u ||T||), each iterate
//      orthogonalised twice against the vectors already found in its cluster
//      (eigenvalues closer than 1e-3 ||T||), equal eigenvalues shifted apart by
//      ten ulps of ||T||. The reflections are then applied back,
//      x = H_0 H_1 ... H_{n-3} z.
// The three steps are the textbook ones (Wilkinson 1965; Parlett, The
// Symmetric Eigenvalue Problem, 1980, chapters 7 and 4). The eigenvalues carry
// an absolute error of a few u ||A||, the vectors u ||A|| / gap, as for any
// backward-stable method.
#include <algorithm>
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace st {

namespace {

constexpr double kU = 0x1p-53;

__device__ inline double wsum(double v) { return dpp_wave_sum(v); }
__device__ inline double wmax(double v) { return dpp_wave_max(v); }
__device__ inline double wmin(double v) { return -wmax(-v); }

// Block-wide sum / max (every thread active), the result in every thread;
// scratch holds one double per wave.
__device__ inline double bsum(double v, double *scratch) {
  const int nw = (int)(blockDim.x >> 6);
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t += scratch[w];
  return t;
}

__device__ inline double bmax(double v, double *scratch) {
  const int nw = (int)(blockDim.x >> 6);
  v = wmax(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, scratch[w]);
  return t;
}

// 1 / q: the hardware reciprocal refined by two Newton steps (about 1 ulp).
__device__ inline double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// Start vector of inverse iteration: a multiplicative hash of (row, vector)
// mapped to [-1, 1); any vector with a component along the wanted one works.
__device__ inline double start_value(int i, int c) {
  uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull + (uint64_t)(c + 1) * 0xBF58476D1CE4E5B9ull;
  h ^= h >> 31;
  h *= 0x94D049BB133111EBull;
  h ^= h >> 29;
  return (double)(h >> 11) * 0x1p-52 - 1.0;
}

// work = [Vh (n x n, column j holds v of step j in rows j+1..n-1), beta (n),
//         d (n), e (n)]; A is read from its lower triangle.
// The matrix stays in registers: thread (row = tid % 128, part = tid / 128)
// holds A(row, part + PARTS s), s < 128 / PARTS, PARTS = NTH / 128. The column
// being reduced, v and p pass through LDS; the reflections, d, e and beta are
// collected in LDS and written out once at the end.
template <int NTH>
__global__ __launch_bounds__(NTH) void eig_tridiag_kernel(const double *__restrict__ A, int n,
                                                         double *__restrict__ work) {
  constexpr int PARTS = NTH / 128, NS = 128 / PARTS;
  __shared__ double xb[128], vb[128], pb[128], pp[PARTS * 128], tb[3 * 128];
  extern __shared__ double vhs[];  // n x n
  double *bts = tb, *dds = tb + 128, *ees = tb + 256;
  const int tid = threadIdx.x, lane = tid & 63;
  const int row = tid & 127, part = tid >> 7;
  double ar[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = part + PARTS * s;
    ar[s] = (row < n && c < n) ? (row >= c ? A[row + (size_t)n * c] : A[c + (size_t)n * row])
                               : 0.0;
  }
  if (part == 0) xb[row] = ar[0];  // column 0 (zero past n)
  __syncthreads();
  for (int j = 0; j + 2 < n; ++j) {
    const int jn = j + 1;
    // sigma = sum_{i >= j+2} A(i, j)^2, formed alike in every wave
    double s2 = 0.0;
    for (int i = j + 2 + lane; i < n; i += 64) s2 += xb[i] * xb[i];
    s2 = wsum(s2);
    const double x0 = xb[jn];
    if (tid == 0) dds[j] = xb[j];
    if (s2 == 0.0) {  // already reduced: H_j = I (every thread takes this branch)
      if (tid == 0) {
        ees[j] = x0;
        bts[j] = 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (part + PARTS * s == jn) xb[row] = ar[s];  // the next column
      __syncthreads();
      continue;
    }
    const double alpha = -copysign(sqrt(x0 * x0 + s2), x0);
    const double v0 = x0 - alpha;
    const double bt = 2.0 / (v0 * v0 + s2);
    // partial sums of A v over this thread's columns; columns up to j (where v
    // vanishes) and past n are skipped, and so are waves whose rows all lie
    // outside the trailing block (both tests are uniform per wave)
    const bool live = (row | 63) > j && (row & ~63) < n;
    double acc0 = 0.0, acc1 = 0.0;
    if (live) {
#pragma unroll
      for (int s = 0; s < NS; s += 2) {
        const int c = part + PARTS * s, c1 = c + PARTS;
        if (c > j && c < n) acc0 = fma(ar[s], (c > jn) ? xb[c] : v0, acc0);
        if (c1 > j && c1 < n) acc1 = fma(ar[s + 1], (c1 > jn) ? xb[c1] : v0, acc1);
      }
    }
    pp[part * 128 + row] = acc0 + acc1;
    __syncthreads();
    if (tid < 128) {
      double p = 0.0, vi = 0.0;
      if (tid > j && tid < n) {
#pragma unroll
        for (int q = 0; q < PARTS; ++q) p += pp[q * 128 + tid];
        p *= bt;
        vi = (tid == jn) ? v0 : xb[tid];
        vhs[tid + n * j] = vi;
      }
      pb[tid] = p;
      vb[tid] = vi;
    }
    if (tid == 0) {
      ees[j] = alpha;
      bts[j] = bt;
    }
    __syncthreads();
    // K = (beta / 2) p^T v, formed alike in every wave; w = p - K v; A -= v w^T + w v^T
    const double K = 0.5 * bt * wsum(pb[lane] * vb[lane] + pb[lane + 64] * vb[lane + 64]);
    const double vr = vb[row], wr = pb[row] - K * vr;
    if (live) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int c = part + PARTS * s;
        if (c > j && c < n) {  // v and w vanish elsewhere
          const double vc = vb[c], wc = pb[c] - K * vc;
          ar[s] -= vr * wc + wr * vc;
          if (c == jn) xb[row] = ar[s];  // the next column, updated
        }
      }
    }
    __syncthreads();
  }
  if (n >= 2 && tid == 0) {
    dds[n - 2] = xb[n - 2];
    ees[n - 2] = xb[n - 1];
    bts[n - 2] = 0.0;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (row == n - 1 && part + PARTS * s == n - 1) {
      dds[n - 1] = ar[s];
      bts[n - 1] = 0.0;
    }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += NTH) work[idx] = vhs[idx];
  double *beta = work + (size_t)n * n;
  for (int i = tid; i < n; i += NTH) {
    beta[i] = bts[i];
    beta[n + i] = dds[i];
    beta[2 * n + i] = (i + 1 < n) ? ees[i] : 0.0;
  }
}

// w[i] (ascending) = the i-th eigenvalue of T; one wave per eigenvalue.
__global__ __launch_bounds__(256) void eig_values_kernel(const double *__restrict__ work, int n,
                                                        double *__restrict__ w) {
  __shared__ double sd[kEigMaxN], se2[kEigMaxN];
  const int tid = threadIdx.x, lane = tid & 63;
  const double *dd = work + (size_t)n * n + n, *ee = dd + n;
  for (int r = tid; r < n; r += blockDim.x) {
    sd[r] = dd[r];
    se2[r] = (r + 1 < n) ? ee[r] * ee[r] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * 4 + (tid >> 6);
  if (i >= n) return;  // the whole wave
  // Gershgorin interval, widened by a few ulps, and the pivot floor
  double lo_l = INFINITY, hi_l = -INFINITY, em2 = 0.0;
  for (int r = lane; r < n; r += 64) {
    const double rad = (r >= 1 ? fabs(ee[r - 1]) : 0.0) + (r + 1 < n ? fabs(ee[r]) : 0.0);
    lo_l = fmin(lo_l, sd[r] - rad);
    hi_l = fmax(hi_l, sd[r] + rad);
    em2 = fmax(em2, se2[r]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, wmax(em2));
  const double glo = wmin(lo_l), ghi = wmax(hi_l);
  const double tn = fmax(fabs(glo), fabs(ghi));
  double lo = glo - (4.0 * kU * tn + pivmin), hi = ghi + (4.0 * kU * tn + pivmin);
  for (int it = 0; it < 16; ++it) {
    const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
    double q = sd[0] - x;
    q = (fabs(q) < pivmin) ? -pivmin : q;
    int cnt = q < 0.0 ? 1 : 0;
#pragma unroll 4
    for (int kk = 1; kk < n; ++kk) {
      q = fma(-se2[kk - 1], recip(q), sd[kk] - x);
      q = (fabs(q) < pivmin) ? -pivmin : q;
      cnt += q < 0.0 ? 1 : 0;
    }
    // lambda_i >= x exactly where fewer than i + 1 eigenvalues lie below x: a
    // prefix of the (ascending) lanes
    const unsigned long long ok = __ballot(cnt <= i);
    const int l = (ok == ~0ull) ? 64 : __builtin_ctzll(~ok);
    const double nlo = (l > 0) ? lane_value(x, l - 1) : lo;
    const double nhi = (l < 64) ? lane_value(x, l) : hi;
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[i] = 0.5 * (lo + hi);
}

// Eigenvectors of the k largest eigenvalues (w ascending): vector c (eigenvalue
// w[n-1-c]) goes to column c of Q (desc_cols) or to column n-1-c. Thread 0 runs
// the recurrences of inverse iteration on LDS arrays (their loads do not
// depend on the running values, so they are issued ahead), the block the
// vector operations; then the reflections, staged in LDS, are applied by every
// wave.
// With k > 1, vectors whose eigenvalue is isolated (gap above gap_tol to both
// kept neighbours) need no orthogonalisation: they are found in parallel first, one
// thread each, kb at a time, with their right-hand sides and LU factors in the
// dynamic LDS (interleaved by vector) before it takes the reflections. The
// vectors of clusters follow one at a time, as above, with CGS2 in the cluster.
__global__ __launch_bounds__(256) void eig_vectors_kernel(const double *__restrict__ work, int n,
                                                         const double *__restrict__ w, int k,
                                                         double *Q, int64_t ldq, int desc_cols,
                                                         int kb) {
  __shared__ double sd[kEigMaxN], se[kEigMaxN], lm[kEigMaxN], ri[kEigMaxN], ua[kEigMaxN],
      ub[kEigMaxN], pv[kEigMaxN], xs[kEigMaxN], coef[kEigMaxN], red[4];
  extern __shared__ double vh[];  // the isolated vectors' scratch, then n x n reflections
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double *beta = work + (size_t)n * n, *dd = beta + n, *ee = dd + n;
  auto colq = [&](int c) { return Q + ldq * (desc_cols ? c : n - 1 - c); };
  for (int i = tid; i < n; i += blockDim.x) {
    sd[i] = dd[i];
    se[i] = (i + 1 < n) ? ee[i] : 0.0;
  }
  const double tn = bmax(tid < n ? fabs(dd[tid]) : 0.0, red) +
                    2.0 * bmax(tid + 1 < n ? fabs(ee[tid]) : 0.0, red);
  const double gap_tol = 1e-3 * tn, sep = 10.0 * kU * tn;
  const double tiny = fmax(kU * tn, DBL_MIN);
  // vector c opens a cluster when its gap to vector c - 1 exceeds gap_tol
  auto opens = [&](int c) { return c == 0 || w[n - c] - w[n - 1 - c] > gap_tol; };
  // (a lone vector, k = 1, takes the block-wide loop below: one thread's serial
  // normalisation costs more than the block reductions there)
  auto isolated = [&](int c) { return k > 1 && opens(c) && (c + 1 >= k || opens(c + 1)); };
  for (int b0 = 0; b0 < k && k > 1; b0 += kb) {
    // the batch's start vectors, by all threads (X(i, t) at vh[i kb + t])
    for (int idx = tid; idx < n * kb; idx += blockDim.x)
      if (b0 + idx % kb < k) vh[idx] = start_value(idx / kb, b0 + idx % kb);
    __syncthreads();
    const int t = tid, c = b0 + tid;
    if (t < kb && c < k && isolated(c)) {
      double *X = vh + t, *Lm = X + (size_t)n * kb, *Ri = Lm + (size_t)n * kb,
             *Ua = Ri + (size_t)n * kb, *Ub = Ua + (size_t)n * kb, *Pv = Ub + (size_t)n * kb;
      const double lam = w[n - 1 - c];
      // T - lam I = P L U, as below
      double p = sd[0] - lam, q = se[0];
      for (int kk = 0; kk + 1 < n; ++kk) {
        const double dn = sd[kk + 1] - lam, ek = se[kk], en = se[kk + 1];
        const bool sw = fabs(p) < fabs(ek);
        const double pz = (!sw && p == 0.0) ? tiny : p;
        const double r1 = recip(sw ? ek : pz);
        const double l = (sw ? pz : ek) * r1;
        const size_t o = (size_t)kk * kb;
        Lm[o] = l;
        Ri[o] = r1;
        Ua[o] = sw ? dn : q;
        Ub[o] = sw ? en : 0.0;
        Pv[o] = sw ? 1.0 : 0.0;
        const double pn = sw ? fma(-l, dn, q) : fma(-l, q, dn);
        q = sw ? -l * en : en;
        p = pn;
      }
      p = (fabs(p) < tiny) ? ((p < 0.0) ? -tiny : tiny) : p;
      const size_t ol = (size_t)(n - 1) * kb;
      Ri[ol] = recip(p);
      Ua[ol] = 0.0;
      Ub[ol] = 0.0;
      for (int it = 0; it < 3; ++it) {
        double carry = X[0];
#pragma unroll 4
        for (int kk = 0; kk + 1 < n; ++kk) {
          const size_t o = (size_t)kk * kb;
          const double nx = X[o + kb];
          const bool sw = Pv[o] != 0.0;
          const double a = sw ? nx : carry;
          carry = fma(-Lm[o], a, sw ? carry : nx);
          X[o] = a;
        }
        X[ol] = carry;
        double y1 = 0.0, y2 = 0.0, mx = 0.0;
#pragma unroll 4
        for (int kk = n - 1; kk >= 0; --kk) {
          const size_t o = (size_t)kk * kb;
          const double y = fma(-Ub[o], y2, fma(-Ua[o], y1, X[o])) * Ri[o];
          X[o] = y;
          mx = fmax(mx, fabs(y));
          y2 = y1;
          y1 = y;
        }
        // scaled by the largest entry first (no overflow in the squares); by a
        // reciprocal unless the largest entry is so small that it overflows
        const bool by_div = mx > 0.0 && mx < 0x1p-1000;
        const double rm = (mx > 0.0 && !by_div) ? 1.0 / mx : 1.0;
        double nr = 0.0;
        for (int i = 0; i < n; ++i) {
          const double x = X[(size_t)i * kb], y = by_div ? x / mx : x * rm;
          nr = fma(y, y, nr);
        }
        const double rn = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0, sc = rm * rn;
        for (int i = 0; i < n; ++i) {
          const double x = X[(size_t)i * kb];
          X[(size_t)i * kb] = by_div ? (x / mx) * rn : x * sc;
        }
      }
      double *z = colq(c);
      for (int i = 0; i < n; ++i) z[i] = X[(size_t)i * kb];
    }
    __syncthreads();  // the scratch is reused by the next batch
  }
  int cs = 0;
  double lam_prev = 0.0;
  for (int c = 0; c < k; ++c) {
    double lam = w[n - 1 - c];
    if (c > 0) {
      const double gap = w[n - c] - lam;
      if (gap > gap_tol) cs = c;                  // a new cluster starts
      else if (gap <= sep) lam = lam_prev - sep;  // equal: shift apart
    }
    lam_prev = lam;
    if (isolated(c)) continue;  // found above
    if (tid == 0) {
      // T - lam I = P L U (U with two superdiagonals): multipliers lm, 1/u1 in
      // ri, u2 in ua, u3 in ub, row swaps in pv
      double p = sd[0] - lam, q = se[0];
      for (int kk = 0; kk + 1 < n; ++kk) {
        const double dn = sd[kk + 1] - lam, ek = se[kk], en = se[kk + 1];
        const bool sw = fabs(p) < fabs(ek);
        const double pz = (!sw && p == 0.0) ? tiny : p;
        const double r1 = recip(sw ? ek : pz);
        const double l = (sw ? pz : ek) * r1;
        lm[kk] = l;
        ri[kk] = r1;
        ua[kk] = sw ? dn : q;
        ub[kk] = sw ? en : 0.0;
        pv[kk] = sw ? 1.0 : 0.0;
        const double pn = sw ? fma(-l, dn, q) : fma(-l, q, dn);
        q = sw ? -l * en : en;
        p = pn;
      }
      p = (fabs(p) < tiny) ? ((p < 0.0) ? -tiny : tiny) : p;
      ri[n - 1] = recip(p);
      ua[n - 1] = 0.0;  // (multiplied by zero in the back substitution)
      ub[n - 1] = 0.0;
    }
    double xi = (tid < n) ? start_value(tid, c) : 0.0;
    for (int it = 0; it < 3; ++it) {
      if (tid < n) xs[tid] = xi;
      __syncthreads();
      if (tid == 0) {
        // the row swaps and L, then U
        double carry = xs[0];
#pragma unroll 4
        for (int kk = 0; kk + 1 < n; ++kk) {
          const double nx = xs[kk + 1];
          const bool sw = pv[kk] != 0.0;
          const double a = sw ? nx : carry;
          carry = fma(-lm[kk], a, sw ? carry : nx);
          xs[kk] = a;
        }
        xs[n - 1] = carry;
        double y1 = 0.0, y2 = 0.0;
#pragma unroll 4
        for (int kk = n - 1; kk >= 0; --kk) {
          const double y = fma(-ub[kk], y2, fma(-ua[kk], y1, xs[kk])) * ri[kk];
          xs[kk] = y;
          y2 = y1;
          y1 = y;
        }
      }
      __syncthreads();
      double yi = (tid < n) ? xs[tid] : 0.0;
      // twice against the cluster's vectors found so far (still in T's basis)
      for (int rep = 0; rep < 2 && c > cs; ++rep) {
        for (int p = cs + wid; p < c; p += 4) {
          const double *zp = colq(p);
          double sp = 0.0;
          for (int i = lane; i < n; i += 64) sp += zp[i] * xs[i];
          sp = wsum(sp);
          if (lane == 0) coef[p - cs] = sp;
        }
        __syncthreads();
        if (tid < n) {
          double acc = yi;
          for (int p = cs; p < c; ++p) acc -= coef[p - cs] * colq(p)[tid];
          yi = acc;
        }
        __syncthreads();
        if (tid < n) xs[tid] = yi;
        __syncthreads();
      }
      const double mx = bmax(fabs(yi), red);
      if (mx > 0.0) yi /= mx;
      const double nr = bsum(yi * yi, red);
      xi = nr > 0.0 ? yi / sqrt(nr) : 0.0;
    }
    if (tid < n) colq(c)[tid] = xi;
    __syncthreads();  // the vector is read by the next ones of its cluster
  }
  // back to A's basis: x = H_0 ... H_{n-3} z; wave wid takes vectors wid, wid + 4, ...
  for (int idx = tid; idx < n * n; idx += blockDim.x) vh[idx] = work[idx];
  __syncthreads();
  for (int c = wid; c < k; c += 4) {
    double *zc = colq(c);
    double z0 = lane < n ? zc[lane] : 0.0, z1 = lane + 64 < n ? zc[lane + 64] : 0.0;
    for (int j = n - 3; j >= 0; --j) {
      const double bj = beta[j];
      if (bj == 0.0) continue;
      const double *v = vh + (size_t)n * j;
      const double v0 = (lane > j && lane < n) ? v[lane] : 0.0;
      const double v1 = (lane + 64 > j && lane + 64 < n) ? v[lane + 64] : 0.0;
      const double sj = bj * wsum(v0 * z0 + v1 * z1);
      z0 -= sj * v0;
      z1 -= sj * v1;
    }
    if (lane < n) zc[lane] = z0;
    if (lane + 64 < n) zc[lane + 64] = z1;
  }
}

}  // namespace

size_t eig_work_elems(int n) { return (size_t)n * n + 3 * (size_t)n; }

// dynamic LDS of the tridiagonalisation and of the vectors (the staged
// reflections); each kernel adds at most 16 KiB of static LDS
// (the vectors' LDS also holds, before the reflections, six n-long arrays for
// each of up to kb isolated vectors at a time: at least min(k, 16) of them)
static size_t vectors_lds_elems(int n, int k) {
  return std::max((size_t)n * n, 6 * (size_t)n * (size_t)std::min(k, 16));
}
static size_t vectors_lds_bytes(int n) { return vectors_lds_elems(n, 16) * sizeof(double); }

bool eig_small_supported(int n) {
  if (n < 1 || n > kEigMaxN) return false;
  // the opt-in shared memory per block of the current device, queried once
  // (a thread-safe static initialisation; the library runs one device type)
  static const int limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
      v = 0;
    return v;
  }();
  return vectors_lds_bytes(n) + 16384 <= (size_t)limit;
}

template <int NTH>
static hipError_t launch_tridiag_t(const double *A, int n, double *work, hipStream_t s) {
  const size_t lds = (size_t)n * n * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)eig_tridiag_kernel<NTH>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eig_tridiag_kernel<NTH>), dim3(1), dim3(NTH), lds, s, A, n, work);
  return hipGetLastError();
}

hipError_t launch_eig_tridiag(const double *A, int n, double *work, hipStream_t s) {
  if (n < 1 || n > kEigMaxN) return hipErrorInvalidValue;
  // 16 waves: each step is a chain of short phases between barriers, and with
  // fewer waves per SIMD their latencies are not covered (512 threads took
  // 1.3x and 256 threads 2.5x as long at n = 128)
  return launch_tridiag_t<1024>(A, n, work, s);
}

hipError_t launch_eig_values(const double *work, int n, double *w, hipStream_t s) {
  if (n < 1 || n > kEigMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(eig_values_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, work, n,
                     w);
  return hipGetLastError();
}

hipError_t launch_eig_vectors(const double *work, int n, const double *w, int k, double *Q,
                              int64_t ldq, int desc_cols, hipStream_t s) {
  if (n < 1 || n > kEigMaxN || k < 0 || k > n || ldq < n) return hipErrorInvalidValue;
  if (k == 0) return hipSuccess;
  const size_t elems = vectors_lds_elems(n, k), lds = elems * sizeof(double);
  const int kb = (int)std::min((size_t)k, elems / (6 * (size_t)n));  // >= min(k, 16), <= 21
  hipError_t e = hipFuncSetAttribute((const void *)eig_vectors_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_vectors_kernel, dim3(1), dim3(256), lds, s, work, n, w, k, Q, ldq,
                     desc_cols, kb);
  return hipGetLastError();
}

}  // namespace st
