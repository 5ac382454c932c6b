// Symmetric eigendecomposition of the small FP64 Gram matrices of Alg. 1
// (TruncatedSVD through the Gram), order n <= kEigMaxN: every eigenvalue, and
// eigenvectors only for the k largest, the ones the rank rule keeps.
//
//   1. Householder tridiagonalisation in one block with the whole matrix in
//      LDS. Step j reflects column j below the diagonal onto its first entry
//      (H_j = I - beta v v^T, the sign chosen against cancellation) and updates
//      the trailing block as B <- B - v w^T - w v^T with p = beta B v and
//      w = p - (beta / 2)(p^T v) v. The vectors v and the beta are kept.
//   2. Every eigenvalue of the tridiagonal T by multisection: one wave per
//      eigenvalue, each lane evaluating the Sturm count (the number of negative
//      pivots of the LDL^T factorisation of T - x I, which is the number of
//      eigenvalues below x) at one of 64 points of the current interval, so
//      each step shrinks it 65-fold; tiny pivots are replaced by -pivmin.
//   3. For each kept eigenvalue, inverse iteration on T: three solves with
//      T - lambda I factored by Gaussian elimination with partial pivoting (a
//      zero or tiny last pivot replaced by u ||T||), each iterate
//      orthogonalised twice against the vectors already found in its cluster
//      (eigenvalues closer than 1e-3 ||T||), equal eigenvalues shifted apart by
//      ten ulps of ||T||. The reflections are then applied back,
//      x = H_0 H_1 ... H_{n-3} z.
// The three steps are the textbook ones (Wilkinson 1965; Parlett, The
// Symmetric Eigenvalue Problem, 1980, chapters 7 and 4). The eigenvalues carry
// an absolute error of a few u ||A||, the vectors u ||A|| / gap, as for any
// backward-stable method.
#include <cfloat>

#include "common.hpp"
#include "kernels.hpp"

namespace st {

namespace {

constexpr double kU = 0x1p-53;

// LDS of the tridiagonalisation: the matrix, 8 x 128 partial sums of B v, p, v
size_t tridiag_lds_bytes(int n) { return ((size_t)n * n + 8 * 128 + 2 * 128) * sizeof(double); }

__device__ inline double block_max(double v, double *scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, scratch[w]);
  return t;
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
__global__ __launch_bounds__(1024) void eig_tridiag_kernel(const double *__restrict__ A, int n,
                                                          double *__restrict__ work) {
  extern __shared__ double lds[];
  double *a = lds;              // n x n, ld n
  double *pp = a + n * n;       // partial sums of B v: 8 x 128
  double *pb = pp + 8 * 128;    // p = beta B v
  double *vb = pb + 128;        // v
  const int tid = threadIdx.x, lane = tid & 63;
  double *Vh = work, *beta = work + (size_t)n * n, *dd = beta + n, *ee = dd + n;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, k = idx / n;
    a[idx] = (i >= k) ? A[i + (size_t)n * k] : A[k + (size_t)n * i];
  }
  __syncthreads();
  const int row = tid & 127, part = tid >> 7;  // 8 threads per row of the trailing block
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const double *x = a + (j + 1) + (size_t)n * j;  // column j below the diagonal
    // sigma = sum_{i >= 1} x_i^2, formed alike in every wave
    double s = 0.0;
    for (int i = 1 + lane; i < m; i += 64) s += x[i] * x[i];
    s = wave_sum(s);
    const double x0 = x[0];
    if (tid == 0) dd[j] = a[j + (size_t)n * j];
    if (s == 0.0) {  // already reduced: H_j = I (every thread takes this branch)
      if (tid == 0) {
        ee[j] = x0;
        beta[j] = 0.0;
      }
      continue;
    }
    const double alpha = -copysign(sqrt(x0 * x0 + s), x0);
    const double v0 = x0 - alpha;
    const double bt = 2.0 / (v0 * v0 + s);
    if (row < m) {
      const double *brow = a + (j + 1 + row);
      double acc = 0.0;
      for (int kk = part; kk < m; kk += 8) {
        const double vk = (kk == 0) ? v0 : x[kk];
        acc += brow[(size_t)n * (j + 1 + kk)] * vk;
      }
      pp[part * 128 + row] = acc;
    }
    __syncthreads();
    if (tid < m) {
      double p = 0.0;
      for (int q = 0; q < 8; ++q) p += pp[q * 128 + tid];
      pb[tid] = bt * p;
      const double vi = (tid == 0) ? v0 : x[tid];
      vb[tid] = vi;
      Vh[(j + 1 + tid) + (size_t)n * j] = vi;
    }
    if (tid == 0) {
      ee[j] = alpha;
      beta[j] = bt;
    }
    __syncthreads();
    // K = (beta / 2) p^T v, formed alike in every wave; w = p - K v
    double kv = 0.0;
    for (int i = lane; i < m; i += 64) kv += pb[i] * vb[i];
    const double K = 0.5 * bt * wave_sum(kv);
    if (row < m) {
      const double vi = vb[row], wi = pb[row] - K * vi;
      double *brow = a + (j + 1 + row);
      for (int kk = part; kk < m; kk += 8) {
        const double vk = vb[kk], wk = pb[kk] - K * vk;
        brow[(size_t)n * (j + 1 + kk)] -= vi * wk + wi * vk;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = a[(n - 2) + (size_t)n * (n - 2)];
      ee[n - 2] = a[(n - 1) + (size_t)n * (n - 2)];
      beta[n - 2] = 0.0;
    }
    dd[n - 1] = a[(n - 1) + (size_t)n * (n - 1)];
    beta[n - 1] = 0.0;
  }
}

// w[i] (ascending) = the i-th eigenvalue of T; one wave per eigenvalue.
__global__ __launch_bounds__(256) void eig_values_kernel(const double *__restrict__ work, int n,
                                                        double *__restrict__ w) {
  __shared__ double sd[kEigMaxN], se2[kEigMaxN], bnd[3];
  const int tid = threadIdx.x, lane = tid & 63;
  const double *dd = work + (size_t)n * n + n, *ee = dd + n;
  for (int i = tid; i < n; i += blockDim.x) {
    sd[i] = dd[i];
    se2[i] = (i + 1 < n) ? ee[i] * ee[i] : 0.0;
  }
  if (tid == 0) {
    // Gershgorin interval, widened by a few ulps, and the pivot floor
    double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
      lo = fmin(lo, dd[i] - r);
      hi = fmax(hi, dd[i] + r);
      if (i + 1 < n) emax2 = fmax(emax2, ee[i] * ee[i]);
    }
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double tn = fmax(fabs(lo), fabs(hi));
    bnd[0] = lo - (4.0 * kU * tn + pivmin);
    bnd[1] = hi + (4.0 * kU * tn + pivmin);
    bnd[2] = pivmin;
  }
  __syncthreads();
  const int i = blockIdx.x * 4 + (tid >> 6);
  if (i >= n) return;
  double lo = bnd[0], hi = bnd[1];
  const double pivmin = bnd[2];
  for (int it = 0; it < 16; ++it) {
    const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
    double q = sd[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0 ? 1 : 0;
    for (int kk = 1; kk < n; ++kk) {
      q = (sd[kk] - x) - se2[kk - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0 ? 1 : 0;
    }
    // lambda_i >= x exactly where fewer than i + 1 eigenvalues lie below x: a
    // prefix of the (ascending) lanes
    const unsigned long long ok = __ballot(cnt <= i);
    const int l = (ok == ~0ull) ? 64 : __builtin_ctzll(~ok);
    const double nlo = (l > 0) ? __shfl(x, l - 1, kWave) : lo;
    const double nhi = (l < 64) ? __shfl(x, l, kWave) : hi;
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[i] = 0.5 * (lo + hi);
}

// Eigenvectors of the k largest eigenvalues (w ascending): vector c (eigenvalue
// w[n-1-c]) goes to column c of Q (desc_cols) or to column n-1-c.
__global__ __launch_bounds__(256) void eig_vectors_kernel(const double *__restrict__ work, int n,
                                                         const double *__restrict__ w, int k,
                                                         double *Q, int64_t ldq, int desc_cols) {
  __shared__ double sd[kEigMaxN], se[kEigMaxN], u1[kEigMaxN], u2[kEigMaxN], u3[kEigMaxN],
      lm[kEigMaxN], xs[kEigMaxN], coef[kEigMaxN], red[4];
  __shared__ int piv[kEigMaxN];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double *Vh = work, *beta = work + (size_t)n * n, *dd = beta + n, *ee = dd + n;
  auto colq = [&](int c) { return Q + ldq * (desc_cols ? c : n - 1 - c); };
  for (int i = tid; i < n; i += blockDim.x) {
    sd[i] = dd[i];
    se[i] = (i + 1 < n) ? ee[i] : 0.0;
  }
  const double tn = block_max(tid < n ? fabs(dd[tid]) : 0.0, red) +
                    2.0 * block_max(tid + 1 < n ? fabs(ee[tid]) : 0.0, red);
  const double gap_tol = 1e-3 * tn, sep = 10.0 * kU * tn;
  const double tiny = fmax(kU * tn, DBL_MIN);
  int cs = 0;
  double lam_prev = 0.0;
  for (int c = 0; c < k; ++c) {
    double lam = w[n - 1 - c];
    if (c > 0) {
      const double gap = w[n - c] - lam;
      if (gap > gap_tol) cs = c;               // a new cluster starts
      else if (gap <= sep) lam = lam_prev - sep;  // equal: shift apart
    }
    lam_prev = lam;
    if (tid == 0) {
      // T - lam I = P L U, U with two superdiagonals (u2, u3)
      double p = sd[0] - lam, q = (n > 1) ? se[0] : 0.0;
      for (int kk = 0; kk + 1 < n; ++kk) {
        const double dn = sd[kk + 1] - lam, en = (kk + 2 < n) ? se[kk + 1] : 0.0, ek = se[kk];
        if (fabs(p) >= fabs(ek)) {
          if (p == 0.0) p = tiny;
          const double l = ek / p;
          lm[kk] = l;
          u1[kk] = p;
          u2[kk] = q;
          u3[kk] = 0.0;
          piv[kk] = 0;
          p = dn - l * q;
          q = en;
        } else {
          const double l = p / ek;
          lm[kk] = l;
          u1[kk] = ek;
          u2[kk] = dn;
          u3[kk] = en;
          piv[kk] = 1;
          p = q - l * dn;
          q = -l * en;
        }
      }
      if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
      u1[n - 1] = p;
    }
    double xi = (tid < n) ? start_value(tid, c) : 0.0;
    for (int it = 0; it < 3; ++it) {
      if (tid < n) xs[tid] = xi;
      __syncthreads();
      if (tid == 0) {
        for (int kk = 0; kk + 1 < n; ++kk) {
          if (piv[kk]) {
            const double t = xs[kk];
            xs[kk] = xs[kk + 1];
            xs[kk + 1] = t;
          }
          xs[kk + 1] -= lm[kk] * xs[kk];
        }
        xs[n - 1] /= u1[n - 1];
        for (int kk = n - 2; kk >= 0; --kk) {
          double s = xs[kk] - u2[kk] * xs[kk + 1];
          if (kk + 2 < n) s -= u3[kk] * xs[kk + 2];
          xs[kk] = s / u1[kk];
        }
      }
      __syncthreads();
      double yi = (tid < n) ? xs[tid] : 0.0;
      // twice against the cluster's vectors found so far (still in T's basis)
      for (int rep = 0; rep < 2 && c > cs; ++rep) {
        for (int p = cs + wid; p < c; p += 4) {
          const double *zp = colq(p);
          double s = 0.0;
          for (int i = lane; i < n; i += 64) s += zp[i] * xs[i];
          s = wave_sum(s);
          if (lane == 0) coef[p - cs] = s;
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
      const double mx = block_max(fabs(yi), red);
      if (mx > 0.0) yi /= mx;
      const double nr = block_sum(yi * yi, red);
      xi = nr > 0.0 ? yi / sqrt(nr) : 0.0;
    }
    if (tid < n) colq(c)[tid] = xi;
    __syncthreads();  // the vector is read by the next ones of its cluster
  }
  // back to A's basis: x = H_0 ... H_{n-3} z; wave wid takes vectors wid, wid + 4, ...
  for (int c = wid; c < k; c += 4) {
    double *zc = colq(c);
    double z0 = lane < n ? zc[lane] : 0.0, z1 = lane + 64 < n ? zc[lane + 64] : 0.0;
    for (int j = n - 3; j >= 0; --j) {
      const double bj = beta[j];
      if (bj == 0.0) continue;
      const double *v = Vh + (size_t)n * j;
      const double v0 = (lane > j && lane < n) ? v[lane] : 0.0;
      const double v1 = (lane + 64 > j && lane + 64 < n) ? v[lane + 64] : 0.0;
      const double s = bj * wave_sum(v0 * z0 + v1 * z1);
      z0 -= s * v0;
      z1 -= s * v1;
    }
    if (lane < n) zc[lane] = z0;
    if (lane + 64 < n) zc[lane + 64] = z1;
  }
}

}  // namespace

size_t eig_work_elems(int n) { return (size_t)n * n + 3 * (size_t)n; }

bool eig_small_supported(int n) {
  if (n < 1 || n > kEigMaxN) return false;
  static int limit = -1;
  if (limit < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
      v = 0;
    limit = v;
  }
  return tridiag_lds_bytes(n) <= (size_t)limit;
}

hipError_t launch_eig_tridiag(const double *A, int n, double *work, hipStream_t s) {
  if (n < 1 || n > kEigMaxN) return hipErrorInvalidValue;
  const size_t lds = tridiag_lds_bytes(n);
  hipError_t e = hipFuncSetAttribute((const void *)eig_tridiag_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_tridiag_kernel, dim3(1), dim3(1024), lds, s, A, n, work);
  return hipGetLastError();
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
  hipLaunchKernelGGL(eig_vectors_kernel, dim3(1), dim3(256), 0, s, work, n, w, k, Q, ldq,
                     desc_cols);
  return hipGetLastError();
}

}  // namespace st
