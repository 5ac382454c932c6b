// Small dense FP64 kernels for the QR fix of Alg. 3: when the new direction v
// fails the orthogonality check against V, [V v] is replaced by Q of its QR
// factorisation and S' by S' R^T, which is no longer an arrow matrix, so its
// SVD is taken densely. All matrices here are (r + 1) x (r + 1), column-major,
// one block per launch: this path runs only on the rare updates whose check
// fires.
//
// The QR factorisation is taken through the Gram G = [V v]^T [V v] = R^T R
// (Cholesky). [V v] is orthonormal up to the small deviation the check
// measured, so G is close to the identity and the Cholesky QR loses nothing
// to its conditioning. The SVD of S' R^T is one-sided Jacobi (Hestenes):
// plane rotations orthogonalise pairs of columns until every pair is
// orthogonal to the working precision; the rotated columns are U Sigma and the
// accumulated rotations V. Its relative accuracy does not depend on the
// spread of the singular values, which here spans from ||X|| down to eps.
#include "common.hpp"
#include "kernels.hpp"

namespace st {

// G = [[Gtop, vte / sqrt(ee)], [vte^T / sqrt(ee), 1]] (n = r + 1): the Gram of
// [V v] with V^T V = Gtop, V^T e = vte, ||e||^2 = ee and v = e / ||e||.
__global__ void qr_gram_fill_kernel(const double *Gtop, int r, const double *vte,
                                    const double *ee, double *G) {
  const int n = r + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx % n, j = idx / n;
  double v;
  if (i < r && j < r) v = Gtop[i + (size_t)r * j];
  else if (i < r) v = vte[i] / sqrt(ee[0]);
  else if (j < r) v = vte[j] / sqrt(ee[0]);
  else v = 1.0;
  G[i + (size_t)n * j] = v;
}

hipError_t launch_qr_gram_fill(const double *Gtop, int r, const double *vte, const double *ee,
                               double *G, hipStream_t s) {
  const int n = r + 1;
  hipLaunchKernelGGL(qr_gram_fill_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s,
                     Gtop, r, vte, ee, G);
  return hipGetLastError();
}

// In place: G (symmetric positive definite) -> R upper triangular with
// G = R^T R; the strict lower triangle is cleared. status[0] = 1 if a pivot
// is not positive (G not positive definite to working precision).
__global__ __launch_bounds__(1024) void chol_upper_kernel(double *G, int n, int *status) {
  __shared__ double piv;
  const int tid = threadIdx.x;
  if (tid == 0) status[0] = 0;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = G[k + (size_t)n * k];
      if (!(d > 0.0)) status[0] = 1;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      G[k + (size_t)n * k] = piv;
    }
    __syncthreads();
    for (int j = k + 1 + tid; j < n; j += blockDim.x) G[k + (size_t)n * j] /= piv;
    __syncthreads();
    // trailing update of the upper triangle: G(i, j) -= R(k, i) R(k, j), k < i <= j
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t % m, j = k + 1 + t / m;
      if (i <= j) G[i + (size_t)n * j] -= G[k + (size_t)n * i] * G[k + (size_t)n * j];
    }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += blockDim.x) {
    const int i = t % n, j = t / n;
    if (i > j) G[t] = 0.0;
  }
}

hipError_t launch_chol_upper(double *G, int n, int *status, hipStream_t s) {
  hipLaunchKernelGGL(chol_upper_kernel, dim3(1), dim3(1024), 0, s, G, n, status);
  return hipGetLastError();
}

// B = S' R^T with S' = [[diag(S), 0], [p^T, q]] (rows: the r old rows in the
// basis of U_d, then the new slice; columns: [V v]) and q = sqrt(ee[0]).
__global__ void arrow_rt_kernel(const double *S, const double *p, const double *ee,
                                const double *R, int r, double *B) {
  const int n = r + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx % n, j = idx / n;
  double v;
  if (i < r) {
    v = S[i] * R[j + (size_t)n * i];  // R(j, i): zero below the diagonal
  } else {
    v = sqrt(ee[0]) * R[j + (size_t)n * r];
    for (int k = j; k < r; ++k) v += p[k] * R[j + (size_t)n * k];
  }
  B[i + (size_t)n * j] = v;
}

hipError_t launch_arrow_rt(const double *S, const double *p, const double *ee, const double *R,
                           int r, double *B, hipStream_t s) {
  const int n = r + 1;
  hipLaunchKernelGGL(arrow_rt_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, S,
                     p, ee, R, r, B);
  return hipGetLastError();
}

// One-sided Jacobi on the columns of A (n x n): A <- A J, W <- J (W = I on
// entry, set here). Sweeps run the round-robin ordering (every pair once per
// sweep, n/2 disjoint pairs per round, one wavefront per pair) until a sweep
// makes no rotation or max_sweeps is reached (status[0] = 2 then).
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(double *A, int n, double *W,
                                                         int max_sweeps, int *status) {
  __shared__ int rotated;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  for (int t = tid; t < n * n; t += blockDim.x) W[t] = (t % (n + 1) == 0) ? 1.0 : 0.0;
  const int m = n + (n & 1);  // an odd n plays against a dummy index n
  const double tol = (double)n * 0x1p-53;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    __syncthreads();
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      for (int pr = wid; pr < m / 2; pr += nw) {
        int a, b;
        if (pr == 0) {
          a = m - 1;
          b = round;
        } else {
          a = (round + pr) % (m - 1);
          b = (round - pr + (m - 1)) % (m - 1);
        }
        if (a >= n || b >= n) continue;
        const int i = a < b ? a : b, j = a < b ? b : a;
        double *ci = A + (size_t)n * i, *cj = A + (size_t)n * j;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int k = lane; k < n; k += 64) {
          const double x = ci[k], y = cj[k];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int k = lane; k < n; k += 64) {
            const double x = ci[k], y = cj[k];
            ci[k] = c * x - sn * y;
            cj[k] = sn * x + c * y;
          }
          double *wi = W + (size_t)n * i, *wj = W + (size_t)n * j;
          for (int k = lane; k < n; k += 64) {
            const double x = wi[k], y = wj[k];
            wi[k] = c * x - sn * y;
            wj[k] = sn * x + c * y;
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  if (tid == 0) status[1] = sweep;
  if (tid == 0 && sweep == max_sweeps) status[0] = 2;
}

hipError_t launch_jacobi_svd(double *A, int n, double *W, int max_sweeps, int *status,
                             hipStream_t s) {
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
  return hipGetLastError();
}

// From the converged Jacobi state: sigma_j = ||A(:, j)||, columns ordered by
// descending sigma (ties by index); U2(:, o) = A(:, j) / sigma_j and
// V2(:, o) = R^{-1} W(:, j) (back substitution), Snew[o] = sigma_j. U2 and V2
// have leading dimension n. sig holds n doubles of workspace.
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(const double *A, const double *W,
                                                            const double *R, int n, double *U2,
                                                            double *V2, double *Snew,
                                                            double *sig) {
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += blockDim.x) {
    double s2 = 0.0;
    for (int k = 0; k < n; ++k) s2 += A[k + (size_t)n * j] * A[k + (size_t)n * j];
    sig[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += blockDim.x) {
    const double sj = sig[j];
    int o = 0;
    for (int l = 0; l < n; ++l) o += (sig[l] > sj || (sig[l] == sj && l < j)) ? 1 : 0;
    Snew[o] = sj;
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    double *u = U2 + (size_t)n * o;
    for (int k = 0; k < n; ++k) u[k] = A[k + (size_t)n * j] * inv;
    double *x = V2 + (size_t)n * o;
    const double *w = W + (size_t)n * j;
    for (int i = n - 1; i >= 0; --i) {
      double acc = w[i];
      for (int k = i + 1; k < n; ++k) acc -= R[i + (size_t)n * k] * x[k];
      x[i] = acc / R[i + (size_t)n * i];
    }
  }
}

hipError_t launch_jacobi_finish(const double *A, const double *W, const double *R, int n,
                                double *U2, double *V2, double *Snew, double *sig,
                                hipStream_t s) {
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(1), dim3(1024), 0, s, A, W, R, n, U2, V2, Snew,
                     sig);
  return hipGetLastError();
}

}  // namespace st
