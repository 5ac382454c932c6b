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
// makes no rotation or max_sweeps is reached (status[0] = 2 then). A wave
// holds its pair's two columns in registers (KR entries per lane, n <= 64 KR;
// KR = 0: any n, columns re-read from memory), takes the three inner products
// with DPP reductions and rotates from the registers.
template <int KR>
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
        if constexpr (KR > 0) {
          double x[KR], y[KR];
#pragma unroll
          for (int q = 0; q < KR; ++q) {
            const int k = lane + 64 * q;
            x[q] = k < n ? ci[k] : 0.0;
            y[q] = k < n ? cj[k] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < KR; ++q) {
            al = fma(x[q], x[q], al);
            be = fma(y[q], y[q], be);
            ga = fma(x[q], y[q], ga);
          }
          al = dpp_wave_sum(al);
          be = dpp_wave_sum(be);
          ga = dpp_wave_sum(ga);
          if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
            double *wi = W + (size_t)n * i, *wj = W + (size_t)n * j;
            double u[KR], v[KR];
#pragma unroll
            for (int q = 0; q < KR; ++q) {
              const int k = lane + 64 * q;
              u[q] = k < n ? wi[k] : 0.0;
              v[q] = k < n ? wj[k] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < KR; ++q) {
              const int k = lane + 64 * q;
              if (k < n) {
                ci[k] = c * x[q] - sn * y[q];
                cj[k] = sn * x[q] + c * y[q];
                wi[k] = c * u[q] - sn * v[q];
                wj[k] = sn * u[q] + c * v[q];
              }
            }
            if (lane == 0) rotated = 1;
          }
        } else {
          for (int k = lane; k < n; k += 64) {
            const double x = ci[k], y = cj[k];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
          al = dpp_wave_sum(al);
          be = dpp_wave_sum(be);
          ga = dpp_wave_sum(ga);
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
  const int kr = (n + 63) / 64;
  if (kr <= 1)
    hipLaunchKernelGGL(jacobi_svd_kernel<1>, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
  else if (kr == 2)
    hipLaunchKernelGGL(jacobi_svd_kernel<2>, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
  else if (kr == 3)
    hipLaunchKernelGGL(jacobi_svd_kernel<3>, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
  else if (kr == 4)
    hipLaunchKernelGGL(jacobi_svd_kernel<4>, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
  else
    hipLaunchKernelGGL(jacobi_svd_kernel<0>, dim3(1), dim3(1024), 0, s, A, n, W, max_sweeps, status);
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

// ---------------------------------------------------------------------------
// Block form of the streaming update (b new slices at once): small kernels
// around the dense middle matrix.
// ---------------------------------------------------------------------------

// out (rows x ell) = W(:, 0:ell) scaled by lam_j^{-1/2} per column (W: ld ldw)
__global__ void scale_cols_rsqrt_kernel(const double *W, int ldw, int rows, int ell,
                                        const double *lam, double *out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ell) return;
  const int i = idx % rows, j = idx / rows;
  out[i + (size_t)rows * j] = W[i + (size_t)ldw * j] / sqrt(lam[j]);
}

hipError_t launch_scale_cols_rsqrt(const double *W, int ldw, int rows, int ell, const double *lam,
                                   double *out, hipStream_t s) {
  if (rows * ell <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_rsqrt_kernel, dim3((unsigned)((rows * ell + 255) / 256)),
                     dim3(256), 0, s, W, ldw, rows, ell, lam, out);
  return hipGetLastError();
}

// The block middle matrix, zero-padded to n x n (n = rd + b):
//   K = [[diag(S), 0], [P^T, W_l Lambda_l^{1/2}]]   ((rd + b) x (rd + l))
// P is rd x b (ld rd), W b x b (ld ldw), lam the eigenvalues (descending).
__global__ void block_k_kernel(const double *S, const double *P, int rd, int b, const double *W,
                               int ldw, const double *lam, int ell, double *K) {
  const int n = rd + b;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx % n, j = idx / n;
  double v = 0.0;
  if (i < rd) {
    if (j == i) v = S[i];
  } else if (j < rd) {
    v = P[j + (size_t)rd * (i - rd)];
  } else if (j < rd + ell) {
    v = W[(i - rd) + (size_t)ldw * (j - rd)] * sqrt(lam[j - rd]);
  }
  K[idx] = v;
}

hipError_t launch_block_k(const double *S, const double *P, int rd, int b, const double *W, int ldw,
                          const double *lam, int ell, double *K, hipStream_t s) {
  const int n = rd + b;
  hipLaunchKernelGGL(block_k_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, S,
                     P, rd, b, W, ldw, lam, ell, K);
  return hipGetLastError();
}

// G (c x c, c = rd + l) = [[Gtop, VQ], [VQ^T, QQ]]: the Gram of [V Q]
__global__ void gram_block_fill_kernel(const double *Gtop, int rd, const double *VQ,
                                       const double *QQ, int ell, double *G) {
  const int c = rd + ell;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx % c, j = idx / c;
  double v;
  if (i < rd && j < rd) v = Gtop[i + (size_t)rd * j];
  else if (i < rd) v = VQ[i + (size_t)rd * (j - rd)];
  else if (j < rd) v = VQ[j + (size_t)rd * (i - rd)];
  else v = QQ[(i - rd) + (size_t)ell * (j - rd)];
  G[idx] = v;
}

hipError_t launch_gram_block_fill(const double *Gtop, int rd, const double *VQ, const double *QQ,
                                  int ell, double *G, hipStream_t s) {
  const int c = rd + ell;
  hipLaunchKernelGGL(gram_block_fill_kernel, dim3((unsigned)((c * c + 255) / 256)), dim3(256), 0,
                     s, Gtop, rd, VQ, QQ, ell, G);
  return hipGetLastError();
}

// In place on K (n x n, ld n): K(:, 0:c) <- K(:, 0:c) R^T for R upper (c x c, ld c);
// one thread per row (each row of K is read before it is written).
__global__ void right_mul_rt_kernel(double *K, int n, const double *R, int c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // (K R^T)(i, j) = sum_{k >= j} K(i, k) R(j, k): ascending j reads only columns >= j
  for (int j = 0; j < c; ++j) {
    double acc = 0.0;
    for (int k = j; k < c; ++k) acc += K[i + (size_t)n * k] * R[j + (size_t)c * k];
    K[i + (size_t)n * j] = acc;
  }
}

hipError_t launch_right_mul_rt(double *K, int n, const double *R, int c, hipStream_t s) {
  hipLaunchKernelGGL(right_mul_rt_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, K, n, R,
                     c);
  return hipGetLastError();
}

// Rpad (n x n) = [[R, 0], [0, I]] for R (c x c, ld c), or the identity (R null)
__global__ void pad_upper_kernel(const double *R, int c, int n, double *Rp) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx % n, j = idx / n;
  double v = (i == j) ? 1.0 : 0.0;
  if (R && i < c && j < c) v = R[i + (size_t)c * j];
  Rp[idx] = v;
}

hipError_t launch_pad_upper(const double *R, int c, int n, double *Rp, hipStream_t s) {
  hipLaunchKernelGGL(pad_upper_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, R, c,
                     n, Rp);
  return hipGetLastError();
}

// U~_d ((nd + b) x c) = [[U_d, 0], [0, I_b]] U'' with U'' ((rd + b) x c, ld ldu2)
__global__ void ud_update_block_kernel(const double *Ud, int64_t ldo, int64_t nd, int rd, int b,
                                       const double *U2, int ldu2, int c, double *Un,
                                       int64_t ldn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = nd + b;
  if (idx >= rows * c) return;
  const int64_t row = idx % rows;
  const int col = (int)(idx / rows);
  const double *u2c = U2 + (size_t)ldu2 * col;
  double acc;
  if (row < nd) {
    acc = 0.0;
    for (int k = 0; k < rd; ++k) acc += Ud[row + ldo * k] * u2c[k];
  } else {
    acc = u2c[rd + (row - nd)];
  }
  Un[row + ldn * col] = acc;
}

hipError_t launch_ud_update_block(const double *Ud, int64_t ldo, int64_t nd, int rd, int b,
                                  const double *U2, int ldu2, int c, double *Un, int64_t ldn,
                                  hipStream_t s) {
  const int64_t total = (nd + b) * c;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(ud_update_block_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     s, Ud, ldo, nd, rd, b, U2, ldu2, c, Un, ldn);
  return hipGetLastError();
}

// SVD of the block middle matrix by row appends. [diag(S), 0] (rd x c,
// c = rd + l), padded with l zero rows, has the SVD I_c diag(S, 0) I_c^T; each
// new row of K is then appended by the secular-equation SVD of a diagonal
// matrix plus one row. Start: VK = I_c (ld ldv), UK(0:c, :) = I_c (ld ldu),
// sig = [S, 0].
__global__ void block_rows_init_kernel(const double *S, int rd, int c, double *VK, int ldv,
                                       double *UK, int ldu, double *sig) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx % c, j = idx / c;
  const double v = (i == j) ? 1.0 : 0.0;
  VK[i + (size_t)ldv * j] = v;
  UK[i + (size_t)ldu * j] = v;
  if (j == 0) sig[i] = (i < rd) ? S[i] : 0.0;
}

hipError_t launch_block_rows_init(const double *S, int rd, int c, double *VK, int ldv, double *UK,
                                  int ldu, double *sig, hipStream_t s) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_rows_init_kernel, dim3((unsigned)((c * c + 255) / 256)), dim3(256), 0,
                     s, S, rd, c, VK, ldv, UK, ldu, sig);
  return hipGetLastError();
}

// z = VK^T k for k = row `row` of K (ld n) over its first c columns: the new
// row in the coordinates of the current right singular vectors. One wave per
// entry of z (a column of VK, read contiguously), summed in a fixed order.
__global__ __launch_bounds__(256) void block_row_z_kernel(const double *VK, int ldv, int c,
                                                          const double *K, int n, int row,
                                                          double *z) {
  const int t = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= c) return;
  double a = 0.0;
  for (int i = lane; i < c; i += 64) a += VK[i + (size_t)ldv * t] * K[row + (size_t)n * i];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) z[t] = a;
}

hipError_t launch_block_row_z(const double *VK, int ldv, int c, const double *K, int n, int row,
                              double *z, hipStream_t s) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_row_z_kernel, dim3((unsigned)((c + 3) / 4)), dim3(256), 0, s, VK, ldv,
                     c, K, n, row, z);
  return hipGetLastError();
}

// The finished factors in the layout of the dense path (ld n2 = rd + b):
// V'' = VK (c x c), U'' rows 0..rd-1 from UK's first rows and rows rd..rd+b-1
// from the appended rows c..c+b-1 (UK's rows rd..c-1 are the padding, zero up
// to rounding: the appended block has rank l), S = sig.
__global__ void block_rows_finish_kernel(const double *VK, int ldv, const double *UK, int ldu,
                                         const double *sig, int rd, int b, int c, double *V2,
                                         double *U2, double *Snew) {
  const int n2 = rd + b;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n2 * c) return;
  const int i = idx % n2, j = idx / n2;
  if (i < c) V2[i + (size_t)n2 * j] = VK[i + (size_t)ldv * j];
  U2[i + (size_t)n2 * j] = UK[(i < rd ? i : c + (i - rd)) + (size_t)ldu * j];
  if (idx < c) Snew[idx] = sig[idx];
}

hipError_t launch_block_rows_finish(const double *VK, int ldv, const double *UK, int ldu,
                                    const double *sig, int rd, int b, int c, double *V2,
                                    double *U2, double *Snew, hipStream_t s) {
  const int total = (rd + b) * c;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_rows_finish_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     s, VK, ldv, UK, ldu, sig, rd, b, c, V2, U2, Snew);
  return hipGetLastError();
}

// A (c x c, ld c) = R V diag(s): R upper triangular (c x c, ld c), V (c x c,
// ld ldv). The QR fix of a block: with K = U_K diag(s) V^T from the row
// appends, K R^T = U_K A^T, and the columns of A are orthogonal up to the
// deviation of [V Q] from orthonormality (a_i^T a_j = s_i s_j v_i^T R^T R v_j).
__global__ void form_rvs_kernel(const double *R, int c, const double *V, int ldv,
                                const double *sv, double *A) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx % c, j = idx / c;
  double acc = 0.0;
  for (int k = i; k < c; ++k) acc += R[i + (size_t)c * k] * V[k + (size_t)ldv * j];
  A[idx] = acc * sv[j];
}

hipError_t launch_form_rvs(const double *R, int c, const double *V, int ldv, const double *sv,
                           double *A, hipStream_t s) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(form_rvs_kernel, dim3((unsigned)((c * c + 255) / 256)), dim3(256), 0, s, R,
                     c, V, ldv, sv, A);
  return hipGetLastError();
}

// After the one-sided Jacobi on A = R V_K diag(sK) (A J has orthogonal columns
// of norms sigma'): K R^T = (U_K J) diag(sigma') (A J diag(1/sigma'))^T, and
// R^{-1} A J = V_K diag(sK) J, so the QR-fixed factors are U'' = U_K Jp and
// V'' = V_K JpS with Jp = J's columns by descending sigma' (ties by index) and
// JpS = diag(sK) Jp diag(1/sigma'). One block of 1024 threads, c <= 1024: the
// column norms one wave per column, the order one thread per column (a NaN
// sorts last, so the order is a permutation whatever the values), then Jp,
// JpS (c x c, ld c) and Snew[0:c].
__global__ __launch_bounds__(1024) void qr_order_kernel(const double *A, const double *J, int c,
                                                        const double *sK, double *Snew,
                                                        double *Jp, double *JpS) {
  __shared__ double sg[kQrOrderMax];
  __shared__ int perm[kQrOrderMax];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  for (int j = wid; j < c; j += nw) {
    double s2 = 0.0;
    for (int k = lane; k < c; k += 64) {
      const double a = A[k + (size_t)c * j];
      s2 += a * a;
    }
    s2 = dpp_wave_sum(s2);
    if (lane == 0) sg[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < c; j += blockDim.x) {
    const double sj = sg[j];
    const double kj = sj == sj ? sj : -1.0;
    int o = 0;
    for (int l = 0; l < c; ++l) {
      const double kl = sg[l] == sg[l] ? sg[l] : -1.0;
      o += (kl > kj || (kl == kj && l < j)) ? 1 : 0;
    }
    perm[o] = j;
    Snew[o] = sj;
  }
  __syncthreads();
  for (int idx = tid; idx < c * c; idx += blockDim.x) {
    const int k = idx % c, j = perm[idx / c];
    const double v = J[k + (size_t)c * j], sj = sg[j];
    Jp[idx] = v;
    JpS[idx] = sj > 0.0 ? sK[k] * v / sj : 0.0;
  }
}

hipError_t launch_qr_order(const double *A, const double *J, int c, const double *sK,
                           double *Snew, double *Jp, double *JpS, hipStream_t s) {
  if (c <= 0) return hipSuccess;
  if (c > kQrOrderMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(qr_order_kernel, dim3(1), dim3(1024), 0, s, A, J, c, sK, Snew, Jp, JpS);
  return hipGetLastError();
}

// dst (Rn x cols, FP64) = src (FP32, old row layout, ld ld_src) through the row map
__global__ void remap_rows_f32_kernel(const float *src, int64_t ld_src, RowMap map, int64_t Rn,
                                      int cols, double *dst) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Rn) return;
  const int64_t o = map_new_to_old(map, row);
  for (int j = 0; j < cols; ++j) dst[row + Rn * j] = (o >= 0) ? (double)src[o + ld_src * j] : 0.0;
}

hipError_t launch_remap_rows_f32(const float *src, int64_t ld_src, RowMap map, int64_t Rn, int cols,
                                 double *dst, hipStream_t s) {
  if (Rn <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(remap_rows_f32_kernel, dim3((unsigned)((Rn + 255) / 256)), dim3(256), 0, s,
                     src, ld_src, map, Rn, cols, dst);
  return hipGetLastError();
}

}  // namespace st
