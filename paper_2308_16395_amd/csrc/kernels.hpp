// Launchers of the streaming-mode and helper kernels (k_isvd.hip).
#pragma once

#include "common.hpp"
#include "secular.hpp"

namespace st {

struct IsvdArgs {
  const double *V;     // old V, column-major
  int64_t ldv;         // its leading dimension (old row count)
  int r;               // columns
  int64_t R;           // rows at the new ranks
  RowMap map;          // new row -> old row
  const double *d;     // [R] new slice projection
  const double *p1;    // [r] (pass 2)
  double *colpart;     // [r * nblocks], column-major
  double *q2part;      // [nblocks] (pass 2)
  double *e1out;       // [R] optional copy of e1 (pass 2)
};

int isvd_blocks(int64_t R, int r);
hipError_t launch_gather3(double *dst, const double *a, int na, int oa, const double *b, int nb,
                          int ob, const double *c, int nc, int oc, hipStream_t s);
hipError_t launch_isvd_pass(int pass, IsvdArgs a, int nblocks, hipStream_t s);
hipError_t launch_colsum(const double *part, int nb, int r, double *out, const double *add,
                         double *out2, const double *q2part, double *q2, hipStream_t s);
// q enters S' as given, or as sqrt(*qsq) read on the device when qsq is not null
hipError_t launch_secular_svd(SecData s, const double *S, const double *p, double q,
                              const double *qsq, int grow, double tol, int ntrip, double *U2,
                              double *V2, double *Snew, hipStream_t st);
hipError_t launch_ud_update(const double *Ud, int64_t ldo, int64_t nd, int r, const double *U2,
                            int c, double *Un, int64_t ldn, hipStream_t s);
hipError_t launch_build_rot_w(const double *U2, const double *V2, int r, int c, int kv,
                              double inv_q, double *Wv, int64_t ldv, float *Wc, int64_t ldc,
                              hipStream_t s);
hipError_t launch_init_vc(const double *A, int64_t R, int64_t nd, const double *Ud,
                          int64_t ldu, int rd, const double *S, double *V, float *Cc,
                          hipStream_t s);
hipError_t launch_new_columns(const double *Q, int64_t n, const double *U, int r, int k,
                              double *W, double *coef, hipStream_t s);
hipError_t launch_append_cols(const double *W, int64_t n, int c0, int k, double *U64, float *Uf,
                              float *Ut, __bf16 *Uh, __bf16 *Ul, int64_t ldb, hipStream_t s);
hipError_t launch_sumsq(const float *x, int64_t count, double *partials, int nblocks,
                        hipStream_t s);
hipError_t launch_ud_row(const double *Ud, int64_t ld, int64_t t, int rd, float *w,
                         hipStream_t s);

hipError_t launch_split_rows(const float *w, int64_t rows, int64_t n, int64_t ldw, __bf16 *hi,
                             __bf16 *lo, int64_t ldb, hipStream_t s);

hipError_t launch_f32_to_f64(const float *x, int64_t n, double *y, hipStream_t s);

// ---- factored streaming mode: V = V0 M ----
// y = M^T x (trans) or M x; M is n x n column-major (ld n). If add is not null
// also y2 = y + add.
hipError_t launch_small_gemv(const double *M, int n, const double *x, int trans, double *y,
                             const double *add, double *y2, hipStream_t s);
// out[row] = scale * ((base ? base[row] : 0) - sum_l V0[row + R l] w[l]) for
// row < R, written as FP64 (out64) or FP32 (out32).
hipError_t launch_vcol(const double *V0, int64_t R, int r, const double *w, const double *base,
                       double scale, double *out64, float *out32, hipStream_t s);
// Mn (c x c, ld c) = blockdiag(M, 1)[0:c, 0:rows] V2[0:rows, 0:c] with M r x r
// (ld r) and V2 (r + 1) x c (ld r + 1); c = r + grow, rows = r + grow.
hipError_t launch_m_update(const double *M, int r, const double *V2, int c, int grow,
                           double *Mn, hipStream_t s);
// dst[row + Rn j] = src[map(row) + ld_src j] (0 for padded rows), j < cols.
hipError_t launch_remap_rows(const double *src, int64_t ld_src, RowMap map, int64_t Rn,
                             int cols, double *dst, hipStream_t s);
// W[m * ldw + k] = M[k + n m] * (S ? S[m] : 1): the row-major rotation matrix of
// V0 -> V0 M diag(S) for the fibre kernels.
hipError_t launch_mt_rows(const double *M, int n, const double *S, double *W, int64_t ldw,
                          hipStream_t s);
hipError_t launch_f64_to_f32(const double *x, int64_t n, float *y, hipStream_t s);
hipError_t launch_identity(double *M, int n, hipStream_t s);
// out[j] = Ud[t + ld j] * S[j], j < rd (row t of U_d S).
hipError_t launch_ud_row64(const double *Ud, int64_t ld, int64_t t, int rd, const double *S,
                           double *out, hipStream_t s);

// V0^T x partials (rows split over blocks, see k_isvd.hip) and the r x r part
// of the two Gram-Schmidt passes with G0 = V0^T V0 maintained.
int gemv_t_blocks(int64_t R);
hipError_t launch_gemv_t(const double *V0, int64_t R, int r, const double *x, double *part,
                         int nb, hipStream_t s);
hipError_t launch_gemv_t_mapped(const double *V, int64_t ldv, const RowMap &map, int64_t R, int r,
                                const double *x, double *part, int nb, hipStream_t s);
hipError_t launch_small_gemm(int transA, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, int m, int n, int k,
                             hipStream_t s);
hipError_t launch_isvd_gram(const double *M, const double *G0, int r, const double *t1,
                            const double *dd, int given, double *p1, double *w1, double *t2,
                            double *p2, double *w2, double *p, double *ws, double *sc,
                            double *g, double *ge, hipStream_t s);
hipError_t launch_g0_update(const double *G0, int r, const double *g, const double *ee, int grow,
                            double *Gn, hipStream_t s);
hipError_t launch_scale_rsqrt(double *x, int64_t n, const double *ss, hipStream_t s);
hipError_t launch_vadd(const double *a, const double *b, int64_t n, double *out, hipStream_t s);
// QR fix of Alg. 3 (k_dense.hip): Gram of [V v], its Cholesky factor R,
// B = S' R^T, one-sided Jacobi SVD of B and the finished U'', V'' = R^{-1} V_B,
// S (descending). status[0]: 0 ok, 1 not positive definite, 2 no convergence;
// status[1]: sweeps taken.
hipError_t launch_qr_gram_fill(const double *Gtop, int r, const double *vte, const double *ee,
                               double *G, hipStream_t s);
hipError_t launch_chol_upper(double *G, int n, int *status, hipStream_t s);
hipError_t launch_arrow_rt(const double *S, const double *p, const double *ee, const double *R,
                           int r, double *B, hipStream_t s);
hipError_t launch_jacobi_svd(double *A, int n, double *W, int max_sweeps, int *status,
                             hipStream_t s);
hipError_t launch_jacobi_finish(const double *A, const double *W, const double *R, int n,
                                double *U2, double *V2, double *Snew, double *sig,
                                hipStream_t s);
// Block updates (k_dense.hip): see the kernels for the layouts.
hipError_t launch_scale_cols_rsqrt(const double *W, int ldw, int rows, int ell, const double *lam,
                                   double *out, hipStream_t s);
hipError_t launch_block_k(const double *S, const double *P, int rd, int b, const double *W, int ldw,
                          const double *lam, int ell, double *K, hipStream_t s);
hipError_t launch_gram_block_fill(const double *Gtop, int rd, const double *VQ, const double *QQ,
                                  int ell, double *G, hipStream_t s);
hipError_t launch_right_mul_rt(double *K, int n, const double *R, int c, hipStream_t s);
hipError_t launch_pad_upper(const double *R, int c, int n, double *Rp, hipStream_t s);
hipError_t launch_ud_update_block(const double *Ud, int64_t ldo, int64_t nd, int rd, int b,
                                  const double *U2, int ldu2, int c, double *Un, int64_t ldn,
                                  hipStream_t s);
hipError_t launch_remap_rows_f32(const float *src, int64_t ld_src, RowMap map, int64_t Rn, int cols,
                                 double *dst, hipStream_t s);
// Symmetric eigendecomposition of small FP64 matrices (k_eig.hip), n <= kEigMaxN:
// tridiagonalise A (lower triangle read) into work (eig_work_elems(n) doubles),
// all eigenvalues ascending into w, then the eigenvectors of the k largest:
// vector c (eigenvalue w[n-1-c]) into column c of Q (desc_cols) or column n-1-c.
// eig_small_supported(n): n in range and its LDS fits the device.
constexpr int kEigMaxN = 128;
size_t eig_work_elems(int n);
bool eig_small_supported(int n);
hipError_t launch_eig_tridiag(const double *A, int n, double *work, hipStream_t s);
hipError_t launch_eig_values(const double *work, int n, double *w, hipStream_t s);
hipError_t launch_eig_vectors(const double *work, int n, const double *w, int k, double *Q,
                              int64_t ldq, int desc_cols, hipStream_t s);
// QR fix of a block from the row appends' SVD (k_dense.hip): A = R V diag(s)
// (R upper, ld c; V ld ldv), and after the Jacobi on A the ordered rotations
// Jp and JpS with the new singular values (c <= kQrOrderMax).
constexpr int kQrOrderMax = 1024;
hipError_t launch_form_rvs(const double *R, int c, const double *V, int ldv, const double *sv,
                           double *A, hipStream_t s);
hipError_t launch_qr_order(const double *A, const double *J, int c, const double *sK,
                           double *Snew, double *Jp, double *JpS, hipStream_t s);
// Block middle-matrix SVD by row appends (k_dense.hip): start, rotated row, finish.
hipError_t launch_block_rows_init(const double *S, int rd, int c, double *VK, int ldv, double *UK,
                                  int ldu, double *sig, hipStream_t s);
hipError_t launch_block_row_z(const double *VK, int ldv, int c, const double *K, int n, int row,
                              double *z, hipStream_t s);
hipError_t launch_block_rows_finish(const double *VK, int ldv, const double *UK, int ldu,
                                    const double *sig, int rd, int b, int c, double *V2,
                                    double *U2, double *Snew, hipStream_t s);
// out[i] = sum over b < nb of part[b * n + i], in a fixed order
hipError_t launch_batch_sum(const double *part, int nb, int64_t n, double *out, hipStream_t s);
// delta = a - b (n rows) and per-block pairs (sum b * delta, sum delta^2) in
// part[2 * nblocks] (reduce with launch_reduce_pairs).
hipError_t launch_delta(const double *a, const double *b, int64_t n, double *delta, double *part,
                        int nblocks, hipStream_t s);

// Message for st_last_error(NULL) after a failed stateless call.
void set_stateless_error(const char *msg);

}  // namespace st
