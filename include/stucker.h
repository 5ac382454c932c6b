/*
 * stucker.h - C ABI of the streaming Tucker (streaming ST-HOSVD) library for
 * AMD MI355X (gfx950).
 *
 * The library keeps a Tucker decomposition X ~ C x_1 U_1 ... x_d U_d of a
 * tensor that grows along its last ("streaming") mode d, one (d-1)-way slice
 * at a time, without storing past slices (paper: De, Li, Kolla, Phipps,
 * "Efficient Computation of Tucker Decomposition for Streaming Scientific
 * Data Compression", Sec. 2.4 problem statement, Sec. 3, Alg. 5).
 *
 * Conventions for every call:
 *  - Return value: ST_OK (0) or a negative ST_E* code. No C++ exception crosses
 *    this boundary. st_last_error() returns a message for the last failure on
 *    that handle (valid until the next call on the handle).
 *  - Tensors are column-major with the first index fastest (Sec. 2.1): a slice
 *    of shape n_1 x ... x n_{d-1} is the flat array Y[i_1 + n_1 (i_2 + n_2 (...))].
 *    A C-contiguous torch tensor of shape (n_{d-1}, ..., n_1) is the same memory.
 *  - Slice inputs are float32 device pointers on the handle's device; the
 *    caller keeps ownership and the library does not retain them.
 *  - Calls are synchronous with respect to the host: when a call returns, its
 *    device work on the handle's stream has finished and the inputs may be
 *    reused. The one exception is st_update (see there). A handle must not be
 *    used from two threads at once.
 *  - Streams: a `stream` argument is a hipStream_t of the HIP runtime this
 *    library links (libamdhip64.so.7), or NULL for that runtime's null stream.
 *    A process may hold a second HIP runtime (for example one bundled with a
 *    Python framework); its stream handles are not valid here and its queued
 *    work is not ordered with this library's: the caller must finish the work
 *    that produces an input (or last used an output buffer) before the call.
 *  - st_update is transactional: on any error the decomposition is unchanged,
 *    and an update whose new singular values fail validation at the next
 *    synchronisation is rolled back before anything else changes (st_update).
 */
#ifndef STUCKER_H
#define STUCKER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ST_MAX_MODES 8

enum st_status {
  ST_OK = 0,
  ST_EINVAL = -1,       /* bad argument (shape, tolerance, pointer, mode index) */
  ST_ENOMEM = -2,       /* device or host allocation failed */
  ST_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  ST_ESTATE = -4,       /* wrong call order (update before init, init twice) */
  ST_ENONFINITE = -5,   /* the input holds NaN or Inf (detected before any change) */
  ST_EDEGENERATE = -6,  /* the initial data is zero: S > 0 cannot hold */
  ST_ESMALL = -7,       /* caller buffer too small; the required size is returned */
  ST_ECAPACITY = -8,    /* a rank exceeded a configured cap */
  ST_ESOLVER = -9       /* a small dense eigensolver reported failure */
};

enum st_precision {
  ST_FP32 = 0,    /* TTM chain and Gram products as FP32 MFMA, FP32 accumulation */
  ST_BF16X3 = 1,  /* the same products as split-BF16 (hi*hi + hi*lo + lo*hi) MFMA */
  ST_FP64 = 2     /* the same products on the FP64 MFMA: FP32 data and state, exact
                     products, FP64 sums (the form that reproduces the FP64 rank
                     decisions; see the header of st_update) */
};
/* In every form V, the partial cores and the slice coordinates d are FP64 and
   the rank tests are taken in FP64. The literal core rotation (FP32 core) runs
   on the FP64 MFMA in ST_FP64 and on the FP32 MFMA in the other two forms, with
   FP32 sums inside each 32-wide block of the contraction and FP64 sums across
   blocks. */

enum st_where { ST_HOST = 0, ST_DEVICE = 1 };

typedef struct st_config {
  int32_t nmodes;              /* d - 1: number of slice modes, 1..ST_MAX_MODES */
  int64_t dims[ST_MAX_MODES];  /* n_1 .. n_{d-1}, each >= 1 */
  double tau;                  /* relative error tolerance (the paper's tau), > 0 */
  int32_t precision;           /* enum st_precision */
  double orth_tol;             /* eps_m of the orthogonality check of Alg. 3 on the new
                                  direction (QR fix when exceeded); 0 = 1e-12 */
  double guard_rel;            /* relative guard band g of the reduced-precision
                                  forms (R9): a slice whose ||E_k|| (Alg. 4) lies
                                  above (1 - g) eps, or whose ISVD residual q
                                  (Alg. 3) lies above (1 - g) eps, has its
                                  decisions and state changes redone from FP64
                                  products; 0 = default (1e-2 FP32, 5e-2
                                  bf16x3); unused by ST_FP64 */
  int64_t max_rank_d;          /* cap on the streaming rank r_d; 0 = no cap */
  void *stream;                /* hipStream_t (of this library's HIP runtime) to
                                  run on; NULL = that runtime's null stream */
  int32_t profile;             /* nonzero: time every kernel group with HIP events */
  int32_t core_update;         /* enum st_core_update */
} st_config;

/* How the core and the auxiliary V are carried between slices.
 * ST_CORE_LITERAL: the last step of Alg. 5 as stated: V and the core C are
 *   both rotated on every slice (C~_(d) = U''^T [C_(d); d^T]); the core keeps
 *   the part of an ignored slice's residual that Alg. 3 drops from V.
 * ST_CORE_FACTORED: the core is C = V x_d S (the Ensure clause of Alg. 5) and V
 *   is kept as the product V0 M of a matrix V0 whose columns are only ever
 *   appended (one per growing slice) and a small orthogonal r_d x r_d matrix M
 *   (the factored ISVD the paper names as future work, Sec. 3.2 and Sec. 6).
 *   Per slice this replaces the two rotations of R x r_d matrices by r_d x r_d
 *   work; rank decisions are the same as with ST_CORE_LITERAL. */
enum st_core_update { ST_CORE_LITERAL = 0, ST_CORE_FACTORED = 1 };

/* Kernel groups timed when st_config.profile is set. */
enum st_kernel_group {
  ST_K_TTM1 = 0,      /* mode-1 projection + residual norm (Alg. 4, first lines) */
  ST_K_TTM = 1,       /* projection + residual norm of modes 2..d-1 */
  ST_K_GRAM = 2,      /* residual Gram (Alg. 1 on E_k) */
  ST_K_EIG = 3,       /* FP64 symmetric eigendecomposition of a Gram */
  ST_K_TTM_EXT = 4,   /* extended projection with [U_k W_k] after growth */
  ST_K_ISVD = 5,      /* the three passes over V that form p, e and q (Alg. 3) */
  ST_K_SVD = 6,       /* secular-equation SVD of S' */
  ST_K_ROT_V = 7,     /* V~ = [V v] V'' (mode-d TTM) */
  ST_K_ROT_C = 8,     /* core update, a mode-d TTM of [C; d] */
  ST_K_UD = 9,        /* U~_d update */
  ST_K_REFINE = 10,   /* FP64-product coordinates of a slice and the ISVD correction
                         sweep (reduced-precision forms, guard band) */
  ST_K_ORTH = 11,     /* Alg. 3's orthogonality check on the new v (growing slices)
                         and its QR fix when the check fires */
  ST_K_GROUPS = 12
};

/* Accumulated timing of one kernel group since the last reset: launches, total
 * device time (ms, from HIP events on the handle's stream), and the algorithmic
 * flops and HBM bytes of those launches (the minimum the operation needs). */
typedef struct st_kernel_profile {
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} st_kernel_profile;

/* Per-slice diagnostics of the last st_update (or of st_init). */
typedef struct st_slice_stats {
  double ynorm;                       /* ||Y||_F */
  double eps;                         /* tau ||Y|| / sqrt(d) (Alg. 5, first step) */
  double e_norm[ST_MAX_MODES];        /* ||E_k||_F of Alg. 4 per slice mode */
  int32_t grew[ST_MAX_MODES];         /* new columns r'_k added to U_k */
  double q;                           /* ||e|| of Alg. 3 */
  int32_t isvd_ignored;               /* 1 if q <= eps (e ignored) */
  int32_t qr_fired;                   /* 1 if the orthogonality check of Alg. 3 fired on
                                         this (growing) slice and its QR fix was applied */
  int32_t guard_hits;                 /* threshold tests re-evaluated with FP64
                                         products (sum of the three refinements) */
  double orth_check;                  /* max_j |V(:,j)^T v| over all columns of V, v the
                                         new unit direction (growing slices; else 0) */
  double delta2;                      /* squared error this slice adds to the bound */
  double ms_total;                    /* wall time of the call, ms */
  double ms_modes;                    /* non-streaming modes (Alg. 4), ms */
  double ms_isvd;                     /* streaming mode (Alg. 3 + core update), ms */
  int32_t refined_modes;              /* 1: a slice mode grew or fell in the guard band,
                                         so every slice mode of this slice was redone
                                         with FP64 products (reduced-precision forms) */
  int32_t refined_isvd;               /* 1: q fell above (1 - g) eps with reduced-
                                         precision coordinates, so d, p and q were
                                         redone from FP64 products */
  int32_t refined_gram;               /* residual Grams redone with FP64 products
                                         because a tail sum of Alg. 1 fell in the
                                         guard band of eps^2 */
  double e_norm_fast[ST_MAX_MODES];   /* ||E_k|| from the form's own products at the
                                         current ranks, before any refinement */
  double q_fast;                      /* q from the form's own products, before any
                                         refinement */
  int64_t qr_total;                   /* QR fixes of Alg. 3 applied since st_init */
} st_slice_stats;

typedef struct st_handle st_handle;

/* Create an empty handle for a d-way stream whose last mode is the streaming
 * (time) mode (the setting of Sec. 3: slices of size n_1 x ... x n_{d-1}
 * arrive one at a time), and allocate its fixed device state (factors U_k at
 * full capacity n_k x n_k, since Alg. 4 only appends columns to them).
 * Ownership: the handle owns all device memory until st_destroy. Errors: ST_EINVAL (bad dims, tau <= 0, nmodes out of range),
 * ST_ENOMEM, ST_EHIP. */
int st_create(const st_config *cfg, st_handle **out);

/* Initial decomposition (Alg. 2, ST-HOSVD with the streaming mode processed
 * last) of x0: device float32, column-major n_1 x ... x n_{d-1} x n_init. Sets
 * S = sqrt of the leading Gram eigenvalues of the last mode and V = A^T U_d S^-1
 * with A the mode-d unfolding of the last partial core (Alg. 1 optional rows,
 * Sec. 3.2), so that C = V x_d S (Assumption 1). Errors: ST_ESTATE (already
 * initialised), ST_EINVAL (n_init < 1), ST_ENONFINITE, ST_EDEGENERATE
 * (||x0|| = 0), ST_ESOLVER, ST_ENOMEM, ST_EHIP. */
int st_init(st_handle *h, const float *x0, int64_t n_init);

/* One streaming update (Alg. 5) with the slice y: device float32, column-major
 * n_1 x ... x n_{d-1}. Runs Alg. 4 for modes 1..d-1, then Alg. 3 on the
 * streaming mode and the core update. Errors: ST_ESTATE (not initialised),
 * ST_ENONFINITE, ST_ECAPACITY, ST_ESOLVER, ST_ENOMEM, ST_EHIP; in every error
 * case the decomposition is unchanged. The call returns once the update is
 * committed (ranks, counters); the tail of its device work (the rotations and
 * the factor update) may still run on the handle's stream, so the next update
 * queues behind it without an idle gap. Every later call on the handle orders
 * after it. y is read only before the first internal synchronisation, so it
 * may be reused when the call returns. The new singular values
 * are validated at the next synchronisation (the next st_update, or any call
 * that reads the decomposition): should one not be positive, that update is
 * rolled back (ranks, counters and the ping-pong halves of the device state
 * return to their values before it, nothing having been overwritten) and the
 * call that found it returns ST_ESOLVER without doing its own work. */
int st_update(st_handle *h, const float *y);

/* Block update: b slices at once (the paper names processing several slices
 * per update as future work, Sec. 6). y holds b slices, device float32,
 * column-major n_1 x ... x n_{d-1} x b (slices in stream order). The
 * per-update tolerance is the block's, eps = tau ||Y_B|| / sqrt(d), which keeps
 * the certified bound of App. D within tau (each update discards at most
 * tau^2 ||Y_B||^2). Alg. 4 runs on the block tensor (the residual Gram of mode k
 * sums over all b slices); the streaming mode generalises Alg. 3: both
 * Gram-Schmidt passes on every slice's core coordinates, the residual block's
 * directions kept by the TruncatedSVD of Alg. 1 (eigenpairs of E^T E, tail rule
 * against eps^2), the middle matrix [[diag S, 0], [P^T, W L^1/2]] with the
 * orthogonality check of [V Q] and its QR fix; its SVD by b secular row
 * appends to [diag S, 0] (after a QR fix [V Q] = Q_f R, K R^T = U_K (R V_K
 * diag(S_K))^T, and a one-sided Jacobi on that nearly orthogonal c x c
 * factor). Both core forms:
 * the literal one rotates V and the core, the factored one (V = V0 M) appends
 * Q to V0 and updates M and V0^T V0. b = 1 is st_update. n_d grows by b;
 * st_stats then reports, per block, q = the norm of the discarded residual
 * directions.
 * Errors: ST_EINVAL (b < 1), the errors of st_update; the decomposition is
 * unchanged on error, as for st_update. */
int st_update_block(st_handle *h, const float *y, int64_t b);

/* Current ranks r_1..r_d (ranks[0..d-1]) of the Tucker decomposition
 * X ~ C x_1 U_1 ... x_d U_d (Sec. 2.2) and the number of slices n_d seen (the
 * row count of U_d, Alg. 5). Host counters only: no synchronisation, so it
 * reports the last update even while its singular values are unvalidated. */
int st_ranks(const st_handle *h, int64_t *ranks, int64_t *n_d);

/* Dense core C (r_1 x ... x r_d, column-major, float32) of the decomposition
 * (Sec. 2.2; the core kept by Alg. 5, or V x_d S in the factored form of
 * Sec. 3.2) into out (host or device pointer per `where`). out == NULL only
 * sets *need (elements).
 * Errors: ST_ESMALL (cap < need; *need is set), ST_ESTATE, ST_EINVAL. */
int st_core(const st_handle *h, float *out, int64_t cap, int64_t *need, int where);

/* The auxiliary tensor V of the core factorization C = V x_d S (Sec. 3.2,
 * Assumption 1(c)) as the column-major float64 matrix V_(d)^T of size
 * (r_1 ... r_{d-1}) x r_d, into out (host or device). V is held in FP64 in
 * every precision form. out == NULL only sets *need.
 * Errors: ST_ESMALL, ST_ESTATE, ST_EINVAL. */
int st_aux_v(const st_handle *h, double *out, int64_t cap, int64_t *need, int where);

/* Dense factor U_mode (Sec. 2.2; mode 0..d-1, orthonormal columns; mode d-1 is
 * the streaming factor of size n_d x r_d that Alg. 3 extends by one row per
 * slice), column-major float64, into out (host or device). out == NULL only
 * sets *rows and *cols. Errors: ST_EINVAL, ST_ESMALL, ST_ESTATE. */
int st_factor(const st_handle *h, int mode, double *out, int64_t cap,
              int64_t *rows, int64_t *cols, int where);

/* The diagonal S (r_d values, descending, positive) of the core factorization
 * C = V x_d S (Sec. 3.2, Assumption 1(c)), i.e. the singular values the ISVD of
 * Alg. 3 maintains, into host memory. Errors: ST_ESMALL (cap < count; *count is
 * set), ST_ESOLVER (a pending update was rolled back, see st_update). */
int st_sv(const st_handle *h, double *s, int64_t cap, int64_t *count);

/* Certified bound on ||X - X^||_F / ||X||_F: sqrt(sum of discarded energy) over
 * ||X||, where the discarded energy is the ST-HOSVD tails at init (Sec. 2.3)
 * plus, per slice, the per-mode residuals of Prop. 3 and q^2 when the ISVD
 * ignores e (Prop. 1, App. D). norm_x = ||X||_F of all data seen. */
int st_recon_error(const st_handle *h, double *rel_bound, double *norm_x);

/* Diagnostics of the last st_update (or st_init): the per-slice tolerance eps
 * and residual norms of Alg. 5 and Alg. 4, q and the orthogonality check of
 * Alg. 3, and the refinements of the reduced-precision forms. Host copy only. */
int st_stats(const st_handle *h, st_slice_stats *out);

/* Slice t (0-based, t < n_d) of the reconstruction C x_1 U_1 ... x_d U_d
 * (the Tucker model of Sec. 2.2: row t of U_d contracted with the core, then
 * modes 1..d-1), written as float32 column-major n_1 x ... x n_{d-1} to the
 * device pointer out. Errors: ST_EINVAL (t out of range), ST_ESTATE. */
int st_reconstruct_slice(const st_handle *h, int64_t t, float *out);

/* Stateless mode-k TTM (Sec. 2.1): out = X x_mode A, for X a dense
 * column-major float32 device tensor of shape dims[0..nmodes-1] and A a float32
 * device matrix of shape rows x dims[mode] stored row-major (equivalently A^T
 * column-major, so a factor U with orthonormal columns passed as `a` gives the
 * projection X x_mode U^T). out is the column-major device tensor with
 * dims[mode] replaced by rows. If norms (host, 2 doubles) is not NULL it
 * receives ||X - (X x_mode A) x_mode A^T||_F^2 and ||X||_F^2 in FP64, the
 * residual and norm of Alg. 4 (rows <= 384 then). precision: enum
 * st_precision. stream: hipStream_t or NULL for the null stream; the call
 * returns after the work has finished. Errors: ST_EINVAL, ST_ENOMEM, ST_EHIP. */
int st_ttm(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode, const float *a,
           int64_t rows, float *out, double *norms, int32_t precision, void *stream);

/* st_ttm for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc). Same
 * arguments, results and errors as st_ttm; it calls no hipMalloc/hipFree and
 * no allocating library routine. Its scratch (the per-block residual-norm
 * partials, their sum, and the FP64 or split-bf16 copy of A for those
 * precisions) lives in one fixed 8 MiB device array per GPU, held until the
 * process ends; a call that would need more (about 2^25 fibres with norms, or
 * rows x dims[mode] above about 10^6 elements in FP64) returns ST_EINVAL with
 * the reason in st_last_error(NULL). Every call on a GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap on one GPU (other
 * host threads, other streams) race and must be serialised by the caller. The
 * array's device address is looked up once per device on the first call. */
int st_ttm_noalloc(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode,
                   const float *a, int64_t rows, float *out, double *norms, int32_t precision,
                   void *stream);

/* Stateless mode-k Gram (Alg. 1, first line) of a dense column-major float32
 * device tensor: G = E_(mode) E_(mode)^T with E = X - (X x_mode A) x_mode A^T
 * (the residual of Alg. 4) when rows > 0, or E = X when rows == 0; A is a
 * rows x dims[mode] row-major float32 device matrix (may be NULL when rows == 0).
 * G is written to the host array g (dims[mode]^2 doubles, column-major).
 * gram_precision: 0 = FP32 products, 1 = bf16x3 products (the residual formed
 * with FP32 products in both; dims[mode] <= 512), 2 = FP64 throughout (the
 * residual formed with FP64 products and kept in FP64; dims[mode] <= 256).
 * rows <= 256. Errors: ST_EINVAL, ST_ENOMEM, ST_EHIP. */
int st_gram(const float *x, int32_t nmodes, const int64_t *dims, int32_t mode, const float *a,
            int64_t rows, double *g, int32_t gram_precision, void *stream);

/* Stateless symmetric eigendecomposition of a small FP64 matrix, the step of
 * Alg. 1 (TruncatedSVD) that follows the Gram: a is an n x n column-major
 * device matrix of which only the lower triangle is read (not modified); w
 * (device, n doubles) receives every eigenvalue in ascending order; q (device,
 * n x k column-major, may be NULL when k == 0) receives orthonormal
 * eigenvectors of the k largest, column c for eigenvalue w[n-1-c]. The
 * library's own kernels (Householder tridiagonalisation, multisection of the
 * Sturm count, inverse iteration), the ones the streaming update uses for its
 * Grams of order <= 128. 1 <= n <= 128, 0 <= k <= n; the call allocates
 * n^2 + 3n doubles of workspace and returns after the work is done.
 * Errors: ST_EINVAL (also when the device cannot hold the matrix in one
 * block's shared memory), ST_ENOMEM, ST_EHIP. */
int st_symeig(const double *a, int64_t n, double *w, double *q, int64_t k, void *stream);

/* ---- Differentiation of the Tucker model (stateless) ----
 *
 * Reconstruct: X^ = G x_1 U_1 ... x_d U_d; Project: G = X x_1 U_1^T ... x_d U_d^T
 * (the multi-TTM form of Sec. 2.1, whose mode-k unfolding is U_k G_(k) K_k^T
 * with K_k the Kronecker product of the other factors). Shapes: dims
 * n_1..n_d, ranks r_1..r_d (1 <= r_k <= n_k, nmodes = d <= ST_MAX_MODES).
 * G has shape r_1 x ... x r_d, X and X^ have shape n_1 x ... x n_d, all
 * column-major float32 device arrays. factors is a host array of d device
 * pointers; U_k is column-major n_k x r_k float32. precision (enum
 * st_precision) selects the product arithmetic of every mode-k TTM and of the
 * factor-gradient contractions (FP32, split-bf16 or FP64 products on the
 * matrix cores; those sums run in FP32 within tiles of 32 fibres and in FP64
 * across them, FP64 throughout for ST_FP64; modes with n_k + r_k above about
 * 1280 take FP64 products). work is a device workspace of at least the
 * size st_tucker_workspace returns (the caller owns it; it holds factor copies
 * and the intermediate partial chains and may be reused across calls on one
 * stream). The work runs on stream (hipStream_t, NULL = null stream) and the
 * call returns after it has finished.
 * Errors: ST_EINVAL (shapes, op, null pointers), ST_ESMALL (work too small),
 * ST_ENOMEM, ST_EHIP. */
enum st_tucker_op { ST_RECONSTRUCT = 0, ST_PROJECT = 1 };

/* Workspace bytes for st_tucker_fwd / st_tucker_bwd with these shapes. */
int st_tucker_workspace(int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                        int32_t precision, int64_t *bytes);

/* Forward: op ST_RECONSTRUCT maps in = G to out = X^; ST_PROJECT maps in = X
 * to out = G. */
int st_tucker_fwd(int32_t op, int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                  const float *in, const float *const *factors, float *out, int32_t precision,
                  void *work, int64_t work_bytes, void *stream);

/* Vector-Jacobian products at (in, factors) for the upstream gradient gout:
 *  ST_RECONSTRUCT (in = G, gout shaped like X^): gin = gout x_1 U_1^T ... x_d U_d^T,
 *    gfactors[k] = (gout x_{j != k} U_j^T)_(k) G_(k)^T;
 *  ST_PROJECT (in = X, gout shaped like G): gin = gout x_1 U_1 ... x_d U_d,
 *    gfactors[k] = (X x_{j != k} U_j^T)_(k) gout_(k)^T.
 * gfactors[k] is a column-major n_k x r_k device array. gin may be NULL, and
 * gfactors (or any entry of it) may be NULL to skip that output. The partial
 * chains are recomputed from a shared prefix, not saved from the forward. */
int st_tucker_bwd(int32_t op, int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                  const float *in, const float *const *factors, const float *gout, float *gin,
                  float *const *gfactors, int32_t precision, void *work, int64_t work_bytes,
                  void *stream);

/* Copy the per-group profile (ST_K_GROUPS entries) into out; reset = 1 also
 * clears the counters. Errors: ST_EINVAL. */
int st_profile(st_handle *h, st_kernel_profile *out, int32_t count, int32_t reset);

/* Free every resource of the handle (NULL is allowed). */
void st_destroy(st_handle *h);

/* Message for the last failure on h (or, when h is NULL, of the last st_create,
 * st_tucker_workspace, st_tucker_fwd or st_tucker_bwd on this thread). */
const char *st_last_error(const st_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* STUCKER_H */
