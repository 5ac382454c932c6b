// Shared definitions for the gfx950 streaming-Tucker kernels and the engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace st {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// Precision of the TTM / Gram contractions: FP32 or split-bf16 MFMA with FP32
// accumulation, or FP64 MFMA (exact products of the FP32 data, FP64 sums).
enum class Prec : int { FP32 = 0, BF16X3 = 1, FP64 = 2 };

// ---------------------------------------------------------------------------
// Wavefront reductions (64 lanes).
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_prod(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v *= __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// The value v holds in lane l (l the same in every lane).
__device__ inline double lane_value(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// v of the lane chosen by the DPP control CTRL (within rows of 16 lanes).
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum (max) over the 64 lanes of a wave with every lane active, the same value
// in every lane and a fixed order: lane swaps within quads, then the mirror
// within half rows and rows (DPP moves, no LDS), then the four row results.
// Faster than wave_sum, whose cross-lane moves go through the LDS crossbar.
__device__ inline double dpp_wave_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ inline double dpp_wave_prod(double v) {
  v *= dpp_move<0xB1>(v);
  v *= dpp_move<0x4E>(v);
  v *= dpp_move<0x141>(v);
  v *= dpp_move<0x140>(v);
  return (lane_value(v, 0) * lane_value(v, 16)) * (lane_value(v, 32) * lane_value(v, 48));
}

__device__ inline double dpp_wave_max(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x141>(v));
  v = fmax(v, dpp_move<0x140>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// Block-wide sum of one double per thread; result valid in every thread.
// `scratch` must hold blockDim.x / 64 doubles.
__device__ inline double block_sum(double v, double *scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  return t;
}

// q = f / a, r = f % a for f, a >= 0, with 32-bit division when both fit (a
// 64-bit division is a long instruction sequence on the GPU).
__device__ inline void divmod_index(int64_t f, int64_t a, int64_t &q, int64_t &r) {
  if (a == 1) {
    q = f;
    r = 0;
  } else if (((uint64_t)f | (uint64_t)a) <= 0xffffffffull) {
    const uint32_t qq = (uint32_t)f / (uint32_t)a;
    q = qq;
    r = f - (int64_t)qq * a;
  } else {
    q = f / a;
    r = f - q * a;
  }
}

// ---------------------------------------------------------------------------
// Mapping of a column-major multi-index between two rank tuples.
//
// After Alg. 4 pads the core and V with zero slices along the slice modes, a
// row index of the mode-d matricization at the new ranks r~ addresses either
// an old row (all i_k < r_k) or a padded (zero) row.
// ---------------------------------------------------------------------------
struct RowMap {
  int nm;                      // number of slice modes
  int identity;                // 1: new index == old index
  int32_t r_old[8];
  int32_t r_new[8];
};

__host__ __device__ inline int64_t map_new_to_old(const RowMap &m, int64_t row) {
  if (m.identity) return row;
  if ((uint64_t)row <= 0xffffffffull) {
    // 32-bit divisions (a 64-bit division is a long instruction sequence on the GPU)
    uint32_t rr = (uint32_t)row, old = 0, stride = 1;
    for (int k = 0; k < m.nm; ++k) {
      const uint32_t rn = (uint32_t)m.r_new[k];
      const uint32_t q = rr / rn, ik = rr - q * rn;
      rr = q;
      if (ik >= (uint32_t)m.r_old[k]) return -1;
      old += ik * stride;
      stride *= (uint32_t)m.r_old[k];
    }
    return (int64_t)old;
  }
  int64_t old = 0, stride = 1;
  for (int k = 0; k < m.nm; ++k) {
    const int64_t rn = m.r_new[k];
    const int64_t ik = row % rn;
    row /= rn;
    if (ik >= m.r_old[k]) return -1;
    old += ik * stride;
    stride *= m.r_old[k];
  }
  return old;
}

// ---------------------------------------------------------------------------
// Launchers (host functions; each enqueues kernels on `stream`).
// ---------------------------------------------------------------------------

// Addressing of a tensor viewed as `F` fibres of length `n`:
//  STRIDED: fibre f = i + a*l (i < a) starts at (f % a) + a*n*(f / a);
//           element j sits at base + a*j. (a = 1: contiguous fibres.)
//  MAPPED : fibre f starts at map(f) (or is all-zero if map(f) < 0); element
//           j at base + a*j, and element j == n (one extra element) is taken
//           from `extra[f]` by the rotations.
// The elements are FP32 (x64 = 0) or FP64 (x64 = 1).
struct FiberIn {
  const void *x;
  int x64;
  int64_t a;        // element stride
  int64_t n;        // fibre length (without the extra element)
  int64_t F;        // number of fibres
  int mapped;       // 0: STRIDED, 1: MAPPED
  RowMap map;
  const double *extra;  // MAPPED only: optional element n of every fibre
};

// Output P[f][m] of a fibre contraction at (f % ao) + ao*m + ao*mo*(f / ao),
// FP32 (o64 = 0) or FP64 (o64 = 1).
struct FiberOut {
  void *p;
  int o64;
  int64_t ao;
  int64_t mo;
};

// P[f][m] = sum_j X[f][j] * W[m][j] for m in [m0, m0 + mcount); W is row-major
// with leading dimension ldw over j. When `resid_partials` is not null
// (STRIDED only, m0 = 0, mcount = all rows of W), also computes
// E = X - P x W^T per fibre and writes per-block FP64 partial sums
// {sum E^2, sum X^2} to resid_partials[2 * block].
// `w_hi`/`w_lo` are the bf16 splits of W (row-major, ld = ldw_bf) for BF16X3;
// `w64` its FP64 form (ld = ldw) for Prec::FP64.
struct FiberW {
  const float *w;
  int64_t ldw;
  const __bf16 *w_hi;
  const __bf16 *w_lo;
  int64_t ldw_bf;
  const double *w64;
};

// Input/output element types: FP32 -> FP32, FP32 -> FP64 and FP64 -> FP64.
// resid_partials must hold 2 * fiber_max_blocks(in.F) doubles; `nparts`
// (optional) receives the number of blocks that wrote a pair.
int fiber_max_blocks(int64_t F);
hipError_t launch_fiber_project(const FiberIn &in, const FiberW &w, int m0, int mcount,
                                const FiberOut &out, double *resid_partials, Prec prec,
                                hipStream_t s, int *nparts = nullptr);

// The contiguous-fibre special case of launch_fiber_project (FP32 slice,
// a == 1, all rows from 0, n <= 128, n % 4 == 0, at most 64 rows, FP32 or
// split-bf16 products): a persistent kernel that streams 64-fibre tiles
// through LDS. launch_fiber_project takes it whenever it is eligible.
bool ttm_contig_eligible(const FiberIn &in, int m0, int mcount, const FiberOut &out, Prec prec,
                         bool resid);
hipError_t launch_ttm_contig(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                             double *partials, Prec prec, hipStream_t s, int *nparts);

// Mode-d rotation (MAPPED input) with FP64 products and sums:
// P[f][m] = sum_k X'[f][k] W[m][k] (W row-major, ld ldw), X'[f][k] = X[f][k]
// for k < n; element n: none (extra_mode 0), extra[f] (1), or
// extra[f] - sum_{k<n} X[f][k] pvec[k] formed in FP64 (2).
// `w64` selects FP64 X, W and P; otherwise all three are FP32 (the output is
// rounded once). With `f32m` (FP32 only) the products run on the FP32 MFMA with
// FP32 sums inside each 32-wide K block and FP64 sums across blocks.
hipError_t launch_rot64(const FiberIn &in, const void *w, int w64, int64_t ldw, int m0,
                        int mcount, const FiberOut &out, int extra_mode, const double *pvec,
                        hipStream_t s, int f32m = 0);

// Gram of the residual E = X - (X x W^T) x W (or of X itself when rows == 0)
// over all fibres, summed in FP64 in a fixed order into G (n x n,
// column-major; when G is null only the per-block partials of the
// lower-triangular 16x16 tiles are written, for launch_gram_reduce). The
// residual is formed with FP64 products when `e64` (W.w64 must be set), else
// with FP32 products; the Gram products use `gp` (FP64: E kept in FP64; when E
// of all n rows does not fit LDS, the Gram is formed over pairs of 128-row
// chunks and G must be given). `partials` holds gram_partial_elems doubles.
enum class GramPrec : int { FP32 = 0, BF16X3 = 1, FP64 = 2 };
// Mode-1 residual Gram of contiguous FP32 fibres (n <= 128, rows <= 64, FP32 or
// bf16x3 Gram precision) from the exact FP64 projection P (F x rows, fibre-major,
// ld rows) and U (FP64, n x rows, ld ldu): per-block partials as launch_gram's
// (k_gramc.hip); reduce them with launch_gram_reduce.
bool gram_contig_eligible(const FiberIn &in, int rows, GramPrec gp);
hipError_t launch_gram_contig(const FiberIn &in, const double *U, int64_t ldu, int rows,
                              const double *P, double *partials, int nblocks, hipStream_t s);
int gram_blocks(int64_t F, int64_t n, GramPrec gp);
size_t gram_partial_elems(int64_t n, int nblocks, GramPrec gp);
hipError_t launch_gram(const FiberIn &in, const FiberW &w, int rows, double *partials,
                       int nblocks, GramPrec gp, bool e64, hipStream_t s, double *G);
hipError_t launch_gram_reduce(const double *partials, int nblocks, int64_t n, double *G,
                              hipStream_t s);

// Sum `count` pairs of FP64 partials into out[0], out[1] (fixed order).
hipError_t launch_reduce_pairs(const double *partials, int count, double *out, hipStream_t s);

// Typed fibre launchers (one translation unit each).
hipError_t launch_fiber_ff(const FiberIn &in, const FiberW &w, int m0, int mcount,
                           const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                           int *nparts);
hipError_t launch_fiber_fd(const FiberIn &in, const FiberW &w, int m0, int mcount,
                           const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                           int *nparts);
hipError_t launch_fiber_dd(const FiberIn &in, const FiberW &w, int m0, int mcount,
                           const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                           int *nparts);

}  // namespace st
