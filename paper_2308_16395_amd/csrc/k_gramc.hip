// Residual Gram of the mode-1 growth (Alg. 4 with Alg. 1 on E_1) for the
// slice itself: contiguous FP32 fibres of length n <= 128, with the exact
// projection P = U^T X already formed in FP64 by the FP64-product pass that
// precedes every growth decision.
//
// Each wave owns 16 fibres at a time and walks its tiles persistently; nothing
// of E leaves its registers:
//   reconstruction  R^T (16 fibres x 16 rows, per row tile) = P^T U^T on the FP64
//                   MFMA (16x16x4 f64; lane L supplies P(fibre L%16, ranks) and
//                   U(row L%16, ranks) from LDS, and holds R^T[(L/16) + 4v][L%16]),
//   residual        e = x - r in FP64, rounded to FP32: lane L then holds E of row
//                   16 jt + L%16 for the fibres (L/16) + 4 v,
//   Gram            G(I, J) += sum_v E_I[., v] E_J[., v]^T on the FP32 MFMA
//                   (16x16x4 f32): that register layout is exactly its operand
//                   layout (A: row L%16, B: column L%16, K: the four fibres
//                   (L/16) + 4 v of step v), so the lower-triangular tiles of G
//                   accumulate straight from the reconstruction.
// The waves of a block add their tiles in a fixed order in LDS and the block
// writes FP64 partials, summed over blocks by gram_reduce_kernel (deterministic).
#include <algorithm>

#include "k_fiber.hpp"

namespace st {

namespace {

using namespace fk;

__host__ __device__ constexpr int u_pitch(int rq) { return 4 * rq + 1; }  // doubles, odd

template <int JT, int RQ>
__host__ __device__ constexpr size_t gramc_lds_bytes() {
  // U (16 JT rows x 4 RQ ranks, FP64), later reused for the block's tile sums
  const size_t u = (size_t)16 * JT * u_pitch(RQ) * 8;
  const size_t g = (size_t)(JT * (JT + 1) / 2) * 256 * 8;
  return u > g ? u : g;
}

template <int JT, int RQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void gram_contig_kernel(
    const float *__restrict__ x, int64_t F, int n, const double *__restrict__ P, int rows,
    const double *__restrict__ U, int64_t ldu, double *partials, int64_t ntiles) {
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int up = u_pitch(RQ);
  extern __shared__ double lds[];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int col = lane & 15, g = lane >> 4;
  // U(j, m) into LDS, zero past n rows and `rows` ranks
  for (int idx = tid; idx < 16 * JT * 4 * RQ; idx += 256) {
    const int j = idx / (4 * RQ), m = idx - j * (4 * RQ);
    lds[j * up + m] = (j < n && m < rows) ? U[j + ldu * m] : 0.0;
  }
  __syncthreads();

  f32x4 gacc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) gacc[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  const int64_t wave0 = (int64_t)blockIdx.x * 4 + wid, nwaves = (int64_t)gridDim.x * 4;
  // The operands of the next wave tile are loaded while this one is computed
  // (one wave per SIMD: the latency has to be covered inside the wave). A fibre
  // past F, a row past n or a rank past `rows` reads a valid element and is
  // zeroed where consumed (U is zero past `rows` and past n in LDS).
  double pn[RQ];
  float xn[JT][4];
  auto fetch = [&](int64_t t) {
    const int64_t f0 = t * 16;
    const double *pr = P + (f0 + col < F ? f0 + col : 0) * (int64_t)rows;
#pragma unroll
    for (int s = 0; s < RQ; ++s) {
      const int m = 4 * s + g;
      pn[s] = pr[m < rows ? m : rows - 1];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t f = f0 + g + 4 * v;
      const float *xr = x + (f < F ? f : 0) * (int64_t)n;
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        const int j = 16 * jt + col;
        xn[jt][v] = xr[j < n ? j : n - 1];
      }
    }
  };
  if (wave0 < ntiles) fetch(wave0);
  for (int64_t t = wave0; t < ntiles; t += nwaves) {
    const int64_t f0 = t * 16;
    double pa[RQ];
    float xv[JT][4];
#pragma unroll
    for (int s = 0; s < RQ; ++s) pa[s] = pn[s];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
#pragma unroll
      for (int v = 0; v < 4; ++v) xv[jt][v] = xn[jt][v];
    if (t + nwaves < ntiles) fetch(t + nwaves);
    const bool fa = f0 + col < F;
    bool fx[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) fx[v] = f0 + g + 4 * v < F;
#pragma unroll
    for (int s = 0; s < RQ; ++s) pa[s] = fa ? pa[s] : 0.0;
    // reconstruction and residual, JG row tiles at a time: their FP64 MFMA
    // chains interleave, so the matrix core is not left waiting on one chain
    constexpr int JG = JT < 4 ? JT : 4;
    float ev[JT][4];
#pragma unroll
    for (int j0 = 0; j0 < JT; j0 += JG) {
      f64x4 racc[JG];
#pragma unroll
      for (int u = 0; u < JG; ++u) racc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < RQ; ++s)
#pragma unroll
        for (int u = 0; u < JG; ++u)
          if (j0 + u < JT)
            racc[u] = mfma_f64(pa[s], lds[(16 * (j0 + u) + col) * up + 4 * s + g], racc[u]);
#pragma unroll
      for (int u = 0; u < JG; ++u) {
        const int jt = j0 + u;
        if (jt < JT) {
          const bool jok = 16 * jt + col < n;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double xd = (jok && fx[v]) ? (double)xv[jt][v] : 0.0;
            ev[jt][v] = (float)(xd - racc[u][v]);
          }
        }
      }
      // one group's LDS operands at a time (hoisting every group's reads costs
      // more registers than the wave has)
      __builtin_amdgcn_sched_barrier(0);
    }
    // lower-triangular tiles (I >= J) of G, tile index I (I + 1) / 2 + J; the
    // step v runs over all tiles before the next, so consecutive MFMAs are
    // independent
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int I = 0; I < JT; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
          const int q = I * (I + 1) / 2 + J;
          gacc[q] = mfma4(ev[I][v], ev[J][v], gacc[q]);
        }
  }

  // block sum of the tiles in LDS (waves in a fixed order), FP64
  __syncthreads();  // U no longer read
  double *gs = lds;
  for (int w = 0; w < 4; ++w) {
    if (wid == w) {
#pragma unroll
      for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = (4 * g + v) * 16 + col;
          const double val = (double)gacc[q][v];
          gs[q * 256 + e] = (w == 0) ? val : gs[q * 256 + e] + val;
        }
    }
    __syncthreads();
  }
  double *dst = partials + (size_t)blockIdx.x * NT * 256;
  for (int idx = tid; idx < NT * 256; idx += 256) dst[idx] = gs[idx];
}

template <int JT, int RQ>
hipError_t launch_gramc_t(const float *x, int64_t F, int n, const double *P, int rows,
                          const double *U, int64_t ldu, double *partials, int nblocks,
                          hipStream_t s) {
  const size_t lds = gramc_lds_bytes<JT, RQ>();
  const void *fn = (const void *)gram_contig_kernel<JT, RQ>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t ntiles = (F + 15) / 16;
  hipLaunchKernelGGL((gram_contig_kernel<JT, RQ>), dim3((unsigned)nblocks), dim3(256), lds, s, x,
                     F, n, P, rows, U, ldu, partials, ntiles);
  return hipGetLastError();
}

template <int JT>
hipError_t launch_gramc_j(const float *x, int64_t F, int n, const double *P, int rows,
                          const double *U, int64_t ldu, double *partials, int nblocks,
                          hipStream_t s) {
  switch ((rows + 3) / 4) {
    case 1: case 2: case 3: case 4:
      return launch_gramc_t<JT, 4>(x, F, n, P, rows, U, ldu, partials, nblocks, s);
    case 5: case 6: case 7: case 8:
      return launch_gramc_t<JT, 8>(x, F, n, P, rows, U, ldu, partials, nblocks, s);
    case 9: case 10: case 11: case 12:
      return launch_gramc_t<JT, 12>(x, F, n, P, rows, U, ldu, partials, nblocks, s);
    default:
      return launch_gramc_t<JT, 16>(x, F, n, P, rows, U, ldu, partials, nblocks, s);
  }
}

}  // namespace

bool gram_contig_eligible(const FiberIn &in, int rows, GramPrec gp) {
  return !in.x64 && !in.mapped && in.a == 1 && in.n >= 1 && in.n <= 128 && rows >= 1 &&
         rows <= 64 && gp != GramPrec::FP64 && in.F >= 1;
}

hipError_t launch_gram_contig(const FiberIn &in, const double *U, int64_t ldu, int rows,
                              const double *P, double *partials, int nblocks, hipStream_t s) {
  if (!gram_contig_eligible(in, rows, GramPrec::FP32) || P == nullptr || U == nullptr ||
      nblocks < 1)
    return hipErrorInvalidValue;
  const float *x = static_cast<const float *>(in.x);
  const int n = (int)in.n;
  // JT = ceil(n / 16): the tile layout the partial-sum reduction expects
  switch ((n + 15) / 16) {
    case 1: return launch_gramc_j<1>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 2: return launch_gramc_j<2>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 3: return launch_gramc_j<3>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 4: return launch_gramc_j<4>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 5: return launch_gramc_j<5>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 6: return launch_gramc_j<6>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    case 7: return launch_gramc_j<7>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
    default: return launch_gramc_j<8>(x, in.F, n, P, rows, U, ldu, partials, nblocks, s);
  }
}

}  // namespace st
