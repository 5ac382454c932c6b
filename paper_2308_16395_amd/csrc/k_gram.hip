// Gram of the mode-k residual (Alg. 1 applied to E_k of Alg. 4) and the
// fixed-order FP64 reductions; also the element-type dispatch of the fibre
// projections.
//
// Each block iterates over 64-fibre tiles; every wave forms E^T for its 16
// fibres (all n rows) into LDS, then the waves accumulate their share of the
// lower-triangular 16x16 tiles of G = sum_f e_f e_f^T. Per-block partials are
// summed in a fixed order, so G is deterministic.
#include <algorithm>

#include "k_fiber.hpp"

namespace st {

namespace {

using namespace fk;

constexpr int kGramTPW = 16;  // max tiles per wave per launch group

__host__ __device__ inline void tile_ij(int t, int &ti, int &tj) {
  // t enumerates the lower triangle row by row: (0,0), (1,0), (1,1), (2,0)...
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

template <int GP>
using ElemT = typename std::conditional<GP == 2, double, float>::type;
template <int GP>
constexpr int lde() {
  return GP == 2 ? 65 : 68;  // LDS row stride of E (elements)
}

// Four consecutive elements j0 .. j0 + 3 of one fibre (zero past n or for an
// absent fibre).
template <bool CONTIG, class TIN>
__device__ inline void load_x4(const FiberIn &in, int64_t base, int64_t j0, double (&x)[4]) {
  const TIN *xp = cptr<TIN>(in.x);
  if constexpr (CONTIG && std::is_same<TIN, float>::value) {
    if (base >= 0 && j0 + 4 <= in.n) {
      const f32x4 u = *reinterpret_cast<const f32x4 *>(xp + base + j0);
      x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t j = j0 + v;
    x[v] = (double)load_or0(xp, base + in.a * j, base >= 0 && j < in.n);
  }
}

// GP: product precision of the Gram, 0 = FP32, 1 = bf16x3, 2 = FP64 (E held
// in FP64, exact products). PE: precision of the residual recomputation
// (0 = FP32 products, 2 = FP64 products).
template <int MT, bool CONTIG, int GP, int PE, class TIN>
__global__ __launch_bounds__(kThreads) void gram_kernel(FiberIn in, FiberW w, int rows,
                                                        double *partials, int ntiles) {
  using ET = ElemT<GP>;
  constexpr int LDE = lde<GP>();
  extern __shared__ double es_raw[];
  ET *es = reinterpret_cast<ET *>(es_raw);  // [n_pad][LDE]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t n = in.n;
  const int jtiles = (int)((n + 15) / 16);
  const int group0 = blockIdx.y * 4 * kGramTPW;
  const TIN *xp = cptr<TIN>(in.x);

  AccT<GP == 2 ? 2 : 0> gacc[kGramTPW];
  int tI[kGramTPW], tJ[kGramTPW];
#pragma unroll
  for (int q = 0; q < kGramTPW; ++q) {
    gacc[q] = AccT<GP == 2 ? 2 : 0>{0, 0, 0, 0};
    const int t = group0 + wid + 4 * q;
    if (t < ntiles) {
      tile_ij(t, tI[q], tJ[q]);
    } else {
      tI[q] = -1;
      tJ[q] = -1;
    }
  }

  const int64_t ftiles = (in.F + 63) / 64;
  for (int64_t it = blockIdx.x; it < ftiles; it += gridDim.x) {
    const int64_t fw = it * 64 + wid * 16;
    const int64_t base[1] = {fiber_base(in, fw + col)};
    if (rows > 0) {
      AccT<PE> acc[MT][1];
      double dummy = 0.0;
      project_wave<MT, 1, CONTIG, PE, false, TIN>(in, w, 0, rows, base, acc, dummy);
      for (int jt = 0; jt < jtiles; ++jt) {
        AccT<PE> racc[1];
        recon_tile<MT, 1, PE>(w, rows, n, jt, acc, racc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = 16 * jt + acc_row<PE>(grp, v);
          const double x = (double)load_or0(xp, base[0] + in.a * j, base[0] >= 0 && j < n);
          es[j * LDE + wid * 16 + col] = (ET)(x - (double)racc[0][v]);
        }
      }
    } else {
      for (int jt = 0; jt < jtiles; ++jt) {
        double xv[4];
        load_x4<CONTIG, TIN>(in, base[0], 16 * jt + 4 * grp, xv);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          es[(16 * jt + 4 * grp + v) * LDE + wid * 16 + col] = (ET)xv[v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGramTPW; ++q) {
      if (tI[q] < 0) continue;
      const ET *ra = es + (16 * tI[q] + col) * LDE;
      const ET *rb = es + (16 * tJ[q] + col) * LDE;
#pragma unroll
      for (int kb = 0; kb < 64; kb += 32) {
        if constexpr (GP == 2) {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            gacc[q] = mfma_f64(ra[kb + 8 * grp + s], rb[kb + 8 * grp + s], gacc[q]);
        } else {
          float av[8], bv[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            av[s] = ra[kb + 8 * grp + s];
            bv[s] = rb[kb + 8 * grp + s];
          }
          if constexpr (GP == 0) {
#pragma unroll
            for (int s = 0; s < 8; ++s) gacc[q] = mfma4(av[s], bv[s], gacc[q]);
          } else {
            bf16x8 ah, al, bh, bl;
            split8(av, ah, al);
            split8(bv, bh, bl);
            gacc[q] = mfma_bf(ah, bh, gacc[q]);
            gacc[q] = mfma_bf(ah, bl, gacc[q]);
            gacc[q] = mfma_bf(al, bh, gacc[q]);
          }
        }
      }
    }
    __syncthreads();
  }
  // partials[block][tile][16*16]
#pragma unroll
  for (int q = 0; q < kGramTPW; ++q) {
    if (tI[q] < 0) continue;
    const int t = group0 + wid + 4 * q;
    double *dst = partials + ((size_t)blockIdx.x * ntiles + t) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      dst[acc_row<GP == 2 ? 2 : 0>(grp, v) * 16 + col] = (double)gacc[q][v];
  }
}

// ---------------------------------------------------------------------------
// FP64 Gram for fibres too long to hold E in LDS: rows are split into chunks
// of kChunk and the Gram is formed one chunk pair (I >= J) at a time, with E of
// both chunks in LDS (the projection is recomputed per fibre tile and pass).
// ---------------------------------------------------------------------------
constexpr int kChunk = 128;        // rows per chunk (8 tiles)
constexpr int kChunkT = kChunk / 16;

template <int MT, bool CONTIG, int PE, class TIN>
__global__ __launch_bounds__(kThreads) void gram_pair_kernel(FiberIn in, FiberW w, int rows,
                                                             int64_t i0, int64_t j0,
                                                             double *partials) {
  constexpr int LDE = lde<2>();
  extern __shared__ double es2[];
  double *esI = es2;                    // [kChunk][LDE]
  double *esJ = es2 + kChunk * LDE;     // [kChunk][LDE] (unused when i0 == j0)
  const bool same = i0 == j0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t n = in.n;
  const TIN *xp = cptr<TIN>(in.x);
  const int ntl = same ? kChunkT * (kChunkT + 1) / 2 : kChunkT * kChunkT;
  f64x4 gacc[16];
  int tI[16], tJ[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    gacc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int t = wid + 4 * q;
    if (t < ntl) {
      if (same) {
        tile_ij(t, tI[q], tJ[q]);
      } else {
        tI[q] = t / kChunkT;
        tJ[q] = t % kChunkT;
      }
    } else {
      tI[q] = -1;
      tJ[q] = -1;
    }
  }
  const int64_t ftiles = (in.F + 63) / 64;
  for (int64_t it = blockIdx.x; it < ftiles; it += gridDim.x) {
    const int64_t fw = it * 64 + wid * 16;
    const int64_t base[1] = {fiber_base(in, fw + col)};
    if (rows > 0) {
      AccT<PE> acc[MT][1];
      double dummy = 0.0;
      project_wave<MT, 1, CONTIG, PE, false, TIN>(in, w, 0, rows, base, acc, dummy);
      for (int h = 0; h < (same ? 1 : 2); ++h) {
        const int64_t c0 = h == 0 ? i0 : j0;
        double *es = h == 0 ? esI : esJ;
        for (int lt = 0; lt < kChunkT; ++lt) {
          const int jt = (int)(c0 / 16) + lt;
          AccT<PE> racc[1];
          recon_tile<MT, 1, PE>(w, rows, n, jt, acc, racc);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t j = 16 * (int64_t)jt + acc_row<PE>(grp, v);
            const double x = (double)load_or0(xp, base[0] + in.a * j, base[0] >= 0 && j < n);
            es[(j - c0) * LDE + wid * 16 + col] = (j < n) ? x - (double)racc[0][v] : 0.0;
          }
        }
      }
    } else {
      for (int h = 0; h < (same ? 1 : 2); ++h) {
        const int64_t c0 = h == 0 ? i0 : j0;
        double *es = h == 0 ? esI : esJ;
        for (int lt = 0; lt < kChunkT; ++lt) {
          double xv[4];
          load_x4<CONTIG, TIN>(in, base[0], c0 + 16 * lt + 4 * grp, xv);
#pragma unroll
          for (int v = 0; v < 4; ++v) es[(16 * lt + 4 * grp + v) * LDE + wid * 16 + col] = xv[v];
        }
      }
    }
    __syncthreads();
    const double *eJ = same ? esI : esJ;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (tI[q] < 0) continue;
      const double *ra = esI + (16 * tI[q] + col) * LDE;
      const double *rb = eJ + (16 * tJ[q] + col) * LDE;
#pragma unroll
      for (int kb = 0; kb < 64; kb += 32)
#pragma unroll
        for (int s = 0; s < 8; ++s)
          gacc[q] = mfma_f64(ra[kb + 8 * grp + s], rb[kb + 8 * grp + s], gacc[q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (tI[q] < 0) continue;
    const int t = wid + 4 * q;
    double *dst = partials + ((size_t)blockIdx.x * ntl + t) * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[acc_row<2>(grp, v) * 16 + col] = gacc[q][v];
  }
}

__global__ void gram_pair_reduce_kernel(const double *partials, int nblocks, int64_t i0,
                                        int64_t j0, int64_t n, double *G) {
  const bool same = i0 == j0;
  const int ntl = same ? kChunkT * (kChunkT + 1) / 2 : kChunkT * kChunkT;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ntl * 256) return;
  const int t = (int)(idx / 256), e = (int)(idx % 256);
  int ti, tj;
  if (same) {
    tile_ij(t, ti, tj);
  } else {
    ti = t / kChunkT;
    tj = t % kChunkT;
  }
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partials[((size_t)b * ntl + t) * 256 + e];
  const int64_t i = i0 + 16 * ti + e / 16, j = j0 + 16 * tj + e % 16;
  if (i < n && j < n) {
    G[i + n * j] = s;
    G[j + n * i] = s;
  }
}

// G from the per-block tile partials: a block takes 16 consecutive elements of
// the tile sequence and 16 groups of partial blocks (thread (e, q) sums blocks
// q, q + 16, ... with four interleaved accumulators, so its loads are in flight
// together); the 16 group sums meet in LDS in a fixed order (deterministic).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double *partials, int nblocks,
                                                          int ntiles, int64_t n, double *G) {
  __shared__ double red[16][17];
  const int el = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int64_t idx = (int64_t)blockIdx.x * 16 + el;
  const int64_t total = (int64_t)ntiles * 256;
  const bool ok = idx < total;
  const size_t stride = (size_t)ntiles * 256;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (ok) {
    int b = q, u = 0;
    for (; b + 48 < nblocks; b += 64) {
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] += partials[(size_t)(b + 16 * c) * stride + idx];
    }
    for (; b < nblocks; b += 16, u = (u + 1) & 3) a[u] += partials[(size_t)b * stride + idx];
  }
  red[q][el] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  if (q == 0 && ok) {
    double s = 0.0;
    for (int g = 0; g < 16; ++g) s += red[g][el];
    const int t = (int)(idx / 256), e = (int)(idx % 256);
    int ti, tj;
    tile_ij(t, ti, tj);
    const int64_t i = 16 * ti + e / 16, j = 16 * tj + e % 16;
    if (i < n && j < n) {
      G[i + n * j] = s;
      G[j + n * i] = s;
    }
  }
}

__global__ void reduce_pairs_kernel(const double *partials, int count, double *out) {
  __shared__ double scratch[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  a = block_sum(a, scratch);
  b = block_sum(b, scratch);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

size_t gram_lds(int64_t n, int gp) {
  const int64_t jt = (n + 15) / 16;
  return gp == 2 ? (size_t)jt * 16 * lde<2>() * sizeof(double)
                 : (size_t)jt * 16 * lde<0>() * sizeof(float);
}

template <int MT, bool CONTIG, int GP, int PE, class TIN>
hipError_t launch_gram_k(const FiberIn &in, const FiberW &w, int rows, double *partials,
                         int nblocks, hipStream_t s) {
  const int jt = (int)((in.n + 15) / 16);
  const int ntiles = jt * (jt + 1) / 2;
  const int groups = (ntiles + 4 * kGramTPW - 1) / (4 * kGramTPW);
  const size_t lds = gram_lds(in.n, GP);
  const void *fn = (const void *)gram_kernel<MT, CONTIG, GP, PE, TIN>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((gram_kernel<MT, CONTIG, GP, PE, TIN>), dim3((unsigned)nblocks,
                     (unsigned)groups), dim3(kThreads), lds, s, in, w, rows, partials, ntiles);
  return hipGetLastError();
}

template <int MT, bool CONTIG, int PE, class TIN>
hipError_t launch_gram_g(const FiberIn &in, const FiberW &w, int rows, double *partials,
                         int nblocks, int gp, hipStream_t s) {
  if (gp == 2) return launch_gram_k<MT, CONTIG, 2, PE, TIN>(in, w, rows, partials, nblocks, s);
  if (gp == 1) return launch_gram_k<MT, CONTIG, 1, PE, TIN>(in, w, rows, partials, nblocks, s);
  return launch_gram_k<MT, CONTIG, 0, PE, TIN>(in, w, rows, partials, nblocks, s);
}

template <int MT, class TIN>
hipError_t launch_gram_t(const FiberIn &in, const FiberW &w, int rows, double *partials,
                         int nblocks, bool contig, int gp, bool e64, hipStream_t s) {
  if constexpr (std::is_same<TIN, float>::value) {
    if (contig) {
      if (e64) return launch_gram_g<MT, true, 2, TIN>(in, w, rows, partials, nblocks, gp, s);
      return launch_gram_g<MT, true, 0, TIN>(in, w, rows, partials, nblocks, gp, s);
    }
  }
  if (e64) return launch_gram_g<MT, false, 2, TIN>(in, w, rows, partials, nblocks, gp, s);
  return launch_gram_g<MT, false, 0, TIN>(in, w, rows, partials, nblocks, gp, s);
}

template <class TIN>
hipError_t launch_gram_typed(const FiberIn &in, const FiberW &w, int rows, double *partials,
                             int nblocks, int gp, bool e64, hipStream_t s) {
  const bool contig = contiguous(in);
  const int tiles = (rows + 15) / 16;
  if (tiles <= 1) return launch_gram_t<1, TIN>(in, w, rows, partials, nblocks, contig, gp, e64, s);
  if (tiles <= 2) return launch_gram_t<2, TIN>(in, w, rows, partials, nblocks, contig, gp, e64, s);
  if (tiles <= 4) return launch_gram_t<4, TIN>(in, w, rows, partials, nblocks, contig, gp, e64, s);
  if (tiles <= 8) return launch_gram_t<8, TIN>(in, w, rows, partials, nblocks, contig, gp, e64, s);
  if (tiles <= 16)
    return launch_gram_t<16, TIN>(in, w, rows, partials, nblocks, contig, gp, e64, s);
  return hipErrorInvalidValue;
}

template <int MT, bool CONTIG, int PE, class TIN>
hipError_t launch_gram_pairs_k(const FiberIn &in, const FiberW &w, int rows, double *partials,
                               int nblocks, double *G, hipStream_t s) {
  const size_t lds = (size_t)2 * kChunk * lde<2>() * sizeof(double);
  const void *fn = (const void *)gram_pair_kernel<MT, CONTIG, PE, TIN>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t nch = (in.n + kChunk - 1) / kChunk;
  for (int64_t I = 0; I < nch; ++I)
    for (int64_t J = 0; J <= I; ++J) {
      hipLaunchKernelGGL((gram_pair_kernel<MT, CONTIG, PE, TIN>), dim3((unsigned)nblocks),
                         dim3(kThreads), lds, s, in, w, rows, I * kChunk, J * kChunk, partials);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int ntl = (I == J) ? kChunkT * (kChunkT + 1) / 2 : kChunkT * kChunkT;
      hipLaunchKernelGGL(gram_pair_reduce_kernel, dim3((unsigned)((ntl * 256 + 255) / 256)),
                         dim3(256), 0, s, partials, nblocks, I * kChunk, J * kChunk, in.n, G);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

template <int MT, class TIN>
hipError_t launch_gram_pairs_t(const FiberIn &in, const FiberW &w, int rows, double *partials,
                               int nblocks, bool contig, bool e64, double *G, hipStream_t s) {
  if constexpr (std::is_same<TIN, float>::value) {
    if (contig) {
      if (e64) return launch_gram_pairs_k<MT, true, 2, TIN>(in, w, rows, partials, nblocks, G, s);
      return launch_gram_pairs_k<MT, true, 0, TIN>(in, w, rows, partials, nblocks, G, s);
    }
  }
  if (e64) return launch_gram_pairs_k<MT, false, 2, TIN>(in, w, rows, partials, nblocks, G, s);
  return launch_gram_pairs_k<MT, false, 0, TIN>(in, w, rows, partials, nblocks, G, s);
}

template <class TIN>
hipError_t launch_gram_pairs_typed(const FiberIn &in, const FiberW &w, int rows,
                                   double *partials, int nblocks, bool e64, double *G,
                                   hipStream_t s) {
  const bool contig = contiguous(in);
  const int tiles = (rows + 15) / 16;
  if (tiles <= 1)
    return launch_gram_pairs_t<1, TIN>(in, w, rows, partials, nblocks, contig, e64, G, s);
  if (tiles <= 2)
    return launch_gram_pairs_t<2, TIN>(in, w, rows, partials, nblocks, contig, e64, G, s);
  if (tiles <= 4)
    return launch_gram_pairs_t<4, TIN>(in, w, rows, partials, nblocks, contig, e64, G, s);
  if (tiles <= 8)
    return launch_gram_pairs_t<8, TIN>(in, w, rows, partials, nblocks, contig, e64, G, s);
  if (tiles <= 16)
    return launch_gram_pairs_t<16, TIN>(in, w, rows, partials, nblocks, contig, e64, G, s);
  return hipErrorInvalidValue;
}

}  // namespace

// one 64-fibre block per 64 fibres at most (launches with two fibre tiles per
// wave use half as many)
int fiber_max_blocks(int64_t F) { return (int)((F + 63) / 64); }

hipError_t launch_fiber_project(const FiberIn &in, const FiberW &w, int m0, int mcount,
                                const FiberOut &out, double *resid_partials, Prec prec,
                                hipStream_t s, int *nparts) {
  if (in.mapped && resid_partials != nullptr) return hipErrorInvalidValue;
  if (prec == Prec::FP64 && w.w64 == nullptr) return hipErrorInvalidValue;
  if (prec == Prec::BF16X3 && (w.w_hi == nullptr || w.w_lo == nullptr))
    return hipErrorInvalidValue;
  if (prec == Prec::FP32 && w.w == nullptr) return hipErrorInvalidValue;
  // Split-bf16 products pay off only where the contraction is MFMA-bound on
  // FP32 data. Over an FP64 partial core (modes 2..d-1) the kernels are bound
  // by the 8-byte input and the per-element splits cost VALU time for nothing
  // (measured: 76 vs 30 us per mode at 128^3 x 16); they take FP32 products,
  // whose rounding (2^-24 relative per product) is that of bf16x3.
  if (prec == Prec::BF16X3 && in.x64 && w.w != nullptr) prec = Prec::FP32;
  if (ttm_contig_eligible(in, m0, mcount, out, prec, resid_partials != nullptr))
    return launch_ttm_contig(in, w, mcount, out, resid_partials, prec, s, nparts);
  if (!in.x64 && !out.o64)
    return launch_fiber_ff(in, w, m0, mcount, out, resid_partials, prec, s, nparts);
  if (!in.x64 && out.o64)
    return launch_fiber_fd(in, w, m0, mcount, out, resid_partials, prec, s, nparts);
  if (in.x64 && out.o64)
    return launch_fiber_dd(in, w, m0, mcount, out, resid_partials, prec, s, nparts);
  return hipErrorInvalidValue;  // FP64 -> FP32 is not a path of the update
}

static bool gram_uses_pairs(int64_t n, GramPrec gp) {
  return gp == GramPrec::FP64 && gram_lds(n, 2) > 160 * 1024;
}

static int64_t gram_tiles(int64_t n, GramPrec gp) {
  if (gram_uses_pairs(n, gp)) return kChunkT * kChunkT;  // per chunk pair
  const int64_t jt = (n + 15) / 16;
  return jt * (jt + 1) / 2;
}

int gram_blocks(int64_t F, int64_t n, GramPrec gp) {
  // at most 512 blocks, and partials of at most 64 MB
  const int64_t t = (F + 63) / 64;
  const int64_t by_mem = std::max<int64_t>(16, (64ll << 20) / (gram_tiles(n, gp) * 256 * 8));
  return (int)std::max<int64_t>(1, std::min<int64_t>({t, (int64_t)512, by_mem}));
}

size_t gram_partial_elems(int64_t n, int nblocks, GramPrec gp) {
  return (size_t)nblocks * (size_t)gram_tiles(n, gp) * 256;
}

hipError_t launch_gram(const FiberIn &in, const FiberW &w, int rows, double *partials,
                       int nblocks, GramPrec gp, bool e64, hipStream_t s, double *G) {
  if (in.F <= 0) return hipSuccess;
  const int g = (int)gp;
  if (rows > 0 && (e64 ? w.w64 == nullptr : w.w == nullptr)) return hipErrorInvalidValue;
  if (gram_uses_pairs(in.n, gp)) {
    // E of two row chunks at a time in FP64; G is written directly
    if (G == nullptr) return hipErrorInvalidValue;
    if (in.x64) return launch_gram_pairs_typed<double>(in, w, rows, partials, nblocks, e64, G, s);
    return launch_gram_pairs_typed<float>(in, w, rows, partials, nblocks, e64, G, s);
  }
  if (gram_lds(in.n, g) > 160 * 1024) return hipErrorInvalidValue;  // E tile must fit in LDS
  hipError_t e = in.x64 ? launch_gram_typed<double>(in, w, rows, partials, nblocks, g, e64, s)
                        : launch_gram_typed<float>(in, w, rows, partials, nblocks, g, e64, s);
  if (e == hipSuccess && G != nullptr) e = launch_gram_reduce(partials, nblocks, in.n, G, s);
  return e;
}

hipError_t launch_gram_reduce(const double *partials, int nblocks, int64_t n, double *G,
                              hipStream_t s) {
  const int64_t jt = (n + 15) / 16;
  const int ntiles = (int)(jt * (jt + 1) / 2);
  const int64_t total = (int64_t)ntiles * 256;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 15) / 16)), dim3(256), 0, s,
                     partials, nblocks, ntiles, n, G);
  return hipGetLastError();
}

hipError_t launch_reduce_pairs(const double *partials, int count, double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(1024), 0, s, partials, count, out);
  return hipGetLastError();
}

}  // namespace st
