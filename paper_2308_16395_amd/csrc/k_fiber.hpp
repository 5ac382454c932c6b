// Fibre contractions on MFMA for gfx950 (device templates shared by the
// instantiation units k_fiber_*.hip, k_gram.hip and k_rot.hip).
//
// A mode-k partial core D of shape (r~_1..r~_{k-1}, n_k, ..., n_{d-1}) in
// column-major order is a set of F = a*b fibres of length n = n_k (a = r~_{<k},
// b = n'_{>k}); fibre f = i + a*l starts at (f % a) + a*n*(f / a) with stride a.
// The projection P = D x_k U^T is P[f][m] = sum_j D[f][j] U[j][m]; it is computed
// transposed, P^T = U^T D^T, so that the MFMA accumulator of P^T is directly the
// B operand of the residual product E^T = D^T - U P^T (no data movement).
//
// MFMA 16x16x4 f32 and 16x16x32 bf16: lane L supplies row (L % 16) of A and
// column (L % 16) of B; the accumulator holds D[4*(L/16)+v][L%16], v = 0..3.
// The 16x16x4 f64 form holds D[(L/16)+4*v][L%16] instead.
// The K index is free as long as A and B agree: lane L takes the eight K values
// kb + 8*(L/16) + s, s = 0..7, of every 32-wide K block.
//
// PREC 0: FP32 MFMA; 1: split bf16 (hi*hi + hi*lo + lo*hi) with FP32 accumulation;
// 2: FP64 MFMA (exact products of FP32 or FP64 operands, FP64 sums).
#pragma once

#include <type_traits>

#include "common.hpp"

namespace st {
namespace fk {

constexpr int kThreads = 256;  // 4 waves

__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma_bf(const bf16x8 &a, const bf16x8 &b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int PREC>
using AccT = typename std::conditional<PREC == 2, f64x4, f32x4>::type;
template <int PREC>
using OpT = typename std::conditional<PREC == 2, double, float>::type;

template <int PREC>
__device__ constexpr int acc_row(int grp, int v) {
  return PREC == 2 ? grp + 4 * v : 4 * grp + v;
}

// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even).
__device__ inline void split8(const float (&x)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    __bf16 h = (__bf16)x[s];
    hi[s] = h;
    lo[s] = (__bf16)(x[s] - (float)h);
  }
}

template <class T>
__device__ inline const T *cptr(const void *p) {
  return reinterpret_cast<const T *>(p);
}

// Base offset of fibre f (or -1 for an absent / padded fibre).
__device__ inline int64_t fiber_base(const FiberIn &in, int64_t f) {
  if (f >= in.F) return -1;
  if (in.mapped) return map_new_to_old(in.map, f);
  return (f % in.a) + in.a * in.n * (f / in.a);
}

// Eight consecutive K values k0 .. k0 + 7 of one fibre, as operand type OT.
template <bool CONTIG, class TIN, class OT>
__device__ inline void load_x8(const FiberIn &in, int64_t base, int64_t k0, OT (&x)[8]) {
  const TIN *xp = cptr<TIN>(in.x);
  if constexpr (CONTIG && std::is_same<TIN, float>::value) {
    if (base >= 0 && k0 + 8 <= in.n) {
      const f32x4 *p = reinterpret_cast<const f32x4 *>(xp + base + k0);
      const f32x4 u = p[0], v = p[1];
      x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
      x[4] = v[0]; x[5] = v[1]; x[6] = v[2]; x[7] = v[3];
      return;
    }
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = (base >= 0 && k < in.n) ? (OT)xp[base + in.a * k] : (OT)0;
  }
}

// Eight consecutive K values of row m of the row-major FP32 W.
__device__ inline void load_w8(const FiberW &w, int64_t m, int64_t mend, int64_t K, int64_t k0,
                               float (&x)[8]) {
  if (m < mend && k0 + 8 <= K && (w.ldw & 3) == 0) {
    const f32x4 *p = reinterpret_cast<const f32x4 *>(w.w + m * w.ldw + k0);
    const f32x4 u = p[0], v = p[1];
    x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
    x[4] = v[0]; x[5] = v[1]; x[6] = v[2]; x[7] = v[3];
    return;
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = (m < mend && k < K) ? w.w[m * w.ldw + k] : 0.0f;
  }
}

__device__ inline void load_w8_f64(const double *w, int64_t ldw, int64_t m, int64_t mend,
                                   int64_t K, int64_t k0, double (&x)[8]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = (m < mend && k < K) ? w[m * ldw + k] : 0.0;
  }
}

__device__ inline void load_wbf8(const __bf16 *wb, int64_t ld, int64_t m, int64_t mend, int64_t K,
                                 int64_t k0, bf16x8 &x) {
  if (m < mend && k0 + 8 <= K && (ld & 7) == 0) {
    x = *reinterpret_cast<const bf16x8 *>(wb + m * ld + k0);
    return;
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = (m < mend && k < K) ? wb[m * ld + k] : (__bf16)0.0f;
  }
}

// acc[mt][nt] = sum over K of W[m0+16mt.., k] X[fibres of nt, k]. Also sums the
// squares of every X element this wave loads (each element is loaded once).
template <int MT, int NT, bool CONTIG, int PREC, bool NORMX, class TIN>
__device__ inline void project_wave(const FiberIn &in, const FiberW &w, int64_t m0, int64_t mend,
                                    const int64_t (&base)[NT], AccT<PREC> (&acc)[MT][NT],
                                    double &x2) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t K = in.n;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = AccT<PREC>{0, 0, 0, 0};

  for (int64_t kb = 0; kb < K; kb += 32) {
    const int64_t k0 = kb + 8 * grp;
    OpT<PREC> xv[NT][8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      load_x8<CONTIG, TIN>(in, base[nt], k0, xv[nt]);
      if (NORMX) {
#pragma unroll
        for (int s = 0; s < 8; ++s) x2 += (double)xv[nt][s] * (double)xv[nt][s];
      }
    }
    if constexpr (PREC == 0) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float wv[8];
        load_w8(w, m0 + 16 * mt + col, mend, K, k0, wv);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma4(wv[s], xv[nt][s], acc[mt][nt]);
      }
    } else if constexpr (PREC == 2) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        double wv[8];
        load_w8_f64(w.w64, w.ldw, m0 + 16 * mt + col, mend, K, k0, wv);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_f64(wv[s], xv[nt][s], acc[mt][nt]);
      }
    } else {
      bf16x8 xh[NT], xl[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) split8(xv[nt], xh[nt], xl[nt]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf16x8 wh, wl;
        const int64_t m = m0 + 16 * mt + col;
        load_wbf8(w.w_hi, w.ldw_bf, m, mend, K, k0, wh);
        load_wbf8(w.w_lo, w.ldw_bf, m, mend, K, k0, wl);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          acc[mt][nt] = mfma_bf(wh, xh[nt], acc[mt][nt]);
          acc[mt][nt] = mfma_bf(wh, xl[nt], acc[mt][nt]);
          acc[mt][nt] = mfma_bf(wl, xh[nt], acc[mt][nt]);
        }
      }
    }
  }
}

// Rows j = 16*jt + acc_row(grp, v) of (U P^T) for the NT fibre tiles, with
// U[j][m] = W[m][j] and P^T in the accumulators (MT tiles over m).
template <int MT, int NT, int PREC>
__device__ inline void recon_tile(const FiberW &w, int64_t rows, int64_t n, int jt,
                                  const AccT<PREC> (&acc)[MT][NT], AccT<PREC> (&racc)[NT]) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t j = 16 * jt + col;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) racc[nt] = AccT<PREC>{0, 0, 0, 0};
  if constexpr (PREC == 2) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = 16 * mt + grp + 4 * v;
        const double a = (m < rows && j < n) ? w.w64[m * w.ldw + j] : 0.0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) racc[nt] = mfma_f64(a, acc[mt][nt][v], racc[nt]);
      }
  } else if constexpr (PREC == 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = 16 * mt + 4 * grp + v;
        const float a = (m < rows && j < n) ? w.w[m * w.ldw + j] : 0.0f;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) racc[nt] = mfma4(a, acc[mt][nt][v], racc[nt]);
      }
  } else {
    // K slots s = 0..7 <-> (tile mt = 2q + s/4, v = s%4)
#pragma unroll
    for (int q = 0; q < (MT + 1) / 2; ++q) {
      bf16x8 ah, al;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int mt = 2 * q + s / 4;
        const int64_t m = 16 * mt + 4 * grp + (s & 3);
        const bool ok = mt < MT && m < rows && j < n;
        ah[s] = ok ? w.w_hi[m * w.ldw_bf + j] : (__bf16)0.0f;
        al[s] = ok ? w.w_lo[m * w.ldw_bf + j] : (__bf16)0.0f;
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        float pv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int mt = 2 * q + s / 4;
          pv[s] = (mt < MT) ? acc[mt < MT ? mt : 0][nt][s & 3] : 0.0f;
        }
        bf16x8 ph, pl;
        split8(pv, ph, pl);
        racc[nt] = mfma_bf(ah, ph, racc[nt]);
        racc[nt] = mfma_bf(ah, pl, racc[nt]);
        racc[nt] = mfma_bf(al, ph, racc[nt]);
      }
    }
  }
}

// Projection P = X x W^T (and, with RESID, the residual and norm partials).
// With `stage` (output stride ao == 1, i.e. the outputs of one fibre are
// contiguous and consecutive fibres adjacent), each wave writes its tile
// through LDS so that the stores are contiguous instead of one cache line per
// lane.
template <int MT, int NT, bool CONTIG, bool RESID, int PREC, class TIN, class TOUT>
__global__ __launch_bounds__(kThreads) void fiber_kernel(FiberIn in, FiberW w, int m0, int mcount,
                                                         FiberOut out, double *partials,
                                                         int stage) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t mbeg = (int64_t)m0 + (int64_t)blockIdx.y * (16 * MT);
  const int64_t mend = (int64_t)m0 + mcount;
  const int64_t fwave = ((int64_t)blockIdx.x * 4 + wid) * (16 * NT);
  const TIN *xp = cptr<TIN>(in.x);
  TOUT *op = reinterpret_cast<TOUT *>(out.p);

  int64_t fib[NT], base[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    fib[nt] = fwave + 16 * nt + col;
    base[nt] = fiber_base(in, fib[nt]);
  }
  AccT<PREC> acc[MT][NT];
  double x2 = 0.0, e2 = 0.0;
  project_wave<MT, NT, CONTIG, PREC, RESID, TIN>(in, w, mbeg, mend, base, acc, x2);

  if (stage) {
    extern __shared__ double stage_raw[];
    constexpr int TW = 16 * MT;  // outputs per fibre in this block
    constexpr int TWP = TW + 1;  // padded LDS row (odd: spreads the banks)
    TOUT *tile = reinterpret_cast<TOUT *>(stage_raw) + (size_t)wid * (16 * NT) * TWP;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          tile[(16 * nt + col) * TWP + 16 * mt + acc_row<PREC>(grp, v)] = (TOUT)acc[mt][nt][v];
    __syncthreads();
    const int64_t mlen = (mend - mbeg) < TW ? (mend - mbeg) : TW;
    const int64_t total = (int64_t)(16 * NT) * mlen;
    for (int64_t idx = lane; idx < total; idx += 64) {
      const int64_t fl = idx / mlen, ml = idx - fl * mlen;
      const int64_t f = fwave + fl;
      if (f < in.F) op[mbeg + ml + out.mo * f] = tile[fl * TWP + ml];
    }
  } else {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t f = fib[nt];
      if (f >= in.F) continue;
      const int64_t fq = f / out.ao, fr = f - fq * out.ao;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = mbeg + 16 * mt + acc_row<PREC>(grp, v);
          if (m < mend) op[fr + out.ao * (m + out.mo * fq)] = (TOUT)acc[mt][nt][v];
        }
    }
  }

  if constexpr (RESID) {
    const int jtiles = (int)((in.n + 15) / 16);
    for (int jt = 0; jt < jtiles; ++jt) {
      AccT<PREC> racc[NT];
      recon_tile<MT, NT, PREC>(w, mcount, in.n, jt, acc, racc);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (fib[nt] >= in.F) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = 16 * jt + acc_row<PREC>(grp, v);
          if (j < in.n) {
            const double e = (double)xp[base[nt] + in.a * j] - (double)racc[nt][v];
            e2 += e * e;
          }
        }
      }
    }
    __shared__ double red[2][4];
    e2 = wave_sum(e2);
    x2 = wave_sum(x2);
    if (lane == 0) {
      red[0][wid] = e2;
      red[1][wid] = x2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      partials[2 * blockIdx.x + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      partials[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

template <int MT, int NT, bool CONTIG, bool RESID, int PREC, class TIN, class TOUT>
hipError_t launch_fiber_t(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, hipStream_t s) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            RESID ? 1u : (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  // stage the output tile through LDS when the output stride is 1 and the
  // tile fits (4 waves x 16 NT fibres x 16 MT outputs)
  const size_t lds = (size_t)4 * 16 * NT * (16 * MT + 1) * sizeof(TOUT);
  const int stage = (out.ao == 1 && lds <= 64 * 1024) ? 1 : 0;
  hipLaunchKernelGGL((fiber_kernel<MT, NT, CONTIG, RESID, PREC, TIN, TOUT>), grid,
                     dim3(kThreads), stage ? lds : 0, s, in, w, m0, mcount, out, partials, stage);
  return hipGetLastError();
}

template <int MT, int NT, bool CONTIG, bool RESID, class TIN, class TOUT>
hipError_t launch_fiber_p(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, Prec prec, hipStream_t s) {
  if (prec == Prec::BF16X3)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 1, TIN, TOUT>(in, w, m0, mcount, out, partials, s);
  if (prec == Prec::FP64)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 2, TIN, TOUT>(in, w, m0, mcount, out, partials, s);
  return launch_fiber_t<MT, NT, CONTIG, RESID, 0, TIN, TOUT>(in, w, m0, mcount, out, partials, s);
}

template <int MT, int NT, class TIN, class TOUT>
hipError_t launch_fiber_c(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s) {
  const bool resid = partials != nullptr;
  if constexpr (std::is_same<TIN, float>::value) {
    if (contig) {
      if (resid)
        return launch_fiber_p<MT, NT, true, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s);
      return launch_fiber_p<MT, NT, true, false, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s);
    }
  }
  if (resid)
    return launch_fiber_p<MT, NT, false, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s);
  return launch_fiber_p<MT, NT, false, false, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s);
}

template <int NT, class TIN, class TOUT>
hipError_t launch_fiber_n(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s) {
  // smallest instantiated tile count >= the rows needed (padding wastes MFMA work)
  const int tiles = (mcount + 15) / 16;
#define ST_FIBER_CASE(T)                                                                        \
  if (tiles <= T)                                                                               \
    return launch_fiber_c<T, NT, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s);
  ST_FIBER_CASE(1)
  ST_FIBER_CASE(2)
  ST_FIBER_CASE(3)
  ST_FIBER_CASE(4)
  ST_FIBER_CASE(6)
  ST_FIBER_CASE(8)
  ST_FIBER_CASE(12)
#undef ST_FIBER_CASE
  if (tiles <= 16 || partials == nullptr)
    return launch_fiber_c<16, NT, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s);
  return hipErrorInvalidValue;  // fused residual needs all rows in one block
}

inline bool contiguous(const FiberIn &in) {
  return !in.mapped && !in.x64 && in.a == 1 && (in.n & 3) == 0 &&
         (reinterpret_cast<uintptr_t>(in.x) & 15) == 0;
}

template <class TIN, class TOUT>
hipError_t launch_fiber_typed(const FiberIn &in, const FiberW &w, int m0, int mcount,
                              const FiberOut &out, double *partials, Prec prec, hipStream_t s) {
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  const bool contig = contiguous(in);
  // two fibre tiles per wave when there are enough fibres to fill the chip
  if (in.F >= 256 * 128)
    return launch_fiber_n<2, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s);
  return launch_fiber_n<1, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s);
}

}  // namespace fk
}  // namespace st
