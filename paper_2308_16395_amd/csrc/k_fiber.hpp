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

// p[idx] when ok, else 0, without a branch: the load itself is unconditional
// (it reads p[0] when !ok), so a run of such loads issues back to back instead
// of each waiting behind its own branch.
template <class T>
__device__ inline T load_or0(const T *p, int64_t idx, bool ok) {
  const T v = p[ok ? idx : 0];
  return ok ? v : (T)0;
}

// Row and column of flat index idx in a tile of rows of length len (idx < 2^24,
// len >= 1): a float reciprocal and one correction instead of an integer
// division (idx / len is exact to within one after the float product).
__device__ inline void tile_rc(int idx, int len, float inv_len, int &row, int &colm) {
  int q = (int)((float)idx * inv_len);
  int r = idx - q * len;
  if (r < 0) {
    --q;
    r += len;
  } else if (r >= len) {
    ++q;
    r -= len;
  }
  row = q;
  colm = r;
}

// Base offset of fibre f (or -1 for an absent / padded fibre).
__device__ inline int64_t fiber_base(const FiberIn &in, int64_t f) {
  if (f >= in.F) return -1;
  if (in.mapped) return map_new_to_old(in.map, f);
  int64_t q, r;
  divmod_index(f, in.a, q, r);
  return r + in.a * in.n * q;
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
    x[s] = (OT)load_or0(xp, base + in.a * k, base >= 0 && k < in.n);
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
    x[s] = load_or0(w.w, m * w.ldw + k, m < mend && k < K);
  }
}

__device__ inline void load_w8_f64(const double *w, int64_t ldw, int64_t m, int64_t mend,
                                   int64_t K, int64_t k0, double (&x)[8]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = load_or0(w, m * ldw + k, m < mend && k < K);
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
    x[s] = load_or0(wb, m * ld + k, m < mend && k < K);
  }
}

// Chunked W in LDS: rows [m0, m0 + 16 MT) x columns [c0, c0 + NC) of W, in the
// form the product precision reads, copied into lds as [16 MT][LD] with rows
// past mend and columns past K zero-filled (so readers need no bounds tests),
// and a FiberW view of that chunk (rows and columns counted from its corner).
template <int MT, int PREC, int NC, int LD>
__device__ inline void wchunk_copy(const FiberW &w, int64_t m0, int64_t mend, int64_t K,
                                   int64_t c0, double *lds, FiberW &view) {
  constexpr int total = 16 * MT * NC;
  for (int idx = threadIdx.x; idx < total; idx += kThreads) {
    const int r = idx / NC, c = idx % NC;  // NC is a power of two
    const int64_t m = m0 + r, k = c0 + c;
    const bool ok = m < mend && k < K;
    if constexpr (PREC == 0) {
      reinterpret_cast<float *>(lds)[r * LD + c] = load_or0(w.w, m * w.ldw + k, ok);
    } else if constexpr (PREC == 2) {
      lds[r * LD + c] = load_or0(w.w64, m * w.ldw + k, ok);
    } else {
      __bf16 *h = reinterpret_cast<__bf16 *>(lds);
      h[r * LD + c] = load_or0(w.w_hi, m * w.ldw_bf + k, ok);
      h[16 * MT * LD + r * LD + c] = load_or0(w.w_lo, m * w.ldw_bf + k, ok);
    }
  }
  view = w;
  if constexpr (PREC == 0) {
    view.w = reinterpret_cast<float *>(lds);
    view.ldw = LD;
  } else if constexpr (PREC == 2) {
    view.w64 = lds;
    view.ldw = LD;
  } else {
    view.w_hi = reinterpret_cast<__bf16 *>(lds);
    view.w_lo = view.w_hi + 16 * MT * LD;
    view.ldw_bf = LD;
  }
}
// row strides of the projection (32 columns) and reconstruction (16) chunks:
// multiples of 4 floats / 8 bf16 for the vector reads, padded off the banks
template <int PREC>
constexpr int kChunkLdP = PREC == 0 ? 36 : (PREC == 2 ? 34 : 40);
template <int PREC>
constexpr int kChunkLdR = PREC == 0 ? 20 : (PREC == 2 ? 18 : 24);
template <int MT, int PREC>
constexpr size_t chunk_lds_bytes() {
  constexpr size_t es = PREC == 2 ? 8 : 4;  // bf16: hi and lo
  constexpr size_t p = (size_t)16 * MT * kChunkLdP<PREC> * es;
  constexpr size_t r = (size_t)16 * MT * kChunkLdR<PREC> * es;
  return p > r ? p : r;
}

// acc[mt][nt] = sum over K of W[m0+16mt.., k] X[fibres of nt, k]. Also sums the
// squares of every X element this wave loads (each element is loaded once).
// WC: W is read from an LDS chunk of 32 columns staged per K block by the
// whole block (`lds`); every wave of the block must call this together.
template <int MT, int NT, bool CONTIG, int PREC, bool NORMX, class TIN, bool WC = false>
__device__ inline void project_wave(const FiberIn &in, const FiberW &w, int64_t m0, int64_t mend,
                                    const int64_t (&base)[NT], AccT<PREC> (&acc)[MT][NT],
                                    double &x2, double *lds = nullptr) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t K = in.n;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = AccT<PREC>{0, 0, 0, 0};

  // The X values of K block kb + 32 are loaded while the MFMAs of block kb run.
  // Loads are unconditional; xm (bit 8 nt + s: element in range) zeroes the
  // out-of-range ones when the block is consumed, so the loads stay in flight.
  const TIN *xp = cptr<TIN>(in.x);
  TIN xr[NT][8];
  uint32_t xm = 0;
  auto fetch = [&](int64_t kb) {
    const int64_t k0 = kb + 8 * grp;
    xm = 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      if constexpr (CONTIG && std::is_same<TIN, float>::value) {
        if (base[nt] >= 0 && k0 + 8 <= in.n) {
          const f32x4 *p = reinterpret_cast<const f32x4 *>(xp + base[nt] + k0);
          const f32x4 u = p[0], v = p[1];
          xr[nt][0] = u[0]; xr[nt][1] = u[1]; xr[nt][2] = u[2]; xr[nt][3] = u[3];
          xr[nt][4] = v[0]; xr[nt][5] = v[1]; xr[nt][6] = v[2]; xr[nt][7] = v[3];
          xm |= 0xffu << (8 * nt);
          continue;
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t k = k0 + s;
        const bool ok = base[nt] >= 0 && k < in.n;
        xr[nt][s] = xp[ok ? base[nt] + in.a * k : 0];
        xm |= (ok ? 1u : 0u) << (8 * nt + s);
      }
    }
  };
  // wide tiles (MT NT > 8) load in the iteration instead: the prefetch
  // registers would cost them their second wave per SIMD
  constexpr bool PF = MT * NT <= 8;
  if (PF) fetch(0);
  for (int64_t kb = 0; kb < K; kb += 32) {
    const int64_t k0 = kb + 8 * grp;
    if (!PF) fetch(kb);
    OpT<PREC> xv[NT][8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int s = 0; s < 8; ++s)
        xv[nt][s] = ((xm >> (8 * nt + s)) & 1u) ? (OpT<PREC>)xr[nt][s] : (OpT<PREC>)0;
    if (PF && kb + 32 < K) fetch(kb + 32);
    // the W source of this block: W itself, or its LDS chunk (corner at row m0,
    // column kb; out-of-range entries zero)
    FiberW wsrc = w;
    int64_t wm0 = m0, wmend = mend, wk0 = k0, wK = K;
    if constexpr (WC) {
      __syncthreads();  // every wave is done with the previous chunk
      wchunk_copy<MT, PREC, 32, kChunkLdP<PREC>>(w, m0, mend, K, kb, lds, wsrc);
      __syncthreads();
      wm0 = 0;
      wmend = 16 * MT;
      wk0 = 8 * grp;
      wK = 32;
    }
    if (NORMX) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int s = 0; s < 8; ++s) x2 += (double)xv[nt][s] * (double)xv[nt][s];
    }
    if constexpr (PREC == 0) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float wv[8];
        load_w8(wsrc, wm0 + 16 * mt + col, wmend, wK, wk0, wv);
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma4(wv[s], xv[nt][s], acc[mt][nt]);
      }
    } else if constexpr (PREC == 2) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        double wv[8];
        load_w8_f64(wsrc.w64, wsrc.ldw, wm0 + 16 * mt + col, wmend, wK, wk0, wv);
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
        const int64_t m = wm0 + 16 * mt + col;
        load_wbf8(wsrc.w_hi, wsrc.ldw_bf, m, wmend, wK, wk0, wh);
        load_wbf8(wsrc.w_lo, wsrc.ldw_bf, m, wmend, wK, wk0, wl);
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
        const double a = load_or0(w.w64, m * w.ldw + j, m < rows && j < n);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) racc[nt] = mfma_f64(a, acc[mt][nt][v], racc[nt]);
      }
  } else if constexpr (PREC == 0) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = 16 * mt + 4 * grp + v;
        const float a = load_or0(w.w, m * w.ldw + j, m < rows && j < n);
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
        ah[s] = load_or0(w.w_hi, m * w.ldw_bf + j, ok);
        al[s] = load_or0(w.w_lo, m * w.ldw_bf + j, ok);
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

// Copy rows [mbeg, min(mend, mbeg + 16 MT)) of W (all n columns, in the form
// the product precision reads) into LDS with row stride wld, zero the rows up
// to 16 MT (so every lane can take the vector reads), and point wv at the copy
// (rows then count from mbeg). Thread t copies row t / 32 (+ 8 i), columns
// 4 (t % 32) + 128 j as 16-byte vectors when the strides allow, else single
// elements; no index division. Ends with a block barrier.
template <int MT, int PREC>
__device__ inline void stage_w(const FiberW &w, int64_t mbeg, int64_t mend, int64_t n, int wld,
                               double *lds, FiberW &wv) {
  const int rows = (int)((mend - mbeg) < 16 * MT ? (mend - mbeg) : 16 * MT);
  const int nn = (int)n, r0 = threadIdx.x >> 5, c0 = threadIdx.x & 31;
  if constexpr (PREC == 0) {
    float *d = reinterpret_cast<float *>(lds);
    const bool v4 = (nn & 3) == 0 && (w.ldw & 3) == 0 && (wld & 3) == 0 &&
                    ((uintptr_t)w.w & 15) == 0 && ((mbeg * w.ldw) & 3) == 0;
    for (int r = r0; r < 16 * MT; r += 8) {
      float *dr = d + r * wld;
      if (r < rows) {
        const float *src = w.w + (mbeg + r) * w.ldw;
        if (v4) {
          for (int k = 4 * c0; k < nn; k += 128)
            *reinterpret_cast<f32x4 *>(dr + k) = *reinterpret_cast<const f32x4 *>(src + k);
        } else {
          for (int k = c0; k < nn; k += 32) dr[k] = src[k];
        }
      } else {
        for (int k = c0; k < nn; k += 32) dr[k] = 0.0f;
      }
    }
    wv.w = d;
    wv.ldw = wld;
  } else if constexpr (PREC == 2) {
    for (int r = r0; r < 16 * MT; r += 8) {
      double *dr = lds + r * wld;
      if (r < rows) {
        const double *src = w.w64 + (mbeg + r) * w.ldw;
        for (int k = c0; k < nn; k += 32) dr[k] = src[k];
      } else {
        for (int k = c0; k < nn; k += 32) dr[k] = 0.0;
      }
    }
    wv.w64 = lds;
    wv.ldw = wld;
  } else {
    __bf16 *h = reinterpret_cast<__bf16 *>(lds), *l = h + 16 * MT * wld;
    for (int r = r0; r < 16 * MT; r += 8) {
      __bf16 *hr = h + r * wld, *lr = l + r * wld;
      if (r < rows) {
        const __bf16 *sh = w.w_hi + (mbeg + r) * w.ldw_bf, *sl = w.w_lo + (mbeg + r) * w.ldw_bf;
        for (int k = c0; k < nn; k += 32) {
          hr[k] = sh[k];
          lr[k] = sl[k];
        }
      } else {
        for (int k = c0; k < nn; k += 32) {
          hr[k] = (__bf16)0.0f;
          lr[k] = (__bf16)0.0f;
        }
      }
    }
    wv.w_hi = h;
    wv.w_lo = l;
    wv.ldw_bf = wld;
  }
  __syncthreads();
}

// LDS row stride of the W copy: a multiple of 4 (FP32 / FP64: 16-byte vector
// reads of FP32 rows) or 8 (bf16x8 reads), padded so that consecutive rows
// start in different banks.
template <int PREC>
__host__ __device__ inline int w_lds_stride(int64_t n) {
  return PREC == 1 ? (int)(((n + 7) / 8) * 8 + 8) : (int)(((n + 7) / 8) * 8 + 4);
}
template <int MT, int PREC>
__host__ __device__ inline size_t w_lds_bytes(int wld) {
  // bf16x3 keeps the hi and lo halves (2 x 2 bytes per element)
  return (size_t)16 * MT * wld * (PREC == 2 ? 8 : 4);
}

// Projection P = X x W^T (and, with RESID, the residual and norm partials).
// With `stage` (output stride ao == 1, i.e. the outputs of one fibre are
// contiguous and consecutive fibres adjacent), each wave writes its tile
// through LDS so that the stores are contiguous instead of one cache line per
// lane. With WL the block's rows of W are first copied into LDS (row stride
// wld) and both products read them from there; the output tile then reuses
// that LDS after the residual.
template <int MT, int NT, bool CONTIG, bool RESID, int PREC, class TIN, class TOUT, bool WL,
          bool WC = false>
__global__ __launch_bounds__(kThreads) void fiber_kernel(FiberIn in, FiberW w, int m0, int mcount,
                                                         FiberOut out, double *partials,
                                                         int stage, int wld) {
  extern __shared__ double lds_raw[];
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
  FiberW wv = w;
  int64_t pm0 = mbeg, pmend = mend;
  if constexpr (WL) {
    // rows past mcount are zero in the copy: all 16 MT rows read as data
    stage_w<MT, PREC>(w, mbeg, mend, in.n, wld, lds_raw, wv);
    pm0 = 0;
    pmend = 16 * MT;
  }
  AccT<PREC> acc[MT][NT];
  double x2 = 0.0, e2 = 0.0;
  project_wave<MT, NT, CONTIG, PREC, RESID, TIN, WC>(in, wv, pm0, pmend, base, acc, x2, lds_raw);
  // WC: the reconstruction reads W[:, 16 jt .. 16 jt + 16) from an LDS chunk
  // staged per tile (zero rows past mcount)
  auto recon = [&](int jt, AccT<PREC> (&racc)[NT]) {
    if constexpr (WC) {
      FiberW wr;
      __syncthreads();  // every wave is done with the previous chunk
      wchunk_copy<MT, PREC, 16, kChunkLdR<PREC>>(w, 0, mcount, in.n, 16 * jt, lds_raw, wr);
      __syncthreads();
      recon_tile<MT, NT, PREC>(wr, 16 * MT, 16, 0, acc, racc);
    } else {
      recon_tile<MT, NT, PREC>(wv, WL ? 16 * MT : mcount, in.n, jt, acc, racc);
    }
  };

  if constexpr (RESID) {
    // (with RESID, m0 == 0 and the block holds all mcount rows of W)
    const int jtiles = (int)((in.n + 15) / 16);
    bool fast = false;
    if constexpr (CONTIG && PREC != 2 && std::is_same<TIN, float>::value && MT * NT <= 8)
      fast = in.n % 16 == 0;
    if (fast) {
      // contiguous FP32 fibres, whole tiles: rows 16 jt + 4 grp .. + 3 of each
      // fibre in one 16-byte load, fetched one tile ahead of the reconstruction
      f32x4 xn[NT];
      auto ldx = [&](int jt) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          xn[nt] = *reinterpret_cast<const f32x4 *>(xp + (base[nt] >= 0 ? base[nt] : 0) +
                                                    16 * jt + 4 * grp);
      };
      ldx(0);
      for (int jt = 0; jt < jtiles; ++jt) {
        f32x4 xc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) xc[nt] = xn[nt];
        if (jt + 1 < jtiles) ldx(jt + 1);
        AccT<PREC> racc[NT];
        recon(jt, racc);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          if (fib[nt] >= in.F) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double e = (double)xc[nt][v] - (double)racc[nt][v];
            e2 += e * e;
          }
        }
      }
    }
    for (int jt = 0; jt < (fast ? 0 : jtiles); ++jt) {
      AccT<PREC> racc[NT];
      recon(jt, racc);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (fib[nt] >= in.F) continue;
        if constexpr (CONTIG && PREC != 2) {
          // contiguous FP32 fibre: rows 16 jt + 4 grp .. + 3 in one 16-byte load
          const int64_t j0 = 16 * jt + 4 * grp;
          if (j0 + 4 <= in.n) {
            const f32x4 xv = *reinterpret_cast<const f32x4 *>(xp + base[nt] + j0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const double e = (double)xv[v] - (double)racc[nt][v];
              e2 += e * e;
            }
            continue;
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = 16 * jt + acc_row<PREC>(grp, v);
          const bool ok = j < in.n;
          const double xj = (double)load_or0(xp, base[nt] + in.a * j, ok);
          const double e = ok ? xj - (double)racc[nt][v] : 0.0;
          e2 += e * e;
        }
      }
    }
  }

  if (stage) {
    if constexpr (WL || WC) __syncthreads();  // every wave is done with the W copy
    constexpr int TW = 16 * MT;  // outputs per fibre in this block
    constexpr int TWP = TW + 1;  // padded LDS row (odd: spreads the banks)
    TOUT *tile = reinterpret_cast<TOUT *>(lds_raw) + (size_t)wid * (16 * NT) * TWP;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          tile[(16 * nt + col) * TWP + 16 * mt + acc_row<PREC>(grp, v)] = (TOUT)acc[mt][nt][v];
    __syncthreads();
    const int mlen = (int)((mend - mbeg) < TW ? (mend - mbeg) : TW);
    const int total = 16 * NT * mlen;
    const float inv = 1.0f / (float)mlen;
    for (int idx = lane; idx < total; idx += 64) {
      int fl, ml;
      tile_rc(idx, mlen, inv, fl, ml);
      const int64_t f = fwave + fl;
      if (f < in.F) op[mbeg + ml + out.mo * f] = tile[fl * TWP + ml];
    }
  } else {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t f = fib[nt];
      if (f >= in.F) continue;
      int64_t fq, fr;
      divmod_index(f, out.ao, fq, fr);
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

// ---------------------------------------------------------------------------
// Fused projection + residual with the fibres held in registers.
//
// Lane (col, grp) keeps, for each of its NT fibres, the elements
// j = kidx(i, grp, v) = 16 i + 4 grp + v (16 i + grp + 4 v for the FP64 MFMA),
// i < JT, v < 4: exactly the rows its residual accumulator holds after the
// reconstruction MFMAs of tile i, and a valid K split for the projection MFMAs
// (the four lane groups of one MFMA step cover four distinct k). Each fibre is
// read from memory once; the projection, the residual and both norms run from
// registers. Used when n <= 16 JT and all rows of W fit one block.
// ---------------------------------------------------------------------------
template <int PREC>
__device__ constexpr int kidx(int i, int grp, int v) {
  return 16 * i + (PREC == 2 ? grp + 4 * v : 4 * grp + v);
}

template <int MT, int NT, int JT, int PREC, class TIN, class TOUT, bool WL>
__global__ __launch_bounds__(kThreads) void resid_kernel(FiberIn in, FiberW w, int mcount,
                                                         FiberOut out, double *partials,
                                                         int stage, int wld) {
  extern __shared__ double stage_raw[];
  // element type kept in registers: the input's, or FP64 for the FP64 MFMA
  using XT = typename std::conditional<PREC == 2 || std::is_same<TIN, double>::value, double,
                                       float>::type;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t n = in.n;
  const int64_t fwave = ((int64_t)blockIdx.x * 4 + wid) * (16 * NT);
  const TIN *xp = cptr<TIN>(in.x);
  TOUT *op = reinterpret_cast<TOUT *>(out.p);

  int64_t fib[NT], base[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    fib[nt] = fwave + 16 * nt + col;
    base[nt] = fiber_base(in, fib[nt]);
  }
  // WL: W (all mcount rows) is read from an LDS copy, with the output tile
  // after it in LDS
  FiberW wv = w;
  size_t tile_off = 0;  // doubles
  if constexpr (WL) {
    stage_w<MT, PREC>(w, 0, mcount, n, wld, stage_raw, wv);
    tile_off = (w_lds_bytes<MT, PREC>(wld) + 15) / 16 * 2;
  }
  XT x[NT][JT][4];
  double x2 = 0.0;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int i = 0; i < JT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t k = kidx<PREC>(i, grp, v);
        const XT val = (XT)load_or0(xp, base[nt] + in.a * k, base[nt] >= 0 && k < n);
        x[nt][i][v] = val;
        x2 += (double)val * (double)val;
      }

  AccT<PREC> acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = AccT<PREC>{0, 0, 0, 0};
  if constexpr (PREC == 1) {
    // 16x16x32 bf16 steps over tile pairs (i0, i0 + 1): 8 K values per lane
#pragma unroll
    for (int i0 = 0; i0 < JT; i0 += 2) {
      bf16x8 xh[NT], xl[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        float t[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t[v] = (float)x[nt][i0][v];
          t[4 + v] = (i0 + 1 < JT) ? (float)x[nt][i0 + 1 < JT ? i0 + 1 : i0][v] : 0.0f;
        }
        split8(t, xh[nt], xl[nt]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int m = 16 * mt + col;
        float t[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t k0 = kidx<PREC>(i0, grp, v), k1 = kidx<PREC>(i0 + 1, grp, v);
          t[v] = load_or0(wv.w, m * wv.ldw + k0, m < mcount && k0 < n);
          t[4 + v] = load_or0(wv.w, m * wv.ldw + k1, i0 + 1 < JT && m < mcount && k1 < n);
        }
        bf16x8 wh, wl;
        split8(t, wh, wl);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          acc[mt][nt] = mfma_bf(wh, xh[nt], acc[mt][nt]);
          acc[mt][nt] = mfma_bf(wh, xl[nt], acc[mt][nt]);
          acc[mt][nt] = mfma_bf(wl, xh[nt], acc[mt][nt]);
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < JT; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t k = kidx<PREC>(i, grp, v);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int m = 16 * mt + col;
          const bool ok = m < mcount && k < n;
          if constexpr (PREC == 2) {
            const double a = load_or0(wv.w64, m * wv.ldw + k, ok);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[mt][nt] = mfma_f64(a, (double)x[nt][i][v], acc[mt][nt]);
          } else {
            const float a = load_or0(wv.w, m * wv.ldw + k, ok);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[mt][nt] = mfma4(a, (float)x[nt][i][v], acc[mt][nt]);
          }
        }
      }
  }

  // P = D x_k W^T (this block holds all rows of W)
  const int64_t mend = mcount;
  if (stage) {
    constexpr int TW = 16 * MT;
    constexpr int TWP = TW + 1;
    TOUT *tile = reinterpret_cast<TOUT *>(stage_raw + tile_off) + (size_t)wid * (16 * NT) * TWP;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          tile[(16 * nt + col) * TWP + 16 * mt + acc_row<PREC>(grp, v)] = (TOUT)acc[mt][nt][v];
    __syncthreads();
    const int mlen = (int)mend;
    const int total = 16 * NT * mlen;
    const float inv = 1.0f / (float)mlen;
    for (int idx = lane; idx < total; idx += 64) {
      int fl, ml;
      tile_rc(idx, mlen, inv, fl, ml);
      const int64_t f = fwave + fl;
      if (f < in.F) op[ml + out.mo * f] = tile[fl * TWP + ml];
    }
  } else {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t f = fib[nt];
      if (f >= in.F) continue;
      int64_t fq, fr;
    divmod_index(f, out.ao, fq, fr);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = 16 * mt + acc_row<PREC>(grp, v);
          if (m < mend) op[fr + out.ao * (m + out.mo * fq)] = (TOUT)acc[mt][nt][v];
        }
    }
  }

  // E = D - P x_k W: reconstruction tile i holds rows kidx(i, grp, v) per lane
  double e2 = 0.0;
#pragma unroll
  for (int i = 0; i < JT; ++i) {
    AccT<PREC> racc[NT];
    recon_tile<MT, NT, PREC>(wv, mcount, n, i, acc, racc);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      if (fib[nt] >= in.F) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (kidx<PREC>(i, grp, v) < n) {
          const double e = (double)x[nt][i][v] - (double)racc[nt][v];
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

template <int MT, int NT, int JT, int PREC, class TIN, class TOUT>
hipError_t launch_resid_w(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                          double *partials, hipStream_t s, int *np) {
  const size_t lds = (size_t)4 * 16 * NT * (16 * MT + 1) * sizeof(TOUT);
  const int stage = (out.ao == 1 && lds <= 64 * 1024) ? 1 : 0;
  const size_t slds = stage ? lds : 0;
  dim3 grid((unsigned)((in.F + 64 * NT - 1) / (64 * NT)));
  // W read from an LDS copy when it fits beside the output tile
  const int wld = w_lds_stride<PREC>(in.n);
  const size_t wb = (w_lds_bytes<MT, PREC>(wld) + 15) / 16 * 16;
  if (wb + slds <= 96 * 1024) {
    if (wb + slds > 64 * 1024) {
      const void *fn = (const void *)resid_kernel<MT, NT, JT, PREC, TIN, TOUT, true>;
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(wb + slds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((resid_kernel<MT, NT, JT, PREC, TIN, TOUT, true>), grid, dim3(kThreads),
                       wb + slds, s, in, w, mcount, out, partials, stage, wld);
  } else {
    hipLaunchKernelGGL((resid_kernel<MT, NT, JT, PREC, TIN, TOUT, false>), grid, dim3(kThreads),
                       slds, s, in, w, mcount, out, partials, stage, 0);
  }
  if (np) *np = (int)grid.x;
  return hipGetLastError();
}

template <int MT, int JT, int PREC, class TIN, class TOUT>
hipError_t launch_resid_t(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                          double *partials, hipStream_t s, int *np) {
  // two fibre tiles per wave when the registers allow it and there are enough
  // fibres to fill the chip
  constexpr bool wide = !(PREC == 2 || std::is_same<TIN, double>::value) && JT * MT <= 24;
  if (wide && in.F >= 256 * 128)
    return launch_resid_w<MT, wide ? 2 : 1, JT, PREC, TIN, TOUT>(in, w, mcount, out, partials, s,
                                                                 np);
  return launch_resid_w<MT, 1, JT, PREC, TIN, TOUT>(in, w, mcount, out, partials, s, np);
}

template <int MT, int JT, class TIN, class TOUT>
hipError_t launch_resid_p(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                          double *partials, Prec prec, hipStream_t s, int *np) {
  if (prec == Prec::BF16X3)
    return launch_resid_t<MT, JT, 1, TIN, TOUT>(in, w, mcount, out, partials, s, np);
  if (prec == Prec::FP64)
    return launch_resid_t<MT, JT, 2, TIN, TOUT>(in, w, mcount, out, partials, s, np);
  return launch_resid_t<MT, JT, 0, TIN, TOUT>(in, w, mcount, out, partials, s, np);
}

template <int MT, class TIN, class TOUT>
hipError_t launch_resid_j(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                          double *partials, Prec prec, hipStream_t s, int *np) {
  const int64_t jt = (in.n + 15) / 16;
  if (jt <= 1) return launch_resid_p<MT, 1, TIN, TOUT>(in, w, mcount, out, partials, prec, s, np);
  if (jt <= 2) return launch_resid_p<MT, 2, TIN, TOUT>(in, w, mcount, out, partials, prec, s, np);
  if (jt <= 4) return launch_resid_p<MT, 4, TIN, TOUT>(in, w, mcount, out, partials, prec, s, np);
  return launch_resid_p<MT, 8, TIN, TOUT>(in, w, mcount, out, partials, prec, s, np);
}

// The register-resident residual kernel, when it applies (returns false if not).
template <class TIN, class TOUT>
bool try_launch_resid(const FiberIn &in, const FiberW &w, int m0, int mcount, const FiberOut &out,
                      double *partials, Prec prec, hipStream_t s, hipError_t &err, int *np) {
  // used for the FP64 partial cores (modes 2..d-1); for FP32 input the
  // streaming kernel with vector loads runs at higher occupancy
  if constexpr (!std::is_same<TIN, double>::value) {
    return false;
  } else {
    if (partials == nullptr || in.mapped || m0 != 0 || in.n > 128 || mcount > 128) return false;
    const int tiles = (mcount + 15) / 16;
#define ST_RESID_CASE(T_)                                                                \
    if (tiles <= T_) {                                                                   \
      err = launch_resid_j<T_, TIN, TOUT>(in, w, mcount, out, partials, prec, s, np);    \
      return true;                                                                       \
    }
    ST_RESID_CASE(1)
    ST_RESID_CASE(2)
    ST_RESID_CASE(3)
    ST_RESID_CASE(4)
    ST_RESID_CASE(6)
    ST_RESID_CASE(8)
#undef ST_RESID_CASE
    return false;
  }
}

template <int MT, int NT, bool CONTIG, bool RESID, int PREC, class TIN, class TOUT>
hipError_t launch_fiber_t(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, hipStream_t s, int *nparts) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            RESID ? 1u : (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  // stage the output tile through LDS when the output stride is 1 and the
  // tile fits (4 waves x 16 NT fibres x 16 MT outputs)
  const size_t lds = (size_t)4 * 16 * NT * (16 * MT + 1) * sizeof(TOUT);
  const int stage = (out.ao == 1 && lds <= 64 * 1024) ? 1 : 0;
  const size_t slds = stage ? lds : 0;
  if constexpr (RESID) {
    // the fused residual reads W twice: from an LDS copy when it fits
    const int wld = w_lds_stride<PREC>(in.n);
    const size_t wb = w_lds_bytes<MT, PREC>(wld);
    if (wb <= 64 * 1024) {
      hipLaunchKernelGGL((fiber_kernel<MT, NT, CONTIG, RESID, PREC, TIN, TOUT, true>), grid,
                         dim3(kThreads), wb > slds ? wb : slds, s, in, w, m0, mcount, out,
                         partials, stage, wld);
      if (nparts) *nparts = (int)grid.x;
      return hipGetLastError();
    }
    // too large for one copy: the split-bf16 form stages W (hi and lo) through
    // LDS in chunks shared by the block's four waves (measured on the
    // 512x512x256 stream: mode-1 TTM 0.57 -> 0.40 ms). The FP32 form keeps its
    // direct 16-byte reads of W, which measured faster than the chunk copies.
    constexpr size_t cb = chunk_lds_bytes<MT, PREC>();
    if (PREC == 1 && cb <= 64 * 1024) {
      hipLaunchKernelGGL((fiber_kernel<MT, NT, CONTIG, RESID, PREC, TIN, TOUT, false, true>), grid,
                         dim3(kThreads), cb > slds ? cb : slds, s, in, w, m0, mcount, out,
                         partials, stage, 0);
      if (nparts) *nparts = (int)grid.x;
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((fiber_kernel<MT, NT, CONTIG, RESID, PREC, TIN, TOUT, false>), grid,
                     dim3(kThreads), slds, s, in, w, m0, mcount, out, partials, stage, 0);
  if (nparts) *nparts = (int)grid.x;
  return hipGetLastError();
}

template <int MT, int NT, bool CONTIG, bool RESID, class TIN, class TOUT>
hipError_t launch_fiber_p(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                          int *np) {
  if (prec == Prec::BF16X3)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 1, TIN, TOUT>(in, w, m0, mcount, out, partials, s,
                                                               np);
  if (prec == Prec::FP64)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 2, TIN, TOUT>(in, w, m0, mcount, out, partials, s,
                                                               np);
  return launch_fiber_t<MT, NT, CONTIG, RESID, 0, TIN, TOUT>(in, w, m0, mcount, out, partials, s,
                                                             np);
}

template <int MT, int NT, class TIN, class TOUT>
hipError_t launch_fiber_c(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s, int *np) {
  const bool resid = partials != nullptr;
  if constexpr (std::is_same<TIN, float>::value) {
    if (contig) {
      if (resid)
        return launch_fiber_p<MT, NT, true, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s, np);
      return launch_fiber_p<MT, NT, true, false, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s, np);
    }
  }
  if (resid)
    return launch_fiber_p<MT, NT, false, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s, np);
  return launch_fiber_p<MT, NT, false, false, TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s, np);
}

template <int NT, class TIN, class TOUT>
hipError_t launch_fiber_n(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s, int *np) {
  // smallest instantiated tile count >= the rows needed (padding wastes MFMA work)
  const int tiles = (mcount + 15) / 16;
#define ST_FIBER_CASE(T)                                                                        \
  if (tiles <= T)                                                                               \
    return launch_fiber_c<T, NT, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s, np);
  ST_FIBER_CASE(1)
  ST_FIBER_CASE(2)
  ST_FIBER_CASE(3)
  ST_FIBER_CASE(4)
  ST_FIBER_CASE(6)
  ST_FIBER_CASE(8)
  ST_FIBER_CASE(12)
#undef ST_FIBER_CASE
  if (tiles <= 16 || partials == nullptr)
    return launch_fiber_c<16, NT, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s, np);
  return hipErrorInvalidValue;  // fused residual needs all rows in one block
}

inline bool contiguous(const FiberIn &in) {
  return !in.mapped && !in.x64 && in.a == 1 && (in.n & 3) == 0 &&
         (reinterpret_cast<uintptr_t>(in.x) & 15) == 0;
}

// nparts (optional) receives the number of blocks that wrote residual partials;
// it never exceeds fiber_max_blocks(in.F).
template <class TIN, class TOUT>
hipError_t launch_fiber_typed(const FiberIn &in, const FiberW &w, int m0, int mcount,
                              const FiberOut &out, double *partials, Prec prec, hipStream_t s,
                              int *nparts) {
  if (nparts) *nparts = 0;
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  hipError_t rerr = hipSuccess;
  if (try_launch_resid<TIN, TOUT>(in, w, m0, mcount, out, partials, prec, s, rerr, nparts))
    return rerr;
  const bool contig = contiguous(in);
  const int tiles = (mcount + 15) / 16;
  if (partials != nullptr && tiles > 16) {
    // fused residual with more than 256 rows: all of them in one block, one
    // fibre tile per wave
    if (tiles > 24) return hipErrorInvalidValue;
    if constexpr (std::is_same<TIN, float>::value) {
      if (contig) {
        if (tiles <= 20)
          return launch_fiber_p<20, 1, true, true, TIN, TOUT>(in, w, m0, mcount, out, partials,
                                                              prec, s, nparts);
        return launch_fiber_p<24, 1, true, true, TIN, TOUT>(in, w, m0, mcount, out, partials,
                                                            prec, s, nparts);
      }
    }
    if (tiles <= 20)
      return launch_fiber_p<20, 1, false, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec,
                                                           s, nparts);
    return launch_fiber_p<24, 1, false, true, TIN, TOUT>(in, w, m0, mcount, out, partials, prec,
                                                         s, nparts);
  }
  // two fibre tiles per wave when there are enough fibres to fill the chip
  if (in.F >= 256 * 128)
    return launch_fiber_n<2, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s, nparts);
  return launch_fiber_n<1, TIN, TOUT>(in, w, m0, mcount, out, partials, contig, prec, s, nparts);
}

}  // namespace fk
}  // namespace st
