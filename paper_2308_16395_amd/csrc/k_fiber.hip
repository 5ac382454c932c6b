// Fibre contractions on MFMA for gfx950: the mode-k TTM of Alg. 4 with its
// fused residual norm, and the Gram of the residual (Alg. 1 applied to E_k).
//
// A mode-k partial core D of shape (r~_1..r~_{k-1}, n_k, ..., n_{d-1}) in
// column-major order is a set of F = a*b fibres of length n = n_k (a = r~_{<k},
// b = n'_{>k}); fibre f = i + a*l starts at (f % a) + a*n*(f / a) with stride a.
// The projection P = D x_k U^T is P[f][m] = sum_j D[f][j] U[j][m]; we compute it
// transposed, P^T = U^T D^T, so that the MFMA accumulator of P^T is directly the
// B operand of the residual product E^T = D^T - U P^T (no data movement).
//
// MFMA 16x16x4 f32 and 16x16x32 bf16: lane L supplies row (L % 16) of A and
// column (L % 16) of B; the accumulator holds D[4*(L/16)+v][L%16], v = 0..3.
// (The 16x16x4 f64 form holds D[(L/16)+4*v][L%16] instead.)
// The K index is free as long as A and B agree: lane L takes the eight K values
// kb + 8*(L/16) + s, s = 0..7, of every 32-wide K block.
#include "common.hpp"

namespace st {

namespace {

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

// Accumulator of one 16x16 output tile: FP32 for the FP32 and bf16 forms, FP64
// for the FP64 form. Lane L, element v holds row acc_row(L/16, v), column L%16.
template <int PREC>
struct AccT {
  using type = f32x4;
};
template <>
struct AccT<2> {
  using type = f64x4;
};
template <int PREC>
__device__ constexpr int acc_row(int grp, int v) {
  return PREC == 2 ? grp + 4 * v : 4 * grp + v;
}

__device__ inline void load_w8_f64(const double *w, int64_t ldw, int64_t m, int64_t mend,
                                   int64_t K, int64_t k0, double (&x)[8]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    x[s] = (m < mend && k < K) ? w[m * ldw + k] : 0.0;
  }
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

// Base offset of fibre f (or -1 for an absent / padded fibre).
__device__ inline int64_t fiber_base(const FiberIn &in, int64_t f) {
  if (f >= in.F) return -1;
  if (in.mapped) return map_new_to_old(in.map, f);
  return (f % in.a) + in.a * in.n * (f / in.a);
}

// Eight consecutive K values kb+8g .. kb+8g+7 of one fibre.
template <bool CONTIG>
__device__ inline void load_x8(const FiberIn &in, int64_t base, int64_t f, int64_t K, int64_t k0,
                               float (&x)[8]) {
  if (CONTIG) {
    if (base >= 0 && k0 + 8 <= K) {
      const f32x4 *p = reinterpret_cast<const f32x4 *>(in.x + base + k0);
      f32x4 u = p[0], v = p[1];
      x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
      x[4] = v[0]; x[5] = v[1]; x[6] = v[2]; x[7] = v[3];
      return;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t k = k0 + s;
      x[s] = (base >= 0 && k < K) ? in.x[base + k] : 0.0f;
    }
    return;
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t k = k0 + s;
    float v = 0.0f;
    if (k < in.n) {
      if (base >= 0) v = in.x[base + in.a * k];
    } else if (k == in.n && in.extra != nullptr && f < in.F) {
      v = in.extra[f];
    }
    x[s] = v;
  }
}

// Eight consecutive K values of row m of the row-major W.
__device__ inline void load_w8(const FiberW &w, int64_t m, int64_t mend, int64_t K, int64_t k0,
                               float (&x)[8]) {
  if (m < mend && k0 + 8 <= K && (w.ldw & 3) == 0) {
    const f32x4 *p = reinterpret_cast<const f32x4 *>(w.w + m * w.ldw + k0);
    f32x4 u = p[0], v = p[1];
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

// acc[mt][nt] += W[m0+16mt.., kb..kb+31] * X[fibres of nt, kb..kb+31]^T for all K.
// Also accumulates the sum of squares of every X element this wave loads.
template <int MT, int NT, bool CONTIG, int PREC, bool NORMX>
__device__ inline void project_wave(const FiberIn &in, const FiberW &w, int64_t m0, int64_t mend,
                                    const int64_t (&fib)[NT], const int64_t (&base)[NT],
                                    typename AccT<PREC>::type (&acc)[MT][NT], double &x2) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t K = in.n + ((in.mapped && in.extra) ? 1 : 0);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = typename AccT<PREC>::type{0, 0, 0, 0};

  for (int64_t kb = 0; kb < K; kb += 32) {
    const int64_t k0 = kb + 8 * grp;
    float xv[NT][8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      load_x8<CONTIG>(in, base[nt], fib[nt], K, k0, xv[nt]);
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
          for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = mfma_f64(wv[s], (double)xv[nt][s], acc[mt][nt]);
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

// R^T tile rows j = 16*jt + 4*grp + v of (U P^T) for the NT fibre tiles, with
// U[j][m] = W[m][j] and P^T in the accumulators (MT tiles over m).
template <int MT, int NT, int PREC>
__device__ inline void recon_tile(const FiberW &w, int64_t rows, int64_t n, int jt,
                                  const typename AccT<PREC>::type (&acc)[MT][NT],
                                  typename AccT<PREC>::type (&racc)[NT]) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t j = 16 * jt + col;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) racc[nt] = typename AccT<PREC>::type{0, 0, 0, 0};
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

// Four consecutive elements j0..j0+3 of a STRIDED fibre.
template <bool CONTIG>
__device__ inline void load_x4(const FiberIn &in, int64_t base, int64_t j0, float (&x)[4]) {
  if (CONTIG && base >= 0 && j0 + 4 <= in.n) {
    f32x4 u = *reinterpret_cast<const f32x4 *>(in.x + base + j0);
    x[0] = u[0]; x[1] = u[1]; x[2] = u[2]; x[3] = u[3];
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t j = j0 + v;
    x[v] = (base >= 0 && j < in.n) ? in.x[base + in.a * j] : 0.0f;
  }
}

template <int MT, int NT, bool CONTIG, bool RESID, int PREC>
__global__ __launch_bounds__(kThreads) void fiber_kernel(FiberIn in, FiberW w, int m0, int mcount,
                                                         FiberOut out, double *partials) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t mbeg = (int64_t)m0 + (int64_t)blockIdx.y * (16 * MT);
  const int64_t mend = (int64_t)m0 + mcount;
  const int64_t fwave = ((int64_t)blockIdx.x * 4 + wid) * (16 * NT);

  int64_t fib[NT], base[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    fib[nt] = fwave + 16 * nt + col;
    base[nt] = fiber_base(in, fib[nt]);
  }
  typename AccT<PREC>::type acc[MT][NT];
  double x2 = 0.0, e2 = 0.0;
  project_wave<MT, NT, CONTIG, PREC, RESID>(in, w, mbeg, mend, fib, base, acc, x2);

  // store P[f][m]
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
        if (m < mend) out.p[fr + out.ao * (m + out.mo * fq)] = (float)acc[mt][nt][v];
      }
  }

  if (RESID) {
    const int jtiles = (int)((in.n + 15) / 16);
    for (int jt = 0; jt < jtiles; ++jt) {
      typename AccT<PREC>::type racc[NT];
      recon_tile<MT, NT, PREC>(w, mcount, in.n, jt, acc, racc);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (fib[nt] >= in.F) continue;
        float xv[4];
        if constexpr (PREC == 2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t j = 16 * jt + grp + 4 * v;
            xv[v] = (base[nt] >= 0 && j < in.n) ? in.x[base[nt] + in.a * j] : 0.0f;
          }
        } else {
          load_x4<CONTIG>(in, base[nt], 16 * jt + 4 * grp, xv);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = 16 * jt + acc_row<PREC>(grp, v);
          if (j < in.n) {
            const double e = (double)xv[v] - (double)racc[nt][v];
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

// ---------------------------------------------------------------------------
// Mode-d rotations with FP64 products and sums (FP32 state in and out).
//
// The rotations V~ = [V v] V'' and C~^T = [C^T d] U'' are applied to the whole
// auxiliary matrix and core on every slice. FP32 accumulation adds a random
// error of about u sqrt(K) per entry per slice; over hundreds of slices that
// perturbs span(V) by more than the ISVD tolerance can absorb (at tau = 1e-4,
// eps / ||d|| is about 4.5e-5), so these products run on the FP64 MFMA: the
// FP32 inputs are exact in FP64 and each output is rounded to FP32 once.
// ---------------------------------------------------------------------------
template <int MT, int NT>
__global__ __launch_bounds__(kThreads) void rot64_kernel(FiberIn in, const double *w, int64_t ldw,
                                                         int m0, int mcount, FiberOut out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t mbeg = (int64_t)m0 + (int64_t)blockIdx.y * (16 * MT);
  const int64_t mend = (int64_t)m0 + mcount;
  const int64_t fwave = ((int64_t)blockIdx.x * 4 + wid) * (16 * NT);
  const int64_t K = in.n + ((in.mapped && in.extra) ? 1 : 0);
  int64_t fib[NT], base[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    fib[nt] = fwave + 16 * nt + col;
    base[nt] = fiber_base(in, fib[nt]);
  }
  f64x4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int64_t kb = 0; kb < K; kb += 32) {
    const int64_t k0 = kb + 8 * grp;
    float xv[NT][8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) load_x8<false>(in, base[nt], fib[nt], K, k0, xv[nt]);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      double wv[8];
      load_w8_f64(w, ldw, mbeg + 16 * mt + col, mend, K, k0, wv);
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = mfma_f64(wv[s], (double)xv[nt][s], acc[mt][nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int64_t f = fib[nt];
    if (f >= in.F) continue;
    const int64_t fq = f / out.ao, fr = f - fq * out.ao;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = mbeg + 16 * mt + grp + 4 * v;  // FP64 accumulator layout
        if (m < mend) out.p[fr + out.ao * (m + out.mo * fq)] = (float)acc[mt][nt][v];
      }
  }
}

template <int MT, int NT>
hipError_t launch_rot64_t(const FiberIn &in, const double *w, int64_t ldw, int m0, int mcount,
                          const FiberOut &out, hipStream_t s) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  hipLaunchKernelGGL((rot64_kernel<MT, NT>), grid, dim3(kThreads), 0, s, in, w, ldw, m0, mcount,
                     out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual Gram. Each block iterates over 64-fibre tiles; every wave forms E^T
// for its 16 fibres (all n rows) into LDS, then the waves accumulate their
// share of the lower-triangular 16x16 tiles of G = sum_f e_f e_f^T.
// ---------------------------------------------------------------------------
constexpr int kGramTPW = 16;  // max tiles per wave per launch group

__device__ inline void tile_ij(int t, int &ti, int &tj) {
  // t enumerates the lower triangle row by row: (0,0), (1,0), (1,1), (2,0)...
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// GP: product precision of the Gram, 0 = FP32, 1 = bf16x3, 2 = FP64 (the FP32
// inputs are exact in FP64, so this accumulates the exact products). The
// residual itself is always recomputed with FP32 products.
template <int MT, bool CONTIG, int GP, int PE>
__global__ __launch_bounds__(kThreads) void gram_kernel(FiberIn in, FiberW w, int rows,
                                                        double *partials, int ntiles) {
  extern __shared__ float es[];  // [n_pad][68]
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t n = in.n;
  const int jtiles = (int)((n + 15) / 16);
  constexpr int LDE = 68;
  const int group0 = blockIdx.y * 4 * kGramTPW;

  f32x4 gacc[kGramTPW];
  f64x4 gacc64[GP == 2 ? kGramTPW : 1];
  int tI[kGramTPW], tJ[kGramTPW];
#pragma unroll
  for (int q = 0; q < kGramTPW; ++q) {
    gacc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (GP == 2) gacc64[q] = f64x4{0.0, 0.0, 0.0, 0.0};
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
    int64_t fib[1] = {fw + col};
    int64_t base[1] = {fiber_base(in, fib[0])};
    if (rows > 0) {
      typename AccT<PE>::type acc[MT][1];
      double dummy = 0.0;
      project_wave<MT, 1, CONTIG, PE, false>(in, w, 0, rows, fib, base, acc, dummy);
      for (int jt = 0; jt < jtiles; ++jt) {
        typename AccT<PE>::type racc[1];
        recon_tile<MT, 1, PE>(w, rows, n, jt, acc, racc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = 16 * jt + acc_row<PE>(grp, v);
          const float x = (base[0] >= 0 && j < n) ? in.x[base[0] + in.a * j] : 0.0f;
          es[j * LDE + wid * 16 + col] = (float)((double)x - (double)racc[0][v]);
        }
      }
    } else {
      for (int jt = 0; jt < jtiles; ++jt) {
        float xv[4];
        load_x4<CONTIG>(in, base[0], 16 * jt + 4 * grp, xv);
#pragma unroll
        for (int v = 0; v < 4; ++v) es[(16 * jt + 4 * grp + v) * LDE + wid * 16 + col] = xv[v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGramTPW; ++q) {
      if (tI[q] < 0) continue;
      const float *ra = es + (16 * tI[q] + col) * LDE;
      const float *rb = es + (16 * tJ[q] + col) * LDE;
#pragma unroll
      for (int kb = 0; kb < 64; kb += 32) {
        float av[8], bv[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          av[s] = ra[kb + 8 * grp + s];
          bv[s] = rb[kb + 8 * grp + s];
        }
        if (GP == 0) {
#pragma unroll
          for (int s = 0; s < 8; ++s) gacc[q] = mfma4(av[s], bv[s], gacc[q]);
        } else if (GP == 1) {
          bf16x8 ah, al, bh, bl;
          split8(av, ah, al);
          split8(bv, bh, bl);
          gacc[q] = mfma_bf(ah, bh, gacc[q]);
          gacc[q] = mfma_bf(ah, bl, gacc[q]);
          gacc[q] = mfma_bf(al, bh, gacc[q]);
        } else {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            gacc64[GP == 2 ? q : 0] = mfma_f64((double)av[s], (double)bv[s], gacc64[GP == 2 ? q : 0]);
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
    // accumulator rows: FP32 and bf16 forms hold row 4*(L/16)+v, the FP64 form
    // holds row (L/16)+4*v (both with column L%16)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (GP == 2)
        dst[(grp + 4 * v) * 16 + col] = gacc64[GP == 2 ? q : 0][v];
      else
        dst[(4 * grp + v) * 16 + col] = (double)gacc[q][v];
    }
  }
}

__global__ void gram_reduce_kernel(const double *partials, int nblocks, int ntiles, int64_t n,
                                   double *G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ntiles * 256) return;
  const int t = (int)(idx / 256), e = (int)(idx % 256);
  int ti, tj;
  tile_ij(t, ti, tj);
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partials[((size_t)b * ntiles + t) * 256 + e];
  const int64_t i = 16 * ti + e / 16, j = 16 * tj + e % 16;
  if (i < n && j < n) {
    G[i + n * j] = s;
    G[j + n * i] = s;
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

template <int MT, int NT, bool CONTIG, bool RESID, int PREC>
hipError_t launch_fiber_t(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, hipStream_t s) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            RESID ? 1u : (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  hipLaunchKernelGGL((fiber_kernel<MT, NT, CONTIG, RESID, PREC>), grid, dim3(kThreads), 0, s, in,
                     w, m0, mcount, out, partials);
  return hipGetLastError();
}

template <int MT, int NT, bool CONTIG, bool RESID>
hipError_t launch_fiber_p(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, Prec prec, hipStream_t s) {
  if (prec == Prec::BF16X3)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 1>(in, w, m0, mcount, out, partials, s);
  if (prec == Prec::FP64)
    return launch_fiber_t<MT, NT, CONTIG, RESID, 2>(in, w, m0, mcount, out, partials, s);
  return launch_fiber_t<MT, NT, CONTIG, RESID, 0>(in, w, m0, mcount, out, partials, s);
}

template <int MT, int NT>
hipError_t launch_fiber_c(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s) {
  const bool resid = partials != nullptr;
  if (contig) {
    if (resid) return launch_fiber_p<MT, NT, true, true>(in, w, m0, mcount, out, partials, prec, s);
    return launch_fiber_p<MT, NT, true, false>(in, w, m0, mcount, out, partials, prec, s);
  }
  if (resid) return launch_fiber_p<MT, NT, false, true>(in, w, m0, mcount, out, partials, prec, s);
  return launch_fiber_p<MT, NT, false, false>(in, w, m0, mcount, out, partials, prec, s);
}

template <int NT>
hipError_t launch_fiber_n(const FiberIn &in, const FiberW &w, int m0, int mcount,
                          const FiberOut &out, double *partials, bool contig, Prec prec,
                          hipStream_t s) {
  // smallest instantiated tile count >= the rows needed (padding wastes MFMA work)
  const int tiles = (mcount + 15) / 16;
#define ST_FIBER_CASE(T) \
  if (tiles <= T) return launch_fiber_c<T, NT>(in, w, m0, mcount, out, partials, contig, prec, s);
  ST_FIBER_CASE(1)
  ST_FIBER_CASE(2)
  ST_FIBER_CASE(3)
  ST_FIBER_CASE(4)
  ST_FIBER_CASE(5)
  ST_FIBER_CASE(6)
  ST_FIBER_CASE(8)
  ST_FIBER_CASE(10)
  ST_FIBER_CASE(12)
#undef ST_FIBER_CASE
  if (tiles <= 16 || partials == nullptr)
    return launch_fiber_c<16, NT>(in, w, m0, mcount, out, partials, contig, prec, s);
  return hipErrorInvalidValue;  // fused residual needs all rows in one block
}

template <int MT, bool CONTIG, int PE>
hipError_t launch_gram_c(const FiberIn &in, const FiberW &w, int rows, double *partials,
                         int nblocks, int gp, hipStream_t s) {
  const int jt = (int)((in.n + 15) / 16);
  const int ntiles = jt * (jt + 1) / 2;
  const int groups = (ntiles + 4 * kGramTPW - 1) / (4 * kGramTPW);
  const size_t lds = (size_t)jt * 16 * 68 * sizeof(float);
  dim3 grid((unsigned)nblocks, (unsigned)groups);
  if (gp == 2) {
    hipFuncSetAttribute((const void *)gram_kernel<MT, CONTIG, 2, PE>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_kernel<MT, CONTIG, 2, PE>), grid, dim3(kThreads), lds, s, in, w, rows,
                       partials, ntiles);
  } else if (gp == 1) {
    hipFuncSetAttribute((const void *)gram_kernel<MT, CONTIG, 1, PE>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_kernel<MT, CONTIG, 1, PE>), grid, dim3(kThreads), lds, s, in, w, rows,
                       partials, ntiles);
  } else {
    hipFuncSetAttribute((const void *)gram_kernel<MT, CONTIG, 0, PE>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_kernel<MT, CONTIG, 0, PE>), grid, dim3(kThreads), lds, s, in, w, rows,
                       partials, ntiles);
  }
  return hipGetLastError();
}

template <int MT>
hipError_t launch_gram_t(const FiberIn &in, const FiberW &w, int rows, double *partials,
                         int nblocks, bool contig, int gp, bool e64, hipStream_t s) {
  if (e64) {
    if (contig) return launch_gram_c<MT, true, 2>(in, w, rows, partials, nblocks, gp, s);
    return launch_gram_c<MT, false, 2>(in, w, rows, partials, nblocks, gp, s);
  }
  if (contig) return launch_gram_c<MT, true, 0>(in, w, rows, partials, nblocks, gp, s);
  return launch_gram_c<MT, false, 0>(in, w, rows, partials, nblocks, gp, s);
}

}  // namespace

static bool contiguous(const FiberIn &in) {
  return !in.mapped && in.a == 1 && (in.n & 3) == 0 &&
         (reinterpret_cast<uintptr_t>(in.x) & 15) == 0;
}

int fiber_blocks(int64_t F) { return (int)((F + 127) / 128); }

hipError_t launch_fiber_project(const FiberIn &in, const FiberW &w, int m0, int mcount,
                                const FiberOut &out, double *resid_partials, Prec prec,
                                hipStream_t s) {
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  const bool contig = contiguous(in);
  // Two fibre tiles per wave when there are enough fibres to fill the chip.
  if (in.F >= 256 * 128) {
    return launch_fiber_n<2>(in, w, m0, mcount, out, resid_partials, contig, prec, s);
  }
  return launch_fiber_n<1>(in, w, m0, mcount, out, resid_partials, contig, prec, s);
}

hipError_t launch_rot64(const FiberIn &in, const double *w, int64_t ldw, int m0, int mcount,
                        const FiberOut &out, hipStream_t s) {
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  const int tiles = (mcount + 15) / 16;
  if (tiles <= 2) return launch_rot64_t<2, 2>(in, w, ldw, m0, mcount, out, s);
  if (tiles <= 4) return launch_rot64_t<4, 2>(in, w, ldw, m0, mcount, out, s);
  if (tiles <= 6) return launch_rot64_t<6, 2>(in, w, ldw, m0, mcount, out, s);
  if (tiles <= 8) return launch_rot64_t<8, 1>(in, w, ldw, m0, mcount, out, s);
  if (tiles <= 12) return launch_rot64_t<12, 1>(in, w, ldw, m0, mcount, out, s);
  return launch_rot64_t<16, 1>(in, w, ldw, m0, mcount, out, s);
}

int gram_blocks(int64_t F) {
  const int64_t t = (F + 63) / 64;
  return (int)(t < 512 ? t : 512);
}

size_t gram_partial_elems(int64_t n, int nblocks) {
  const int64_t jt = (n + 15) / 16;
  return (size_t)nblocks * (size_t)(jt * (jt + 1) / 2) * 256;
}

hipError_t launch_gram(const FiberIn &in, const FiberW &w, int rows, double *partials,
                       int nblocks, GramPrec gp, bool e64, hipStream_t s) {
  if (in.F <= 0) return hipSuccess;
  if (in.n > 512) return hipErrorInvalidValue;  // E tile must fit in LDS
  const bool contig = contiguous(in);
  const int g = (int)gp;
  const int tiles = (rows + 15) / 16;
  if (tiles <= 1) return launch_gram_t<1>(in, w, rows, partials, nblocks, contig, g, e64, s);
  if (tiles <= 2) return launch_gram_t<2>(in, w, rows, partials, nblocks, contig, g, e64, s);
  if (tiles <= 4) return launch_gram_t<4>(in, w, rows, partials, nblocks, contig, g, e64, s);
  if (tiles <= 8) return launch_gram_t<8>(in, w, rows, partials, nblocks, contig, g, e64, s);
  if (tiles <= 16) return launch_gram_t<16>(in, w, rows, partials, nblocks, contig, g, e64, s);
  return hipErrorInvalidValue;
}

hipError_t launch_gram_reduce(const double *partials, int nblocks, int64_t n, double *G,
                              hipStream_t s) {
  const int64_t jt = (n + 15) / 16;
  const int ntiles = (int)(jt * (jt + 1) / 2);
  const int64_t total = (int64_t)ntiles * 256;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     partials, nblocks, ntiles, n, G);
  return hipGetLastError();
}

hipError_t launch_reduce_pairs(const double *partials, int count, double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(1024), 0, s, partials, count, out);
  return hipGetLastError();
}

}  // namespace st
