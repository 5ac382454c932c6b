// Mode-1 projection P = X x_1 U^T with the fused residual norm of Alg. 4
// (E = X - P x_1 U, ||E||^2 and ||X||^2) for contiguous FP32 fibres (the slice
// itself: fibre f is x[f n .. f n + n)), on FP32 or split-bf16 MFMA.
//
// The mode-1 TTM streams the whole slice once; its work per fibre is two small
// dense contractions (n x r and r x n). Each wave owns 16 fibres at a time and
// walks such wave tiles persistently; the block only shares one LDS copy of W
// (and, for split-bf16, of U = W^T). Per wave tile:
//   projection  P^T (16 MT x 16) = W (16 MT x n) X^T (n x 16)
//   residual    E^T (n x 16)    = X^T - U P^T, with P^T taken straight from the
//               accumulators as the B operand (its rows are the K index).
// MFMA 16x16x4 f32: lane L supplies row (L % 16) of A and column (L % 16) of B
// and holds C[4 (L / 16) + v][L % 16]. Lane group g holds the fibre elements
// 16 jt + 4 g + v, which serve as its K share of the projection and are the
// rows of E it holds after the reconstruction, so every element is loaded
// once. MFMA 16x16x32 bf16 takes eight K values per lane (two row tiles).
#include <algorithm>

#include "k_fiber.hpp"

namespace st {

namespace {

using namespace fk;

constexpr int kMaxN = 128;     // longest fibre handled here

__host__ __device__ constexpr int w_pitch(int npad) { return npad + 4; }    // FP32 W
__host__ __device__ constexpr int wb_pitch(int npad) { return npad + 8; }   // bf16 W

// bf16x3 also keeps U = W^T (rows j, the K = m of the reconstruction
// contiguous, padded to whole 32-wide K blocks) so both products read vectors.
template <int MT>
__host__ __device__ constexpr int ut_cols() { return 32 * ((MT + 1) / 2); }
__host__ __device__ constexpr int ut_pitch(int cols) { return cols + 8; }

template <int MT, int PREC>
__host__ __device__ constexpr size_t contig_lds_bytes(int npad) {
  return PREC == 0 ? (size_t)16 * MT * w_pitch(npad) * 4
                   : (size_t)2 * 16 * MT * wb_pitch(npad) * 2 +
                         (size_t)2 * npad * ut_pitch(ut_cols<MT>()) * 2;
}

// One wave owns 16 fibres at a time (a wave tile) and walks wave tiles
// persistently; the block only shares the LDS copy of W. Lane (col, g) holds
// the elements k = 16 jt + 4 g + v (jt < JT, v < 4) of fibre col: they are
// its K share in the projection (lane group g supplies k = 16 jt + 4 g + v in
// MFMA step (jt, v)) and exactly the rows of E it holds after the
// reconstruction MFMAs of row tile jt, so each element is loaded once, as 16
// bytes, and the next wave tile's loads are in flight during this one's work.
// JT (16-row tiles per fibre) is a template parameter so that the tile loop
// has no data-dependent branches; rows past n are zero in W and in X.
template <int MT, int JT, int PREC, class TOUT, bool RESID>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void ttm_contig_kernel(
    const float *__restrict__ x, int64_t F, int n, FiberW w, int rows, TOUT *__restrict__ out,
    int64_t mo, double *partials, int64_t ntiles) {
  extern __shared__ double lds_raw[];
  constexpr int npad = 16 * JT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  float *ws = reinterpret_cast<float *>(lds_raw);  // FP32 W (16 MT rows, pitch wp)
  constexpr int wp = w_pitch(npad);
  __bf16 *wh = reinterpret_cast<__bf16 *>(lds_raw);  // bf16x3: hi then lo (pitch wbp)
  constexpr int wbp = wb_pitch(npad);
  __bf16 *wl = wh + 16 * MT * wbp;
  constexpr int utc = ut_cols<MT>(), ubp = ut_pitch(utc);
  __bf16 *uh = wl + 16 * MT * wbp;  // bf16x3: U^T hi then lo (npad rows, pitch ubp)
  __bf16 *ul = uh + npad * ubp;

  // W (rows x n, row-major) into LDS once; rows >= `rows` and columns >= n are
  // zero, so every lane reads whole vectors.
  for (int idx = tid; idx < 16 * MT * npad; idx += 256) {
    const int m = idx / npad, k = idx - m * npad;
    const bool ok = m < rows && k < n;
    if constexpr (PREC == 0) {
      ws[m * wp + k] = ok ? w.w[(int64_t)m * w.ldw + k] : 0.0f;
    } else {
      wh[m * wbp + k] = ok ? w.w_hi[(int64_t)m * w.ldw_bf + k] : (__bf16)0.0f;
      wl[m * wbp + k] = ok ? w.w_lo[(int64_t)m * w.ldw_bf + k] : (__bf16)0.0f;
    }
  }
  if constexpr (PREC == 1) {
    for (int idx = tid; idx < npad * utc; idx += 256) {
      const int j = idx / utc, m = idx - j * utc;
      const bool ok = m < rows && j < n;
      uh[j * ubp + m] = ok ? w.w_hi[(int64_t)m * w.ldw_bf + j] : (__bf16)0.0f;
      ul[j * ubp + m] = ok ? w.w_lo[(int64_t)m * w.ldw_bf + j] : (__bf16)0.0f;
    }
  }
  __syncthreads();

  // Per-lane element offsets inside a wave tile (the same for every tile). A
  // chunk past the fibre, or of a fibre past the tensor, reads the tile's first
  // chunk and is zeroed when the tile is consumed; the loaded registers are not
  // touched before that, so the loads stay in flight.
  const int koff = col * n + 4 * grp;
  int off[JT];
  uint32_t kmask = 0;
#pragma unroll
  for (int jt = 0; jt < JT; ++jt) {
    const bool ok = 16 * jt + 4 * grp < n;
    off[jt] = ok ? koff + 16 * jt : 0;
    kmask |= (ok ? 1u : 0u) << jt;
  }
  const bool kfull = n == npad;  // every chunk of a fibre is data
  // the next wave tile is in flight while this one is consumed
  f32x4 nxt[JT];
  bool fnext = true;  // the fetched tile holds 16 fibres
  bool fcol = true;   // this lane's fibre of the fetched tile exists
  auto fetch = [&](int64_t t) {
    const float *base = x + t * 16 * (int64_t)n;
    fnext = t * 16 + 16 <= F;
    fcol = t * 16 + col < F;
    const int sel = fcol ? 1 : 0;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
      nxt[jt] = *reinterpret_cast<const f32x4 *>(base + sel * off[jt]);
  };

  const int64_t wave0 = (int64_t)blockIdx.x * 4 + wid;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int64_t ocol = mo * col;
  double e2 = 0.0, x2 = 0.0;
  if (wave0 < ntiles) fetch(wave0);
  for (int64_t t = wave0; t < ntiles; t += nwaves) {
    const bool full = fnext, fib_ok = fcol;
    f32x4 xv[JT];
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) xv[jt] = nxt[jt];
    if (!(full && kfull)) {  // (uniform) zero the chunks that are not data
      const uint32_t okm = fib_ok ? kmask : 0u;
#pragma unroll
      for (int jt = 0; jt < JT; ++jt)
        if (!((okm >> jt) & 1u)) xv[jt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    if (t + nwaves < ntiles) fetch(t + nwaves);

    // projection P^T = W X^T: MT independent accumulator chains
    AccT<0> acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = AccT<0>{0, 0, 0, 0};
    if constexpr (PREC == 0) {
      // W operands of step jt + 1 are read while the MFMAs of step jt run; the
      // scheduling barriers keep the compiler from hoisting every step's reads
      // at once (which costs more registers than a wave has)
      const float *wrow = ws + col * wp + 4 * grp;
      f32x4 wv[MT], wn[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        wv[mt] = *reinterpret_cast<const f32x4 *>(wrow + 16 * mt * wp);
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
        if (jt + 1 < JT) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            wn[mt] = *reinterpret_cast<const f32x4 *>(wrow + 16 * mt * wp + 16 * (jt + 1));
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma4(wv[mt][v], xv[jt][v], acc[mt]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) wv[mt] = wn[mt];
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // K blocks of 32 for the bf16 MFMA: lane group g supplies the eight K
      // values {16 jt + 4 g + v} of row tiles jt = 2 b, 2 b + 1; the W operands
      // of block b + 1 are read while the MFMAs of block b run
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      auto wload = [&](const __bf16 *base, int b, int mt) {
        const __bf16 *r = base + (16 * mt + col) * wbp + 32 * b + 4 * grp;
        const bf16x4 lo4 = *reinterpret_cast<const bf16x4 *>(r);
        const bf16x4 hi4 = *reinterpret_cast<const bf16x4 *>(r + 16);
        return bf16x8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]};
      };
      bf16x8 ah[MT], al[MT], ahn[MT], aln[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        ah[mt] = wload(wh, 0, mt);
        al[mt] = wload(wl, 0, mt);
      }
#pragma unroll
      for (int b = 0; b < JT / 2; ++b) {
        if (b + 1 < JT / 2) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            ahn[mt] = wload(wh, b + 1, mt);
            aln[mt] = wload(wl, b + 1, mt);
          }
        }
        float xf[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          xf[v] = xv[2 * b][v];
          xf[4 + v] = xv[2 * b + 1][v];
        }
        bf16x8 xh, xl;
        split8(xf, xh, xl);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma_bf(ah[mt], xh, acc[mt]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma_bf(ah[mt], xl, acc[mt]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma_bf(al[mt], xh, acc[mt]);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          ah[mt] = ahn[mt];
          al[mt] = aln[mt];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // P[fib][m] for m = 16 mt + 4 grp + v (all row tiles but the last are full)
    if (fib_ok) {
      TOUT *op = out + mo * (t * 16) + ocol;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * mt + 4 * grp + v;
          if (mt < MT - 1 || m < rows) op[m] = (TOUT)acc[mt][v];
        }
    }

    if constexpr (RESID) {
      // E^T = X^T - U P^T for all row tiles at once: JT independent chains
      AccT<0> racc[JT];
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) racc[jt] = AccT<0>{0, 0, 0, 0};
      if constexpr (PREC == 0) {
        // K steps (mt, v): the JT operands of the next step are read while the
        // MFMAs of this one run (pipelined as in the projection)
        const float *wcol = ws + 4 * grp * wp + col;
        float a[JT], an[JT];
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) a[jt] = wcol[16 * jt];
#pragma unroll
        for (int st = 0; st < 4 * MT; ++st) {
          const int mt = st / 4, v = st % 4;
          if (st + 1 < 4 * MT) {
            const int m1 = 16 * ((st + 1) / 4) + (st + 1) % 4;
#pragma unroll
            for (int jt = 0; jt < JT; ++jt) an[jt] = wcol[m1 * wp + 16 * jt];
          }
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) racc[jt] = mfma4(a[jt], acc[mt][v], racc[jt]);
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) a[jt] = an[jt];
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // K blocks q of 32 rows m of P: lane group g supplies
        // m = 16 (2 q + s / 4) + 4 g + s % 4, the rows its accumulators hold;
        // A = U[16 jt + col][those m] as two 4-element runs of U^T
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        auto uload = [&](const __bf16 *base, int q, int jt) {
          const __bf16 *r = base + (16 * jt + col) * ubp + 32 * q + 4 * grp;
          const bf16x4 lo4 = *reinterpret_cast<const bf16x4 *>(r);
          const bf16x4 hi4 = *reinterpret_cast<const bf16x4 *>(r + 16);
          return bf16x8{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]};
        };
#pragma unroll
        for (int q = 0; q < (MT + 1) / 2; ++q) {
          float pv[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            const int mt = 2 * q + s / 4;
            pv[s] = mt < MT ? acc[mt < MT ? mt : 0][s & 3] : 0.0f;
          }
          bf16x8 ph, pl;
          split8(pv, ph, pl);
          bf16x8 uh0 = uload(uh, q, 0), ul0 = uload(ul, q, 0);
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) {
            bf16x8 uh1 = uh0, ul1 = ul0;
            if (jt + 1 < JT) {
              uh1 = uload(uh, q, jt + 1);
              ul1 = uload(ul, q, jt + 1);
            }
            racc[jt] = mfma_bf(uh0, ph, racc[jt]);
            racc[jt] = mfma_bf(uh0, pl, racc[jt]);
            racc[jt] = mfma_bf(ul0, ph, racc[jt]);
            uh0 = uh1;
            ul0 = ul1;
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      // norms: padded elements are zero in X and in U P^T, so they add nothing.
      // x - (U P^T) is formed in FP32 (its rounding is relative to the residual
      // itself, which is all the norm needs); ||X||^2 is summed in FP64, the
      // squared residuals of a lane and tile in FP32 first.
      if (fib_ok) {
        float e2t = 0.0f;
#pragma unroll
        for (int jt = 0; jt < JT; ++jt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float e = xv[jt][v] - racc[jt][v];
            e2t = fmaf(e, e, e2t);
            const double xd = (double)xv[jt][v];
            x2 = fma(xd, xd, x2);
          }
        e2 += (double)e2t;
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
    if (tid == 0) {
      partials[2 * blockIdx.x + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
      partials[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
  }
}

int g_num_cu = 0;

int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cu > 0)
      g_num_cu = cu;
    else
      g_num_cu = 256;
  }
  return g_num_cu;
}

template <int MT, int JT, int PREC, class TOUT, bool RESID>
hipError_t launch_contig_t(const FiberIn &in, const FiberW &w, int rows, const FiberOut &out,
                           double *partials, hipStream_t s, int *nparts) {
  const int64_t ntiles = (in.F + 15) / 16;  // wave tiles of 16 fibres
  const size_t lds = contig_lds_bytes<MT, PREC>(16 * JT);
  // persistent: as many blocks as fit a CU at once (three waves per SIMD at
  // most, by registers; fewer when the W copies fill the LDS)
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(3, (160 * 1024) / (int64_t)lds));
  const int64_t nb = std::min<int64_t>((ntiles + 3) / 4, per_cu * (int64_t)num_cu());
  const void *fn = (const void *)ttm_contig_kernel<MT, JT, PREC, TOUT, RESID>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ttm_contig_kernel<MT, JT, PREC, TOUT, RESID>), dim3((unsigned)nb),
                     dim3(256), lds, s, static_cast<const float *>(in.x), in.F, (int)in.n, w,
                     rows, static_cast<TOUT *>(out.p), out.mo, partials, ntiles);
  if (nparts) *nparts = RESID ? (int)nb : 0;
  return hipGetLastError();
}

template <int MT, int JT, int PREC>
hipError_t launch_contig_o(const FiberIn &in, const FiberW &w, int rows, const FiberOut &out,
                           double *partials, hipStream_t s, int *nparts) {
  // (FP64 output always comes with the residual norms: the update's first pass)
  if (out.o64)
    return partials
               ? launch_contig_t<MT, JT, PREC, double, true>(in, w, rows, out, partials, s, nparts)
               : hipErrorNotSupported;
  return partials
             ? launch_contig_t<MT, JT, PREC, float, true>(in, w, rows, out, partials, s, nparts)
             : launch_contig_t<MT, JT, PREC, float, false>(in, w, rows, out, partials, s, nparts);
}

template <int MT, int PREC>
hipError_t launch_contig_m(const FiberIn &in, const FiberW &w, int rows, const FiberOut &out,
                           double *partials, hipStream_t s, int *nparts) {
  if (in.n <= 32) return launch_contig_o<MT, 2, PREC>(in, w, rows, out, partials, s, nparts);
  if (in.n <= 64) return launch_contig_o<MT, 4, PREC>(in, w, rows, out, partials, s, nparts);
  return launch_contig_o<MT, 8, PREC>(in, w, rows, out, partials, s, nparts);
}

template <int PREC>
hipError_t launch_contig_p(const FiberIn &in, const FiberW &w, int rows, const FiberOut &out,
                           double *partials, hipStream_t s, int *nparts) {
  switch ((rows + 15) / 16) {
    case 1: return launch_contig_m<1, PREC>(in, w, rows, out, partials, s, nparts);
    case 2: return launch_contig_m<2, PREC>(in, w, rows, out, partials, s, nparts);
    case 3: return launch_contig_m<3, PREC>(in, w, rows, out, partials, s, nparts);
    default: return launch_contig_m<4, PREC>(in, w, rows, out, partials, s, nparts);
  }
}

}  // namespace

bool ttm_contig_eligible(const FiberIn &in, int m0, int mcount, const FiberOut &out,
                         Prec prec, bool resid) {
  return !in.x64 && !in.mapped && in.a == 1 && m0 == 0 && mcount >= 1 && mcount <= 64 &&
         in.n >= 4 && in.n <= kMaxN && in.n % 4 == 0 && in.F >= 1 && prec != Prec::FP64 &&
         out.ao == 1 && ((uintptr_t)in.x & 15) == 0 && (resid || !out.o64);
}

hipError_t launch_ttm_contig(const FiberIn &in, const FiberW &w, int mcount, const FiberOut &out,
                             double *partials, Prec prec, hipStream_t s, int *nparts) {
  if (prec == Prec::FP32)
    return launch_contig_p<0>(in, w, mcount, out, partials, s, nparts);
  return launch_contig_p<1>(in, w, mcount, out, partials, s, nparts);
}

}  // namespace st
