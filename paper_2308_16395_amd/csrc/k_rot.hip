// Mode-d rotations of the streaming update (Alg. 3 applied to V, and the core
// update of Alg. 5) with FP64 products and sums.
//
// The rotations V~ = [V v] V'' and C~^T = [C^T d] U'' are applied to the whole
// auxiliary matrix and core on every slice. V decides the later rank tests: the
// ISVD residual q = ||(I - V V^T) d|| is compared with eps, and at tau = 1e-4
// eps / ||d|| is about 4.5e-5, so V, its rotation matrix and the products are
// all FP64. The core only feeds the reconstruction; it is FP32 with FP32 W,
// FP64 products and one rounding per output.
#include "k_fiber.hpp"

namespace st {

namespace {

using namespace fk;

// EXTRA: 0 none; 1 element n of fibre f is extra[f]; 2 element n is
// e[f] = extra[f] - sum_k X[f][k] p[k] formed in FP64 from the row itself
// (the ISVD complement e = d - V p, never stored).
// W (type T, row-major) is staged through LDS one 32-wide K block at a time and
// shared by the block's four waves; each wave owns NT x 16 rows. The register
// budget is that of two waves per SIMD (256 VGPRs, accumulators included: the
// library builds this file with the MFMA operands in VGPRs), so one wave's
// LDS and global latency is covered by the other's MFMAs.
// W prefetch for the FP32 core up to 11 column tiles (fits the budget below)
template <class T, int MT>
constexpr bool kRotPrefetchW = std::is_same<T, float>::value && MT <= 11;

// F32M (FP32 core only): the products run on the FP32 MFMA, summed in FP32
// within each 32-wide K block (eight MFMA steps), and the block sums are added
// in FP64. Each output then carries about one FP32 rounding per K block on top
// of the final rounding to FP32, instead of exact products.
template <int MT, int NT, int EXTRA, class T, bool F32M>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void rot_kernel(
    FiberIn in, const T *w, int64_t ldw, int m0, int mcount, FiberOut out, const double *pvec) {
  constexpr int LDW = std::is_same<T, double>::value ? 33 : 36;  // LDS row stride of W
  __shared__ T ws[MT * 16 * LDW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t mbeg = (int64_t)m0 + (int64_t)blockIdx.y * (16 * MT);
  const int64_t mend = (int64_t)m0 + mcount;
  const int64_t fwave = ((int64_t)blockIdx.x * 4 + wid) * (16 * NT);
  const int64_t n = in.n;
  const int64_t K = n + (EXTRA ? 1 : 0);
  const T *xp = cptr<T>(in.x);
  T *op = reinterpret_cast<T *>(out.p);
  int64_t fib[NT], base[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    fib[nt] = fwave + 16 * nt + col;
    base[nt] = fib[nt] < in.F ? map_new_to_old(in.map, fib[nt]) : -1;
  }
  static_assert(!F32M || std::is_same<T, float>::value, "FP32 MFMA for the FP32 core only");
  using AccV = typename std::conditional<F32M, f32x4, f64x4>::type;
  AccV acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = AccV{0, 0, 0, 0};
  // F32M: FP64 totals of the per-block FP32 sums (rows 4 grp + v)
  double tot[F32M ? MT : 1][F32M ? NT : 1][4];
#pragma unroll
  for (int mt = 0; mt < (F32M ? MT : 1); ++mt)
#pragma unroll
    for (int nt = 0; nt < (F32M ? NT : 1); ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) tot[mt][nt][v] = 0.0;
  auto flush = [&]() {
    if constexpr (F32M) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
          for (int v = 0; v < 4; ++v) tot[mt][nt][v] += (double)acc[mt][nt][v];
          acc[mt][nt] = AccV{0, 0, 0, 0};
        }
    }
  };
  double dot[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) dot[nt] = 0.0;

  // The X values of K block kb + 32 (the HBM stream) are loaded into registers
  // while the MFMAs consume block kb; the W slice (small, L2-resident) is
  // staged into LDS at the top of each block. All loads are unconditional:
  // rows of W past mend are clamped (they only feed output rows that are not
  // stored), out-of-range K and X elements read a valid element and are
  // replaced by zero, so the loads of a block issue back to back. The mask
  // xok (bit 8 nt + s: element in range) is applied when the block is
  // consumed, so that the prefetch stays in flight.
  constexpr int WPT = MT * 16 * 32 / kThreads;  // W elements staged per thread
  T xreg[NT][8];
  uint32_t xok = 0;
  auto load_x = [&](int64_t kb) {
    xok = 0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t k = kb + 4 * s + grp;
        const bool ok = k < n && base[nt] >= 0;
        xreg[nt][s] = xp[ok ? base[nt] + in.a * k : 0];
        xok |= (ok ? 1u : 0u) << (8 * nt + s);
      }
  };
  const int wc = threadIdx.x & 31, wr0 = threadIdx.x >> 5;
  // Where the registers allow (PW), the W slice of the next block is fetched
  // with the X prefetch; otherwise it is loaded at the top of its own block.
  constexpr bool PW = kRotPrefetchW<T, MT> && !F32M;
  T wv[WPT];
  auto load_w = [&](int64_t kb) {
    const int64_t kk = (kb + wc < K) ? kb + wc : 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int64_t m = mbeg + wr0 + 8 * q;
      wv[q] = w[(m < mend ? m : mend - 1) * ldw + kk];
    }
  };
  // stage K block kb: W into LDS, X (and the ISVD dot) into xd; start the
  // prefetch of the next block
  auto stage = [&](int64_t kb, double (&xd)[NT][8]) {
    if (!PW) load_w(kb);
    const bool kok = kb + wc < K;
    double pv[8];
    if (EXTRA == 2) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t k = kb + 4 * s + grp;
        pv[s] = pvec[k < n ? k : n - 1];  // multiplies a zero X element when k >= n
      }
    }
    __syncthreads();  // the previous block's LDS reads are done
#pragma unroll
    for (int q = 0; q < WPT; ++q) ws[(wr0 + 8 * q) * LDW + wc] = kok ? wv[q] : (T)0;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int s = 0; s < 8; ++s)
        xd[nt][s] = ((xok >> (8 * nt + s)) & 1u) ? (double)xreg[nt][s] : 0.0;
    if (EXTRA == 2) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int s = 0; s < 8; ++s) dot[nt] += xd[nt][s] * pv[s];
    }
    __syncthreads();
    if (kb + 32 < K) {
      load_x(kb + 32);
      if (PW) load_w(kb + 32);
    }
  };
  // MFMA s covers k = kb + 4 s .. kb + 4 s + 3 (lane group grp holds
  // k = kb + 4 s + grp); the MT column tiles of one step are independent. The
  // W values of step s + 1 are read from LDS while the MFMAs of step s run;
  // the scheduling barrier keeps the compiler from hoisting the reads of all
  // steps at once (which would cost 2 MT registers per step).
  const T *wl = ws + col * LDW + grp;
  auto steps = [&](int count, const double (&xd)[NT][8]) {
    T wa[2][MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) wa[0][mt] = wl[16 * mt * LDW];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (s < count) {
        if (s + 1 < 8 && s + 1 < count) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) wa[(s + 1) & 1][mt] = wl[16 * mt * LDW + 4 * (s + 1)];
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            if constexpr (F32M)
              acc[mt][nt] = mfma4((float)wa[s & 1][mt], (float)xd[nt][s], acc[mt][nt]);
            else
              acc[mt][nt] = mfma_f64((double)wa[s & 1][mt], xd[nt][s], acc[mt][nt]);
          }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  // full blocks below kmain hold no extra element; the last block [kmain, K)
  // holds element n when there is one
  const int64_t kmain = EXTRA ? (n / 32) * 32 : (K / 32) * 32;
  load_x(0);
  if (PW) load_w(0);
  for (int64_t kb = 0; kb < kmain; kb += 32) {
    double xd[NT][8];
    stage(kb, xd);
    steps(8, xd);
    flush();
  }
  if (kmain < K) {
    double xd[NT][8];
    stage(kmain, xd);
    if (EXTRA) {
      const int sl = (int)(n - kmain);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        double ev = 0.0;
        if (EXTRA == 2) {
          // lanes col, col + 16, col + 32, col + 48 hold the partial dots of one row
          double full = dot[nt];
          full += __shfl_xor(full, 16, 64);
          full += __shfl_xor(full, 32, 64);
          if (fib[nt] < in.F) ev = in.extra[fib[nt]] - full;
        } else if (fib[nt] < in.F) {
          ev = in.extra[fib[nt]];
        }
        if (grp == (sl & 3)) {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (s == (sl >> 2)) xd[nt][s] = ev;
        }
      }
    }
    // steps wholly past K are skipped
    steps((int)((K - kmain + 3) >> 2), xd);
    flush();
  }
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
        if constexpr (F32M) {
          const int64_t m = mbeg + 16 * mt + acc_row<0>(grp, v);
          if (m < mend) op[fr + out.ao * (m + out.mo * fq)] = (T)tot[mt][nt][v];
        } else {
          const int64_t m = mbeg + 16 * mt + acc_row<2>(grp, v);
          if (m < mend) op[fr + out.ao * (m + out.mo * fq)] = (T)acc[mt][nt][v];
        }
      }
  }
}

template <int MT, int NT, class T>
hipError_t launch_rot_t(const FiberIn &in, const T *w, int64_t ldw, int m0, int mcount,
                        const FiberOut &out, int extra_mode, const double *pvec, int f32m,
                        hipStream_t s) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  if constexpr (std::is_same<T, double>::value) {
    // the auxiliary matrix: no extra column, or the complement column
    if (extra_mode == 2)
      hipLaunchKernelGGL((rot_kernel<MT, NT, 2, T, false>), grid, dim3(kThreads), 0, s, in, w, ldw, m0,
                         mcount, out, pvec);
    else if (extra_mode == 0)
      hipLaunchKernelGGL((rot_kernel<MT, NT, 0, T, false>), grid, dim3(kThreads), 0, s, in, w, ldw, m0,
                         mcount, out, pvec);
    else
      return hipErrorInvalidValue;
  } else {
    // the core: the new row d^T
    if (extra_mode != 1) return hipErrorInvalidValue;
    if (f32m)
      hipLaunchKernelGGL((rot_kernel<MT, NT, 1, T, true>), grid, dim3(kThreads), 0, s, in, w, ldw,
                         m0, mcount, out, pvec);
    else
      hipLaunchKernelGGL((rot_kernel<MT, NT, 1, T, false>), grid, dim3(kThreads), 0, s, in, w,
                         ldw, m0, mcount, out, pvec);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_rot_typed(const FiberIn &in, const T *w, int64_t ldw, int m0, int mcount,
                            const FiberOut &out, int extra_mode, const double *pvec, int f32m,
                            hipStream_t s) {
  // the smallest instantiated column-tile count that covers mcount (padding
  // columns cost whole MFMAs); wider outputs take several column blocks
  const int tiles = (mcount + 15) / 16;
#define ST_ROT_CASE(T_, NT_) \
  if (tiles <= T_) return launch_rot_t<T_, NT_, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, f32m, s);
  // narrow outputs reuse each staged W value for two fibre tiles; wide ones
  // keep one fibre tile per wave so that the accumulators fit two waves per SIMD
  constexpr int NT6 = std::is_same<T, double>::value ? 1 : 2;
  ST_ROT_CASE(2, 2)
  ST_ROT_CASE(4, 2)
  ST_ROT_CASE(6, NT6)
  ST_ROT_CASE(8, 1)
  ST_ROT_CASE(9, 1)
  ST_ROT_CASE(10, 1)
  ST_ROT_CASE(11, 1)
#undef ST_ROT_CASE
  return launch_rot_t<12, 1, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, f32m, s);
}

}  // namespace

hipError_t launch_rot64(const FiberIn &in, const void *w, int w64, int64_t ldw, int m0,
                        int mcount, const FiberOut &out, int extra_mode, const double *pvec,
                        hipStream_t s, int f32m) {
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  if (!in.mapped || (extra_mode != 0 && in.extra == nullptr) || (extra_mode == 2 && !pvec))
    return hipErrorInvalidValue;
  if ((in.x64 != 0) != (w64 != 0) || (out.o64 != 0) != (w64 != 0)) return hipErrorInvalidValue;
  if (w64)
    return launch_rot_typed<double>(in, static_cast<const double *>(w), ldw, m0, mcount, out,
                                    extra_mode, pvec, 0, s);
  return launch_rot_typed<float>(in, static_cast<const float *>(w), ldw, m0, mcount, out,
                                 extra_mode, pvec, f32m, s);
}

}  // namespace st
