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
// shared by the block's four waves; each wave owns NT x 16 rows.
template <int MT, int NT, int EXTRA, class T>
__global__ __launch_bounds__(kThreads) void rot_kernel(FiberIn in, const T *w, int64_t ldw,
                                                       int m0, int mcount, FiberOut out,
                                                       const double *pvec) {
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
  f64x4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f64x4{0.0, 0.0, 0.0, 0.0};
  double dot[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) dot[nt] = 0.0;

  for (int64_t kb = 0; kb < K; kb += 32) {
    // stage W[mbeg .. mbeg + 16 MT)[kb .. kb + 32) in LDS
    __syncthreads();
    for (int idx = threadIdx.x; idx < MT * 16 * 32; idx += kThreads) {
      const int r = idx >> 5, c = idx & 31;
      const int64_t m = mbeg + r, k = kb + c;
      ws[r * LDW + c] = (m < mend && k < K) ? w[m * ldw + k] : (T)0;
    }
    __syncthreads();
    const int64_t k0 = kb + 8 * grp;
    double xd[NT][8];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int64_t k = k0 + s;
        double x = 0.0;
        if (k < n && base[nt] >= 0) x = (double)xp[base[nt] + in.a * k];
        if (EXTRA == 2 && k < n) dot[nt] += x * pvec[k];
        xd[nt][s] = x;
      }
    }
    if (EXTRA && kb + 32 > n) {  // the block holding element n
      const int sl = (int)(n - kb);
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
        if (grp == (sl >> 3)) {
#pragma unroll
          for (int s = 0; s < 8; ++s)
            if (s == (sl & 7)) xd[nt][s] = ev;
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const T *wr = ws + (16 * mt + col) * LDW + 8 * grp;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const double a = (double)wr[s];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_f64(a, xd[nt][s], acc[mt][nt]);
      }
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
        const int64_t m = mbeg + 16 * mt + acc_row<2>(grp, v);
        if (m < mend) op[fr + out.ao * (m + out.mo * fq)] = (T)acc[mt][nt][v];
      }
  }
}

template <int MT, int NT, class T>
hipError_t launch_rot_t(const FiberIn &in, const T *w, int64_t ldw, int m0, int mcount,
                        const FiberOut &out, int extra_mode, const double *pvec, hipStream_t s) {
  const int64_t per_block = 64 * NT;
  dim3 grid((unsigned)((in.F + per_block - 1) / per_block),
            (unsigned)((mcount + 16 * MT - 1) / (16 * MT)));
  if constexpr (std::is_same<T, double>::value) {
    // the auxiliary matrix: no extra column, or the complement column
    if (extra_mode == 2)
      hipLaunchKernelGGL((rot_kernel<MT, NT, 2, T>), grid, dim3(kThreads), 0, s, in, w, ldw, m0,
                         mcount, out, pvec);
    else if (extra_mode == 0)
      hipLaunchKernelGGL((rot_kernel<MT, NT, 0, T>), grid, dim3(kThreads), 0, s, in, w, ldw, m0,
                         mcount, out, pvec);
    else
      return hipErrorInvalidValue;
  } else {
    // the core: the new row d^T
    if (extra_mode != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((rot_kernel<MT, NT, 1, T>), grid, dim3(kThreads), 0, s, in, w, ldw, m0,
                       mcount, out, pvec);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_rot_typed(const FiberIn &in, const T *w, int64_t ldw, int m0, int mcount,
                            const FiberOut &out, int extra_mode, const double *pvec,
                            hipStream_t s) {
  const int tiles = (mcount + 15) / 16;
  if (tiles <= 2) return launch_rot_t<2, 2, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
  if (tiles <= 4) return launch_rot_t<4, 2, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
  if (tiles <= 6) return launch_rot_t<6, 2, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
  if (tiles <= 8) return launch_rot_t<8, 1, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
  if (tiles <= 10)
    return launch_rot_t<10, 1, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
  return launch_rot_t<12, 1, T>(in, w, ldw, m0, mcount, out, extra_mode, pvec, s);
}

}  // namespace

hipError_t launch_rot64(const FiberIn &in, const void *w, int w64, int64_t ldw, int m0,
                        int mcount, const FiberOut &out, int extra_mode, const double *pvec,
                        hipStream_t s) {
  if (in.F <= 0 || mcount <= 0) return hipSuccess;
  if (!in.mapped || (extra_mode != 0 && in.extra == nullptr) || (extra_mode == 2 && !pvec))
    return hipErrorInvalidValue;
  if ((in.x64 != 0) != (w64 != 0) || (out.o64 != 0) != (w64 != 0)) return hipErrorInvalidValue;
  if (w64)
    return launch_rot_typed<double>(in, static_cast<const double *>(w), ldw, m0, mcount, out,
                                    extra_mode, pvec, s);
  return launch_rot_typed<float>(in, static_cast<const float *>(w), ldw, m0, mcount, out,
                                 extra_mode, pvec, s);
}

}  // namespace st
