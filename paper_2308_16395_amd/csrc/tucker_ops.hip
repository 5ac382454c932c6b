// Reconstruct and Project of a Tucker model and their vector-Jacobian
// products, as chains of mode-k TTMs (the multi-TTM identities of Sec. 2.1:
// X_(k) = U_k G_(k) K_k^T with K_k the Kronecker product of the other factors).
//
//   Reconstruct: X^ = G x_1 U_1 ... x_d U_d.
//     VJP for an upstream gradient R (shaped like X^):
//       dG   = R x_1 U_1^T ... x_d U_d^T
//       dU_k = (R x_{j != k} U_j^T)_(k) G_(k)^T
//   Project: G = X x_1 U_1^T ... x_d U_d^T.
//     VJP for an upstream gradient Gb (shaped like G):
//       dX   = Gb x_1 U_1 ... x_d U_d
//       dU_k = (X x_{j != k} U_j^T)_(k) Gb_(k)^T
//
// Every TTM runs on the MFMA fibre kernels. The partial chains of dU_k are
// recomputed from the shared prefix Z_k = A x_1 U_1^T ... x_k U_k^T rather than
// stored, so the whole set costs about two full-size projections. The final
// contraction dU_k = Y_(k) B_(k)^T is a long-K, small-output product reduced in
// FP64 with per-block partials summed in a fixed order.
#include <algorithm>
#include <cstring>
#include <string>

#include "../../include/stucker.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace st;

namespace {

constexpr size_t kAlign = 256;
constexpr int kCrossFT = 16;   // fibres per LDS tile
constexpr int kCrossOPT = 8;   // outputs per thread
constexpr int kCrossMaxBlocks = 240;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t round8(int64_t x) { return (x + 7) / 8 * 8; }

// Workspace layout for one (dims, ranks, precision).
struct Plan {
  int d = 0;
  int64_t n[ST_MAX_MODES] = {}, r[ST_MAX_MODES] = {};
  Prec prec = Prec::FP32;
  // factor copies: Ut (row-major U, for x_k U_k), FP64 forms, bf16 splits
  size_t ut[ST_MAX_MODES] = {}, u64[ST_MAX_MODES] = {}, ut64[ST_MAX_MODES] = {};
  size_t ph[ST_MAX_MODES] = {}, pl[ST_MAX_MODES] = {}, eh[ST_MAX_MODES] = {},
         el[ST_MAX_MODES] = {};
  int64_t ldb_p[ST_MAX_MODES] = {}, ldb_e[ST_MAX_MODES] = {};
  size_t buf[4] = {};
  int64_t buf_elems = 1;
  size_t part = 0;
  int64_t part_elems = 1;
  size_t total = 0;
};

int64_t prod(const int64_t *v, int from, int to) {
  int64_t p = 1;
  for (int k = from; k < to; ++k) p *= v[k];
  return p;
}

int cross_blocks_x(int64_t F) {
  const int64_t t = (F + kCrossFT - 1) / kCrossFT;
  return (int)std::max<int64_t>(1, std::min<int64_t>(t, kCrossMaxBlocks));
}

int make_plan(int32_t d, const int64_t *dims, const int64_t *ranks, int32_t precision,
              Plan &p) {
  if (d < 1 || d > ST_MAX_MODES || !dims || !ranks || precision < ST_FP32 ||
      precision > ST_FP64)
    return ST_EINVAL;
  p.d = d;
  for (int k = 0; k < d; ++k) {
    if (dims[k] < 1 || ranks[k] < 1 || ranks[k] > dims[k] || dims[k] > (1 << 20))
      return ST_EINVAL;
    p.n[k] = dims[k];
    p.r[k] = ranks[k];
  }
  if (prod(p.n, 0, d) > ((int64_t)1 << 34)) return ST_EINVAL;
  p.prec = precision == ST_BF16X3 ? Prec::BF16X3
                                  : (precision == ST_FP64 ? Prec::FP64 : Prec::FP32);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return at;
  };
  for (int k = 0; k < d; ++k) {
    const int64_t nr = p.n[k] * p.r[k];
    p.ut[k] = take(nr * sizeof(float));
    if (p.prec == Prec::FP64) {
      p.u64[k] = take(nr * sizeof(double));
      p.ut64[k] = take(nr * sizeof(double));
    }
    if (p.prec == Prec::BF16X3) {
      p.ldb_p[k] = round8(p.n[k]);  // rows r_k of U^T
      p.ldb_e[k] = round8(p.r[k]);  // rows n_k of U
      p.ph[k] = take(p.r[k] * p.ldb_p[k] * sizeof(__bf16));
      p.pl[k] = take(p.r[k] * p.ldb_p[k] * sizeof(__bf16));
      p.eh[k] = take(p.n[k] * p.ldb_e[k] * sizeof(__bf16));
      p.el[k] = take(p.n[k] * p.ldb_e[k] * sizeof(__bf16));
    }
  }
  // largest intermediate of the reconstruct chain, the projection prefix and
  // the partial chains of the factor gradients
  int64_t mx = 1;
  for (int k = 0; k + 1 < d; ++k) {
    mx = std::max(mx, prod(p.n, 0, k + 1) * prod(p.r, k + 1, d));  // reconstruct
    mx = std::max(mx, prod(p.r, 0, k + 1) * prod(p.n, k + 1, d));  // project prefix
    for (int m = k + 1; m < d; ++m)
      mx = std::max(mx, prod(p.r, 0, k) * p.n[k] * prod(p.r, k + 1, m + 1) *
                            prod(p.n, m + 1, d));
  }
  p.buf_elems = mx;
  for (int i = 0; i < 4; ++i) p.buf[i] = take(mx * sizeof(float));
  int64_t pe = 1;
  for (int k = 0; k < d; ++k) {
    const int64_t F = prod(p.r, 0, k) * prod(p.r, k + 1, d);
    pe = std::max(pe, (int64_t)cross_blocks_x(F) * p.n[k] * p.r[k]);
  }
  p.part_elems = pe;
  p.part = take(pe * sizeof(double));
  p.total = off;
  return ST_OK;
}

template <class TI, class TO>
__global__ void transpose_kernel(const TI *u, int64_t n, int64_t r, TO *ut) {
  // ut[m * r + j] = u[m + n * j]
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * r) return;
  const int64_t m = idx / r, j = idx - m * r;
  ut[idx] = (TO)u[m + n * j];
}

// Partial sums of out[i + n*j] = sum_f Y[f][i] B[f][j] over this block's fibre
// tiles. Fibre f = lo + a*hi of Y starts at lo + a*n*hi, of B at lo + a*r*hi;
// both have element stride a.
__global__ __launch_bounds__(256) void cross_kernel(const float *Y, const float *B, int64_t a,
                                                    int64_t n, int64_t r, int64_t F,
                                                    double *part) {
  extern __shared__ float sm[];
  float *ys = sm;                      // [FT][n]
  float *bs = sm + kCrossFT * n;       // [FT][r]
  const int tid = threadIdx.x;
  const int64_t nr = n * r;
  const int64_t o0 = (int64_t)blockIdx.y * 256 * kCrossOPT;
  double acc[kCrossOPT];
#pragma unroll
  for (int q = 0; q < kCrossOPT; ++q) acc[q] = 0.0;
  const int64_t tiles = (F + kCrossFT - 1) / kCrossFT;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    __syncthreads();
    for (int64_t idx = tid; idx < kCrossFT * n; idx += 256) {
      const int f = (int)(idx % kCrossFT);
      const int64_t i = idx / kCrossFT, fib = t * kCrossFT + f;
      float v = 0.0f;
      if (fib < F) {
        const int64_t hi = fib / a, lo = fib - hi * a;
        v = Y[lo + a * n * hi + a * i];
      }
      ys[f * n + i] = v;
    }
    for (int64_t idx = tid; idx < kCrossFT * r; idx += 256) {
      const int f = (int)(idx % kCrossFT);
      const int64_t j = idx / kCrossFT, fib = t * kCrossFT + f;
      float v = 0.0f;
      if (fib < F) {
        const int64_t hi = fib / a, lo = fib - hi * a;
        v = B[lo + a * r * hi + a * j];
      }
      bs[f * r + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCrossOPT; ++q) {
      const int64_t o = o0 + tid + 256 * q;
      if (o < nr) {
        const int64_t j = o / n, i = o - j * n;
        double s = 0.0;
#pragma unroll
        for (int f = 0; f < kCrossFT; ++f) s += (double)ys[f * n + i] * (double)bs[f * r + j];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kCrossOPT; ++q) {
    const int64_t o = o0 + tid + 256 * q;
    if (o < nr) part[(size_t)blockIdx.x * nr + o] = acc[q];
  }
}

// The same contraction on the matrix cores, in the precision of the call: a
// block stages kCrossMFT fibres of Y and B in LDS (zero past n, r and F) and
// each wave accumulates TPW output tiles of 16 x 16 (the MFMA K dimension runs
// over the fibres). FP32 products and sums (16x16x4 f32) or split-bf16 products
// hi*hi + hi*lo + lo*hi (16x16x32 bf16) within one staged tile, whose sums are
// then added in FP64; FP64 products and sums of the FP32 data (16x16x4 f64).
// Partials per fibre block in FP64 like cross_kernel.
constexpr int kCrossMFT = 32;
constexpr int kCrossTPW = 4;  // output tiles per wave

int cross_mfma_blocks_x(int64_t F) {
  const int64_t t = (F + kCrossMFT - 1) / kCrossMFT;
  return (int)std::max<int64_t>(1, std::min<int64_t>(t, kCrossMaxBlocks));
}

size_t cross_mfma_lds(int64_t n, int64_t r) {
  return (size_t)kCrossMFT * (16 * ((n + 15) / 16) + 16 * ((r + 15) / 16)) * sizeof(float);
}

template <int P>  // 0 FP32, 1 split bf16, 2 FP64
__global__ __launch_bounds__(256) void cross_mfma_kernel(const float *Y, const float *B,
                                                         int64_t a, int64_t n, int64_t r,
                                                         int64_t F, double *part) {
  extern __shared__ float sm[];
  const int np = 16 * (int)((n + 15) / 16), rp = 16 * (int)((r + 15) / 16);
  float *ys = sm;                   // [kCrossMFT][np]
  float *bs = sm + kCrossMFT * np;  // [kCrossMFT][rp]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int tn = np / 16, ntiles = tn * (rp / 16);
  const int tile0 = (int)blockIdx.y * 4 * kCrossTPW + wid * kCrossTPW;
  double acc[kCrossTPW][4];
#pragma unroll
  for (int t = 0; t < kCrossTPW; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = 0.0;
  const int64_t ftiles = (F + kCrossMFT - 1) / kCrossMFT;
  for (int64_t ft = blockIdx.x; ft < ftiles; ft += gridDim.x) {
    __syncthreads();
    for (int idx = tid; idx < kCrossMFT * np; idx += 256) {
      const int f = idx % kCrossMFT, i = idx / kCrossMFT;
      const int64_t fib = ft * kCrossMFT + f;
      float v = 0.0f;
      if (fib < F && i < n) {
        const int64_t hi = fib / a, lo = fib - hi * a;
        v = Y[lo + a * n * hi + a * i];
      }
      ys[f * np + i] = v;
    }
    for (int idx = tid; idx < kCrossMFT * rp; idx += 256) {
      const int f = idx % kCrossMFT, j = idx / kCrossMFT;
      const int64_t fib = ft * kCrossMFT + f;
      float v = 0.0f;
      if (fib < F && j < r) {
        const int64_t hi = fib / a, lo = fib - hi * a;
        v = B[lo + a * r * hi + a * j];
      }
      bs[f * rp + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kCrossTPW; ++t) {
      const int tile = tile0 + t;
      if (tile >= ntiles) break;  // uniform per wave
      const int i = 16 * (tile % tn) + col, j = 16 * (tile / tn) + col;
      if constexpr (P == 2) {
        f64x4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < kCrossMFT / 4; ++st) {
          const int f = 4 * st + grp;
          c = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ys[f * np + i], (double)bs[f * rp + j],
                                                   c, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] += c[v];
      } else if constexpr (P == 0) {
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int st = 0; st < kCrossMFT / 4; ++st) {
          const int f = 4 * st + grp;
          c = __builtin_amdgcn_mfma_f32_16x16x4f32(ys[f * np + i], bs[f * rp + j], c, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] += (double)c[v];
      } else {
        bf16x8 ah, al, bh, bl;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int f = 8 * grp + q;
          const float x = ys[f * np + i], y = bs[f * rp + j];
          const __bf16 xh = (__bf16)x, yh = (__bf16)y;
          ah[q] = xh;
          al[q] = (__bf16)(x - (float)xh);
          bh[q] = yh;
          bl[q] = (__bf16)(y - (float)yh);
        }
        f32x4 c = {0.0f, 0.0f, 0.0f, 0.0f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] += (double)c[v];
      }
    }
  }
  // accumulator element v of lane (grp, col): row grp + 4 v (FP64) or 4 grp + v,
  // column col of the tile
  const int64_t nr = n * r;
#pragma unroll
  for (int t = 0; t < kCrossTPW; ++t) {
    const int tile = tile0 + t;
    if (tile >= ntiles) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = 16 * (tile % tn) + (P == 2 ? grp + 4 * v : 4 * grp + v);
      const int64_t j = 16 * (tile / tn) + col;
      if (i < n && j < r) part[(size_t)blockIdx.x * nr + i + n * j] = acc[t][v];
    }
  }
}

__global__ void cross_reduce_kernel(const double *part, int nb, int64_t nr, float *out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nr) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * nr + o];
  out[o] = (float)s;
}

struct Run {
  const Plan &p;
  char *ws;
  const float *const *U;
  hipStream_t s;

  template <class T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  float *buf(int i) const { return at<float>(p.buf[i]); }

  // W for x_k U_k^T: rows r_k of U^T (U column-major is U^T row-major)
  FiberW proj(int k) const {
    FiberW w{};
    w.w = U[k];
    w.ldw = p.n[k];
    if (p.prec == Prec::FP64) w.w64 = at<double>(p.u64[k]);
    if (p.prec == Prec::BF16X3) {
      w.w_hi = at<__bf16>(p.ph[k]);
      w.w_lo = at<__bf16>(p.pl[k]);
      w.ldw_bf = p.ldb_p[k];
    }
    return w;
  }
  // W for x_k U_k: rows n_k of U (row-major copy)
  FiberW expand(int k) const {
    FiberW w{};
    w.w = at<float>(p.ut[k]);
    w.ldw = p.r[k];
    if (p.prec == Prec::FP64) w.w64 = at<double>(p.ut64[k]);
    if (p.prec == Prec::BF16X3) {
      w.w_hi = at<__bf16>(p.eh[k]);
      w.w_lo = at<__bf16>(p.el[k]);
      w.ldw_bf = p.ldb_e[k];
    }
    return w;
  }

  hipError_t prepare() const {
    hipError_t e = hipSuccess;
    for (int k = 0; k < p.d && e == hipSuccess; ++k) {
      const int64_t n = p.n[k], r = p.r[k], nr = n * r;
      const unsigned g = (unsigned)((nr + 255) / 256);
      hipLaunchKernelGGL((transpose_kernel<float, float>), dim3(g), dim3(256), 0, s, U[k], n, r,
                         at<float>(p.ut[k]));
      e = hipGetLastError();
      if (e == hipSuccess && p.prec == Prec::FP64) {
        e = launch_f32_to_f64(U[k], nr, at<double>(p.u64[k]), s);
        if (e == hipSuccess) {
          hipLaunchKernelGGL((transpose_kernel<float, double>), dim3(g), dim3(256), 0, s, U[k],
                             n, r, at<double>(p.ut64[k]));
          e = hipGetLastError();
        }
      }
      if (e == hipSuccess && p.prec == Prec::BF16X3) {
        e = launch_split_rows(U[k], r, n, n, at<__bf16>(p.ph[k]), at<__bf16>(p.pl[k]),
                              p.ldb_p[k], s);
        if (e == hipSuccess)
          e = launch_split_rows(at<float>(p.ut[k]), n, r, r, at<__bf16>(p.eh[k]),
                                at<__bf16>(p.el[k]), p.ldb_e[k], s);
      }
    }
    return e;
  }

  // y = x x_k W^T for a tensor of shape `shape` (mode k: nin -> nout)
  hipError_t step(const float *x, const int64_t *shape, int k, int64_t nout, const FiberW &w,
                  float *y) const {
    FiberIn in{};
    in.x = x;
    in.a = prod(shape, 0, k);
    in.n = shape[k];
    in.F = in.a * prod(shape, k + 1, p.d);
    return launch_fiber_project(in, w, 0, (int)nout, FiberOut{y, 0, in.a, nout}, nullptr, p.prec,
                                s);
  }

  // X^ = G x_1 U_1 ... x_d U_d (G shaped r, out shaped n)
  hipError_t reconstruct(const float *g, float *out) const {
    int64_t shape[ST_MAX_MODES];
    std::memcpy(shape, p.r, sizeof(shape));
    const float *cur = g;
    hipError_t e = hipSuccess;
    for (int k = 0; k < p.d && e == hipSuccess; ++k) {
      float *dst = (k == p.d - 1) ? out : buf(k & 1);
      e = step(cur, shape, k, p.n[k], expand(k), dst);
      shape[k] = p.n[k];
      cur = dst;
    }
    return e;
  }

  // Optional projection A x_1 U_1^T ... x_d U_d^T into gproj, and for every k
  // with gfac[k] set, gfac[k] = (A x_{j != k} U_j^T)_(k) B_(k)^T.
  hipError_t project_and_cross(const float *A, const float *B, float *gproj,
                               float *const *gfac) const {
    int64_t zs[ST_MAX_MODES];
    std::memcpy(zs, p.n, sizeof(zs));
    const float *Z = A;
    hipError_t e = hipSuccess;
    for (int k = 0; k < p.d && e == hipSuccess; ++k) {
      if (gfac && gfac[k]) {
        int64_t ys[ST_MAX_MODES];
        std::memcpy(ys, zs, sizeof(ys));
        const float *Y = Z;
        int sel = 0;
        for (int m = k + 1; m < p.d && e == hipSuccess; ++m) {
          float *dst = buf(2 + sel);
          e = step(Y, ys, m, p.r[m], proj(m), dst);
          ys[m] = p.r[m];
          Y = dst;
          sel ^= 1;
        }
        if (e != hipSuccess) break;
        e = cross(Y, B, k, gfac[k]);
      }
      bool need_next = gproj != nullptr;
      for (int j = k + 1; j < p.d; ++j) need_next = need_next || (gfac && gfac[j]);
      if (!need_next || e != hipSuccess) break;
      float *dst = (k == p.d - 1) ? gproj : buf(k & 1);
      e = step(Z, zs, k, p.r[k], proj(k), dst);
      zs[k] = p.r[k];
      Z = dst;
    }
    return e;
  }

  hipError_t cross(const float *Y, const float *B, int k, float *out) const {
    const int64_t a = prod(p.r, 0, k), n = p.n[k], r = p.r[k];
    const int64_t F = a * prod(p.r, k + 1, p.d);
    const int64_t nr = n * r;
    const size_t lm = cross_mfma_lds(n, r);
    if (lm <= 160 * 1024) {
      // matrix cores in the call's precision
      const int nbx = cross_mfma_blocks_x(F);
      const int64_t tiles = ((n + 15) / 16) * ((r + 15) / 16);
      const unsigned nby = (unsigned)((tiles + 4 * kCrossTPW - 1) / (4 * kCrossTPW));
      const void *fn = p.prec == Prec::FP64     ? (const void *)cross_mfma_kernel<2>
                       : p.prec == Prec::BF16X3 ? (const void *)cross_mfma_kernel<1>
                                                : (const void *)cross_mfma_kernel<0>;
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lm);
      if (e != hipSuccess) return e;
      double *part = at<double>(p.part);
      if (p.prec == Prec::FP64)
        hipLaunchKernelGGL(cross_mfma_kernel<2>, dim3((unsigned)nbx, nby), dim3(256), lm, s, Y, B,
                           a, n, r, F, part);
      else if (p.prec == Prec::BF16X3)
        hipLaunchKernelGGL(cross_mfma_kernel<1>, dim3((unsigned)nbx, nby), dim3(256), lm, s, Y, B,
                           a, n, r, F, part);
      else
        hipLaunchKernelGGL(cross_mfma_kernel<0>, dim3((unsigned)nbx, nby), dim3(256), lm, s, Y, B,
                           a, n, r, F, part);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(cross_reduce_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s,
                         part, nbx, nr, out);
      return hipGetLastError();
    }
    // very long modes (n + r above about 1280): FP64 products on the vector units
    const int nbx = cross_blocks_x(F);
    const unsigned nby = (unsigned)((nr + 256 * kCrossOPT - 1) / (256 * kCrossOPT));
    const size_t lds = (size_t)kCrossFT * (n + r) * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)cross_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    double *part = at<double>(p.part);
    hipLaunchKernelGGL(cross_kernel, dim3((unsigned)nbx, nby), dim3(256), lds, s, Y, B, a, n, r,
                       F, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cross_reduce_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s,
                       part, nbx, nr, out);
    return hipGetLastError();
  }
};

int fail_with(int code, const char *what) {
  set_stateless_error(what);
  return code;
}

int status_of(hipError_t e, const char *call, const char *step) {
  if (e == hipSuccess) return ST_OK;
  std::string m = std::string(call) + ": " + step + ": " + hipGetErrorString(e);
  set_stateless_error(m.c_str());
  return e == hipErrorOutOfMemory ? ST_ENOMEM : ST_EHIP;
}

bool factors_ok(int d, const float *const *factors) {
  if (!factors) return false;
  for (int k = 0; k < d; ++k)
    if (!factors[k]) return false;
  return true;
}

}  // namespace

extern "C" {

int st_tucker_workspace(int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                        int32_t precision, int64_t *bytes) {
  if (!bytes) return ST_EINVAL;
  Plan p;
  const int rc = make_plan(nmodes, dims, ranks, precision, p);
  if (rc != ST_OK) return fail_with(rc, "st_tucker_workspace: invalid shapes or precision");
  *bytes = (int64_t)p.total;
  return ST_OK;
}

int st_tucker_fwd(int32_t op, int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                  const float *in, const float *const *factors, float *out, int32_t precision,
                  void *work, int64_t work_bytes, void *stream) {
  Plan p;
  int rc = make_plan(nmodes, dims, ranks, precision, p);
  if (rc != ST_OK) return fail_with(rc, "st_tucker_fwd: invalid shapes or precision");
  if ((op != ST_RECONSTRUCT && op != ST_PROJECT) || !in || !out || !work ||
      !factors_ok(p.d, factors))
    return fail_with(ST_EINVAL, "st_tucker_fwd: bad op or null pointer");
  if (work_bytes < (int64_t)p.total) return fail_with(ST_ESMALL, "st_tucker_fwd: workspace");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);  // also initialises the runtime before any launch
  if (e != hipSuccess) return status_of(e, "st_tucker_fwd", "device");
  Run run{p, static_cast<char *>(work), factors, (hipStream_t)stream};
  e = run.prepare();
  if (e != hipSuccess) return status_of(e, "st_tucker_fwd", "factor copies");
  e = (op == ST_RECONSTRUCT) ? run.reconstruct(in, out)
                             : run.project_and_cross(in, nullptr, out, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  return status_of(e, "st_tucker_fwd", op == ST_RECONSTRUCT ? "reconstruct" : "project");
}

int st_tucker_bwd(int32_t op, int32_t nmodes, const int64_t *dims, const int64_t *ranks,
                  const float *in, const float *const *factors, const float *gout, float *gin,
                  float *const *gfactors, int32_t precision, void *work, int64_t work_bytes,
                  void *stream) {
  Plan p;
  int rc = make_plan(nmodes, dims, ranks, precision, p);
  if (rc != ST_OK) return fail_with(rc, "st_tucker_bwd: invalid shapes or precision");
  if ((op != ST_RECONSTRUCT && op != ST_PROJECT) || !in || !gout || !work ||
      !factors_ok(p.d, factors))
    return fail_with(ST_EINVAL, "st_tucker_bwd: bad op or null pointer");
  if (work_bytes < (int64_t)p.total) return fail_with(ST_ESMALL, "st_tucker_bwd: workspace");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return status_of(e, "st_tucker_bwd", "device");
  Run run{p, static_cast<char *>(work), factors, (hipStream_t)stream};
  e = run.prepare();
  if (e != hipSuccess) return status_of(e, "st_tucker_bwd", "factor copies");
  if (op == ST_RECONSTRUCT) {
    // dG = R x_k U_k^T (all k); dU_k from the partial chains of R against G
    e = run.project_and_cross(gout, in, gin, gfactors);
  } else {
    // dU_k from the partial chains of X against Gb, then dX = Gb x_k U_k (all k)
    e = run.project_and_cross(in, gout, nullptr, gfactors);
    if (e == hipSuccess && gin) e = run.reconstruct(gout, gin);
  }
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  return status_of(e, "st_tucker_bwd", op == ST_RECONSTRUCT ? "reconstruct vjp" : "project vjp");
}

}  // extern "C"
