// Streaming-mode kernels (Alg. 3 and the core update of Alg. 5) plus small
// FP64 helpers for the non-streaming factor growth (Alg. 4 with Alg. 1).
#include "common.hpp"
#include "kernels.hpp"
#include "secular.hpp"

namespace st {

// ---------------------------------------------------------------------------
// Gram-Schmidt passes over V (Alg. 3, first lines, done twice).
//
// V is the old auxiliary matrix (FP64; rows at the old ranks, leading
// dimension ldv, r columns); d is the FP64 slice projection at the new ranks;
// rows are mapped new -> old (padded rows of V are zero). Each block stages
// tiles of TR rows x r columns of V in LDS with coalesced (vector when
// possible) loads, then
//   PASS 1: colpart += V^T d
//   PASS 2: e1 = d - V p1 (FP64 row dots), q2part += ||e1||^2, colpart += V^T e1
// so V is read from HBM once per pass. The second correction p2 = V^T e1 and
// q^2 = ||e1||^2 - ||p2||^2 complete the two-pass projection; the complement
// e = d - V (p1 + p2) itself is formed inside the V rotation.
// ---------------------------------------------------------------------------
template <int PASS, int TR>
__global__ __launch_bounds__(256) void isvd_pass_kernel(IsvdArgs a) {
  extern __shared__ double sh[];
  constexpr int LDT = TR + 1;
  const int r = a.r;
  const int tid = threadIdx.x;
  double *p1s = sh;                   // [r]
  double *ev = p1s + r;               // [TR]
  double *rowred = ev + TR;           // [256 / TR][TR]
  int64_t *orow = reinterpret_cast<int64_t *>(rowred + 256);  // [TR]
  double *tile = reinterpret_cast<double *>(orow + TR);          // [r][LDT]
  if (PASS == 2)
    for (int j = tid; j < r; j += blockDim.x) p1s[j] = a.p1[j];

  constexpr int kMaxCols = 8;  // r <= 2048
  double colacc[kMaxCols];
#pragma unroll
  for (int q = 0; q < kMaxCols; ++q) colacc[q] = 0.0;
  double q2 = 0.0;
  const bool vec = a.map.identity && (a.ldv & 1) == 0;

  // Full tiles of an identity-mapped V with even ld are read as double2:
  // thread t takes rows 2 (t % (TR/2)) .. +1 of columns t / (TR/2) + (512/TR) it.
  // When every thread's columns fit KP registers, the next tile of the block is
  // loaded into registers while the current one is processed.
  constexpr int TPC = TR / 2, CPI = 256 / TPC, KP = 18;
  const int rq = (tid % TPC) * 2, jq = tid / TPC;
  const bool pre_ok = vec && (r + CPI - 1) / CPI <= KP;
  double2 pre[KP];
  auto prefetch = [&](int64_t row0) {
#pragma unroll
    for (int it = 0; it < KP; ++it) {
      const int j = jq + CPI * it;
      if (j < r) pre[it] = *reinterpret_cast<const double2 *>(a.V + row0 + rq + a.ldv * (int64_t)j);
    }
  };
  const int64_t ntiles = (a.R + TR - 1) / TR;
  bool have_pre = pre_ok && (int64_t)blockIdx.x * TR + TR <= a.R;
  if (have_pre) prefetch((int64_t)blockIdx.x * TR);
  for (int64_t tile_i = blockIdx.x; tile_i < ntiles; tile_i += gridDim.x) {
    const int64_t row0 = tile_i * TR;
    __syncthreads();
    if (have_pre) {
#pragma unroll
      for (int it = 0; it < KP; ++it) {
        const int j = jq + CPI * it;
        if (j < r) {
          double *t = tile + j * LDT + rq;
          t[0] = pre[it].x;
          t[1] = pre[it].y;
        }
      }
      const int64_t nrow0 = (tile_i + gridDim.x) * TR;
      have_pre = nrow0 + TR <= a.R;
      if (have_pre) prefetch(nrow0);
    } else if (vec && row0 + TR <= a.R) {
      for (int j = jq; j < r; j += CPI) {
        const double2 v2 =
            *reinterpret_cast<const double2 *>(a.V + row0 + rq + a.ldv * (int64_t)j);
        double *t = tile + j * LDT + rq;
        t[0] = v2.x;
        t[1] = v2.y;
      }
    } else {
      if (tid < TR) {
        const int64_t row = row0 + tid;
        orow[tid] = row < a.R ? map_new_to_old(a.map, row) : -1;
      }
      __syncthreads();
      for (int idx = tid; idx < r * TR; idx += blockDim.x) {
        const int j = idx / TR, i = idx - j * TR;
        const int64_t o = orow[i];
        tile[j * LDT + i] = (o >= 0) ? a.V[o + a.ldv * (int64_t)j] : 0.0;
      }
    }
    __syncthreads();
    // row phase
    if (PASS == 1) {
      if (tid < TR) {
        const int64_t row = row0 + tid;
        ev[tid] = row < a.R ? a.d[row] : 0.0;
      }
    } else {
      // TR == 64: 4 partial dots per row; TR == 32: 8
      constexpr int SUB = 256 / TR;
      const int i = tid % TR, sub = tid / TR;
      double s1 = 0.0;
      for (int j = sub; j < r; j += SUB) s1 += tile[j * LDT + i] * p1s[j];
      rowred[sub * TR + i] = s1;
      __syncthreads();
      if (tid < TR) {
        const int64_t row = row0 + tid;
        double e1 = 0.0;
        if (row < a.R) {
          double dot = 0.0;
          for (int q = 0; q < SUB; ++q) dot += rowred[q * TR + tid];
          e1 = a.d[row] - dot;
          if (a.e1out) a.e1out[row] = e1;
        }
        ev[tid] = e1;
        q2 += e1 * e1;
      }
    }
    __syncthreads();
    // column phase
#pragma unroll
    for (int q = 0; q < kMaxCols; ++q) {
      const int j = tid + q * blockDim.x;
      if (j < r) {
        double acc = 0.0;
        const double *tr = tile + j * LDT;
#pragma unroll 8
        for (int i = 0; i < TR; ++i) acc += tr[i] * ev[i];
        colacc[q] += acc;
      }
    }
  }
  // column-major partials: colpart[j * gridDim.x + block]
#pragma unroll
  for (int q = 0; q < kMaxCols; ++q) {
    const int j = tid + q * blockDim.x;
    if (j < r) a.colpart[(size_t)j * gridDim.x + blockIdx.x] = colacc[q];
  }
  if (PASS == 2) {
    __shared__ double red[16];
    const double t = block_sum(q2, red);
    if (tid == 0) a.q2part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------------------
// Second Gram-Schmidt pass with V held in registers (r <= 4 CPL): a block of
// four waves walks 64-row tiles; lane l of wave w loads row (tile * 64 + l) of
// the columns j = w + 4 c (coalesced 512-byte column segments, one load per
// column, all in flight together), forms its share of the row dot V(row,:) p1,
// the four shares meet in LDS (one barrier per tile, double-buffered), and every
// lane then has e1(row) = d(row) - V(row,:) p1 and adds V(row, j) e1(row) to its
// column accumulators. V goes through registers once, with no LDS staging of
// tiles; the column sums are reduced across lanes once per block at the end.
// Same outputs as isvd_pass_kernel<2, TR>.
// ---------------------------------------------------------------------------
template <int CPL>
__global__ __launch_bounds__(256) void isvd_pass2_reg_kernel(IsvdArgs a) {
  __shared__ double dots[2][4][64];
  __shared__ double p1s[4 * CPL];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = a.r;
  for (int j = threadIdx.x; j < 4 * CPL; j += blockDim.x) p1s[j] = j < r ? a.p1[j] : 0.0;
  __syncthreads();
  double cacc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) cacc[c] = 0.0;
  double q2 = 0.0;
  const int64_t ntiles = (a.R + 63) / 64;
  int buf = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * 64 + lane;
    const bool valid = row < a.R;
    const int64_t src = valid ? map_new_to_old(a.map, row) : -1;
    // Every load is unconditional (a select right after a load would make the
    // wave wait for it before issuing the next): a padded row reads row 0 and
    // columns past r re-read column r - 1; both are masked where consumed (the
    // row by zeroing its dot and e1, the columns by p1 = 0 and by never being
    // stored).
    double v[CPL];
    const double *pc = a.V + (src >= 0 ? src : 0) + a.ldv * (int64_t)(wid < r ? wid : r - 1);
    const int64_t step = 4 * a.ldv;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      v[c] = *pc;
      if (wid + 4 * (c + 1) < r) pc += step;
    }
    const double dv = a.d[valid ? row : 0];
    double dot = 0.0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) dot += v[c] * p1s[wid + 4 * c];
    dots[buf][wid][lane] = src >= 0 ? dot : 0.0;
    __syncthreads();
    const double e1 =
        valid ? dv - (((dots[buf][0][lane] + dots[buf][1][lane]) + dots[buf][2][lane]) +
                      dots[buf][3][lane])
              : 0.0;
    const double e1m = src >= 0 ? e1 : 0.0;
    if (wid == 0) {
      if (valid && a.e1out) a.e1out[row] = e1;
      q2 += e1 * e1;
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) cacc[c] += v[c] * e1m;
    buf ^= 1;
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int j = wid + 4 * c;
    const double t = wave_sum(cacc[c]);
    if (lane == 0 && j < r) a.colpart[(size_t)j * gridDim.x + blockIdx.x] = t;
  }
  if (wid == 0) {
    const double t = wave_sum(q2);
    if (lane == 0) a.q2part[blockIdx.x] = t;
  }
}

// dst[oa + i] = a[i] (i < na), dst[ob + i] = b[i] (i < nb), dst[oc + i] = c[i]
// (i < nc): one launch that publishes small results, typically into pinned
// host memory mapped for the device (no copy engine or blit per array).
__global__ void gather3_kernel(double *dst, const double *a, int na, int oa, const double *b,
                               int nb, int ob, const double *c, int nc, int oc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) dst[oa + i] = a[i];
  else if (i < na + nb) dst[ob + i - na] = b[i - na];
  else if (i < na + nb + nc) dst[oc + i - na - nb] = c[i - na - nb];
}

hipError_t launch_gather3(double *dst, const double *a, int na, int oa, const double *b, int nb,
                          int ob, const double *c, int nc, int oc, hipStream_t s) {
  const int n = na + nb + nc;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, a,
                     na, oa, b, nb, ob, c, nc, oc);
  return hipGetLastError();
}

// One block per column: out[j] = sum_b part[j * nb + b] (fixed tree order);
// optionally out2[j] = out[j] + add[j]; block r (if q2part) sums q2part.
__global__ __launch_bounds__(256) void colsum_kernel(const double *part, int nb, int r,
                                                     double *out, const double *add, double *out2,
                                                     const double *q2part, double *q2) {
  __shared__ double red[16];
  const int j = blockIdx.x;
  const double *src = (j < r) ? part + (size_t)j * nb : q2part;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += src[b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    if (j < r) {
      out[j] = s;
      if (out2) out2[j] = s + add[j];
    } else {
      q2[0] = s;
    }
  }
}

// Grid of the second pass: the register-resident kernel (r <= 192) keeps its
// column sums per block until the end, so larger r takes fewer, longer-lived
// blocks (measured at R = 948480: r = 166 runs 241 us with 512 blocks against
// 258 us with 2048; r = 40 prefers 2048).
int isvd_blocks(int64_t R, int r) {
  const int64_t t = (R + 63) / 64;
  const int64_t cap = (r <= 32 || r > 192) ? 2048 : (r <= 64 ? 1024 : 512);
  return (int)(t < cap ? (t > 0 ? t : 1) : cap);
}

// rowred holds 256 doubles for either tile height
static size_t isvd_lds(int r, int tr) {
  return sizeof(double) * ((size_t)r + tr + 256) + sizeof(int64_t) * tr +
         sizeof(double) * (size_t)r * (tr + 1);
}

static constexpr size_t kIsvdMaxLds = 160 * 1024;

template <int PASS, int TR>
static hipError_t launch_isvd_tr(const IsvdArgs &a, int nblocks, hipStream_t s) {
  const size_t lds = isvd_lds(a.r, TR);
  const void *fn = (const void *)isvd_pass_kernel<PASS, TR>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((isvd_pass_kernel<PASS, TR>), dim3(nblocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_isvd_pass(int pass, IsvdArgs a, int nblocks, hipStream_t s) {
  if (a.r > 8 * 256 || pass < 1 || pass > 2) return hipErrorInvalidValue;
  if (pass == 2 && a.r >= 1 && a.r <= 4 * 48) {
    const dim3 g((unsigned)nblocks), b(256);
    if (a.r <= 4 * 8) hipLaunchKernelGGL(isvd_pass2_reg_kernel<8>, g, b, 0, s, a);
    else if (a.r <= 4 * 16) hipLaunchKernelGGL(isvd_pass2_reg_kernel<16>, g, b, 0, s, a);
    else if (a.r <= 4 * 32) hipLaunchKernelGGL(isvd_pass2_reg_kernel<32>, g, b, 0, s, a);
    else hipLaunchKernelGGL(isvd_pass2_reg_kernel<48>, g, b, 0, s, a);
    return hipGetLastError();
  }
  // 64-row tiles while two blocks fit a CU's LDS, else 32-row tiles (one block
  // per CU leaves the tile load and the two compute phases unoverlapped)
  const bool tall = 2 * isvd_lds(a.r, 64) <= kIsvdMaxLds;
  if (!tall && isvd_lds(a.r, 32) > kIsvdMaxLds) return hipErrorInvalidValue;
  if (pass == 1)
    return tall ? launch_isvd_tr<1, 64>(a, nblocks, s) : launch_isvd_tr<1, 32>(a, nblocks, s);
  return tall ? launch_isvd_tr<2, 64>(a, nblocks, s) : launch_isvd_tr<2, 32>(a, nblocks, s);
}

hipError_t launch_colsum(const double *part, int nb, int r, double *out, const double *add,
                         double *out2, const double *q2part, double *q2, hipStream_t s) {
  const int blocks = r + (q2part ? 1 : 0);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_kernel, dim3(blocks), dim3(256), 0, s, part, nb, r, out, add, out2,
                     q2part, q2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Secular-equation SVD of S' (see secular.hpp).
// ---------------------------------------------------------------------------
struct WaveRed {
  int lane;
  // (the sums and products run with every lane of the wave active: DPP moves)
  template <class F>
  __device__ double sum(int m, F f) const {
    double acc = 0.0;
    for (int j = lane; j < m; j += kWave) acc += f(j);
    return dpp_wave_sum(acc);
  }
  template <class F>
  __device__ double prod(int m, F f) const {
    double acc = 1.0;
    for (int j = lane; j < m; j += kWave) acc *= f(j);
    return dpp_wave_prod(acc);
  }
  template <class F>
  __device__ void for_each(int m, F f) const {
    for (int j = lane; j < m; j += kWave) f(j);
  }
  __device__ void sync() const { __syncthreads(); }
  template <class F>
  __device__ void single(F f) const {
    if (lane == 0) f();
  }
};

// The preparation of sec_prep in parallel on one block: poles and weights,
// active flags, the (rare) rotations of poles closer than tol -- done by one
// thread exactly as sec_prep does, and only when some adjacent poles are that
// close -- and the ordered lists of active and deflated indices by ballot
// prefix sums. zz is summed in the block's fixed order.
__global__ __launch_bounds__(256) void sec_prep_kernel(SecData s, const double *S, const double *p,
                                                       double q, const double *qsq, int grow,
                                                       double tol) {
  __shared__ int close_pair;
  __shared__ int wcount[2][4];
  __shared__ double red[16];
  const int r = s.r, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // zhat is scattered by sec_zhat_kernel into a zeroed array (deflated entries
  // stay zero); clear it here rather than in a launch of its own
  for (int t = tid; t < s.n; t += blockDim.x) s.zh[t] = 0.0;
  for (int t = tid; t <= r; t += blockDim.x) {
    if (t == 0) {
      s.d[0] = 0.0;
      s.z[0] = grow ? (qsq ? sqrt(qsq[0]) : q) : 0.0;
      s.active[0] = grow ? 1 : 0;
    } else {
      const double z = p[r - t];
      s.d[t] = S[r - t];
      s.z[t] = z;
      s.active[t] = fabs(z) > tol ? 1 : 0;
    }
  }
  if (tid == 0) close_pair = 0;
  __syncthreads();
  for (int t = 2 + tid; t <= r; t += blockDim.x)
    if (s.d[t] - s.d[t - 1] <= tol) close_pair = 1;
  __syncthreads();
  if (tid == 0) {
    int nrot = 0;
    if (close_pair) {
      int prev = -1;
      for (int t = 1; t <= r; ++t) {
        if (!s.active[t]) continue;
        if (prev >= 1 && s.d[t] - s.d[prev] <= tol) {
          const double za = s.z[prev], zb = s.z[t];
          const double rho = hypot(za, zb);
          s.z[t] = rho;
          s.z[prev] = 0.0;
          s.active[prev] = 0;
          s.rot_t[2 * nrot] = prev;
          s.rot_t[2 * nrot + 1] = t;
          s.rot_cs[2 * nrot] = zb / rho;
          s.rot_cs[2 * nrot + 1] = za / rho;
          ++nrot;
        }
        prev = t;
      }
    }
    s.counts[2] = nrot;
  }
  __syncthreads();
  int mK = 0, mD = 0;
  double zz = 0.0;
  for (int base = 0; base <= r; base += blockDim.x) {
    const int t = base + tid;
    const int act = (t <= r) ? s.active[t] : 0;
    const int dfl = (t >= 1 && t <= r && !act) ? 1 : 0;
    if (act) zz += s.z[t] * s.z[t];
    const unsigned long long ma = __ballot(act), md = __ballot(dfl);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
      wcount[0][wid] = __popcll(ma);
      wcount[1][wid] = __popcll(md);
    }
    __syncthreads();
    int offK = mK, offD = mD;
    for (int w = 0; w < wid; ++w) {
      offK += wcount[0][w];
      offD += wcount[1][w];
    }
    if (act) s.K[offK + __popcll(ma & below)] = t;
    if (dfl) s.defl[offD + __popcll(md & below)] = t;
    for (int w = 0; w < 4; ++w) {
      mK += wcount[0][w];
      mD += wcount[1][w];
    }
    __syncthreads();
  }
  zz = block_sum(zz, red);
  if (tid == 0) {
    s.counts[0] = mK;
    s.counts[1] = mD;
    s.zz[0] = zz;
  }
}

__global__ __launch_bounds__(256) void sec_roots_kernel(SecData s) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= s.counts[0]) return;
  WaveRed red{(int)(threadIdx.x & 63)};
  int o;
  double mu;
  sec_root(s, i, red, &o, &mu);
  if ((threadIdx.x & 63) == 0) {
    s.org[i] = o;
    s.mu[i] = mu;
  }
}

__global__ __launch_bounds__(256) void sec_zhat_kernel(SecData s) {
  const int jt = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int m = s.counts[0];
  const int lane = threadIdx.x & 63;
  if (jt >= s.n) return;
  if (jt >= m) return;
  WaveRed red{lane};
  const double z = sec_zhat(s, jt, red);
  if (lane == 0) s.zh[s.K[jt]] = z;
}

// One wave (block of 64) per output triplet. U2 and V2 are (r+1) x ntrip,
// column-major with leading dimension r+1, in the original index order of S'.
__global__ __launch_bounds__(64) void sec_vec_kernel(SecData s, int ntrip, double *U2, double *V2,
                                                     double *Snew) {
  extern __shared__ double vs[];
  double *u = vs, *v = vs + s.n;
  const int trip = blockIdx.x;
  const int lane = threadIdx.x;
  WaveRed red{lane};
  double nu, nv;
  const double sigma = sec_vectors(s, trip, u, v, red, &nu, &nv);
  const int col = sec_rank(s, trip, ntrip, red);
  const int r = s.r, ld = r + 1;
  const double iu = nu > 0.0 ? 1.0 / nu : 0.0, iv = nv > 0.0 ? 1.0 / nv : 0.0;
  for (int t = lane; t < s.n; t += kWave) {
    const int orig = (t == 0) ? r : r - t;
    U2[orig + (size_t)ld * col] = u[t] * iu;
    V2[orig + (size_t)ld * col] = v[t] * iv;
  }
  if (lane == 0) Snew[col] = sigma;
}

hipError_t launch_secular_svd(SecData s, const double *S, const double *p, double q,
                              const double *qsq, int grow, double tol, int ntrip, double *U2,
                              double *V2, double *Snew, hipStream_t st) {
  const int n = s.n;
  hipLaunchKernelGGL(sec_prep_kernel, dim3(1), dim3(256), 0, st, s, S, p, q, qsq, grow, tol);
  hipLaunchKernelGGL(sec_roots_kernel, dim3((n + 3) / 4), dim3(256), 0, st, s);
  hipLaunchKernelGGL(sec_zhat_kernel, dim3((n + 3) / 4), dim3(256), 0, st, s);
  const size_t lds = 2 * (size_t)n * sizeof(double);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(
        (const void *)sec_vec_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(sec_vec_kernel, dim3(ntrip), dim3(64), lds, st, s, ntrip, U2, V2, Snew);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// U~_d = [U_d U''(0:r, :); U''(r, :)] (Alg. 3, left factor without forming U').
// ---------------------------------------------------------------------------
__global__ void ud_update_kernel(const double *Ud, int64_t ldo, int64_t nd, int r, const double *U2,
                                 int c, double *Un, int64_t ldn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (nd + 1) * c;
  if (idx >= total) return;
  const int64_t row = idx % (nd + 1);
  const int col = (int)(idx / (nd + 1));
  const double *u2c = U2 + (size_t)(r + 1) * col;
  double s;
  if (row < nd) {
    s = 0.0;
#pragma unroll 8
    for (int k = 0; k < r; ++k) s += Ud[row + ldo * k] * u2c[k];
  } else {
    s = u2c[r];
  }
  Un[row + ldn * col] = s;
}

hipError_t launch_ud_update(const double *Ud, int64_t ldo, int64_t nd, int r, const double *U2,
                            int c, double *Un, int64_t ldn, hipStream_t s) {
  const int64_t total = (nd + 1) * c;
  hipLaunchKernelGGL(ud_update_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Ud,
                     ldo, nd, r, U2, c, Un, ldn);
  return hipGetLastError();
}

// Row-major FP32 rotation matrices for the mode-d TTMs of V and C:
//   Wv[m][k] = V''[k][m] (k < kv), with row r scaled by 1/q when e is kept;
//   Wc[m][k] = U''[k][m] (k <= r).
__global__ void build_rot_w_kernel(const double *U2, const double *V2, int r, int c, int kv,
                                   double inv_q, double *Wv, int64_t ldv, float *Wc,
                                   int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)c * (r + 1);
  if (idx >= total) return;
  const int m = (int)(idx / (r + 1)), k = (int)(idx % (r + 1));
  const size_t src = (size_t)k + (size_t)(r + 1) * m;
  Wc[m * ldc + k] = (float)U2[src];
  if (k < kv) Wv[m * ldv + k] = (k == r) ? V2[src] * inv_q : V2[src];
}

hipError_t launch_build_rot_w(const double *U2, const double *V2, int r, int c, int kv,
                              double inv_q, double *Wv, int64_t ldv, float *Wc, int64_t ldc,
                              hipStream_t s) {
  const int64_t total = (int64_t)c * (r + 1);
  hipLaunchKernelGGL(build_rot_w_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     U2, V2, r, c, kv, inv_q, Wv, ldv, Wc, ldc);
  return hipGetLastError();
}

// Init: C^T = A U_d and V = A U_d S^-1 with A the (R x n_init) FP64 mode-d
// unfolding of the last partial core, accumulated in FP64. With FP32 products
// the columns of small singular value would carry a relative error of about
// u s_1 / s_k and V would not be orthonormal to the accuracy the ISVD residual
// test needs.
// Block (x, m) covers rows 64 x .. 64 x + 63 of column m; its four waves take
// every fourth slice j and their partial sums are added in a fixed order, so a
// long initial batch (large nd) does not run as one serial loop per row.
__global__ __launch_bounds__(256) void init_vc_kernel(const double *A, int64_t R, int64_t nd,
                                                      const double *Ud, int64_t ldu, int rd,
                                                      const double *S, double *V, float *Cc) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 64 + lane;
  const int m = blockIdx.y;
  double acc = 0.0;
  if (row < R)
    for (int64_t j = w; j < nd; j += 4) acc += A[row + R * j] * Ud[j + ldu * m];
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && row < R) {
    const double t = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    if (Cc) Cc[row + R * m] = (float)t;
    V[row + R * m] = t / S[m];
  }
}

hipError_t launch_init_vc(const double *A, int64_t R, int64_t nd, const double *Ud,
                          int64_t ldu, int rd, const double *S, double *V, float *Cc,
                          hipStream_t s) {
  if (R <= 0 || rd <= 0) return hipSuccess;
  if (rd > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(init_vc_kernel, dim3((unsigned)((R + 63) / 64), (unsigned)rd), dim3(256), 0,
                     s, A, R, nd, Ud, ldu, rd, S, V, Cc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Factor growth helpers (FP64).
// ---------------------------------------------------------------------------
// W[:, c] = Q[:, n-1-c] for c < k (eigenvectors in descending eigenvalue order).
__global__ void take_top_kernel(const double *Q, int64_t n, int k, double *W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int c = (int)(idx / n);
  const int64_t i = idx % n;
  W[i + n * c] = Q[i + n * (n - 1 - c)];
}

// coef[j + r*c] = U(:,j)^T W(:,c)
__global__ void proj_coef_kernel(const double *U, int64_t n, int r, const double *W, int k,
                                 double *coef) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r * k) return;
  const int j = idx % r, c = idx / r;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += U[i + n * j] * W[i + n * c];
  coef[idx] = s;
}

// W(i, c) -= sum_j U(i, j) coef[j + r*c]
__global__ void proj_sub_kernel(const double *U, int64_t n, int r, double *W, int k,
                                const double *coef) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx % n;
  const int c = (int)(idx / n);
  double s = 0.0;
  for (int j = 0; j < r; ++j) s += U[i + n * j] * coef[j + r * c];
  W[i + n * c] -= s;
}

// Modified Gram-Schmidt among the k columns of W, then normalisation.
__global__ void mgs_kernel(double *W, int64_t n, int k) {
  __shared__ double red[16];
  for (int c = 0; c < k; ++c) {
    double *wc = W + n * c;
    for (int p = 0; p < c; ++p) {
      const double *wp = W + n * p;
      double s = 0.0;
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += wp[i] * wc[i];
      s = block_sum(s, red);
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) wc[i] -= s * wp[i];
      __syncthreads();
    }
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += wc[i] * wc[i];
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) wc[i] *= inv;
    __syncthreads();
  }
}

hipError_t launch_new_columns(const double *Q, int64_t n, const double *U, int r, int k,
                              double *W, double *coef, hipStream_t s) {
  const int64_t nk = n * k;
  hipLaunchKernelGGL(take_top_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, Q, n, k,
                     W);
  if (r > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(proj_coef_kernel, dim3((r * k + 255) / 256), dim3(256), 0, s, U, n, r, W,
                         k, coef);
      hipLaunchKernelGGL(proj_sub_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, U,
                         n, r, W, k, coef);
    }
  }
  hipLaunchKernelGGL(mgs_kernel, dim3(1), dim3(256), 0, s, W, n, k);
  return hipGetLastError();
}

// Write columns [c0, c0 + k) of U_k from W (n x k, FP64) into the FP64 master
// (col-major, ld n), the FP32 copy Uf (col-major = row-major U^T, ld n), the
// row-major FP32 Ut (ld n) and the bf16 splits of Uf (row-major U^T, ld ldb).
__global__ void append_cols_kernel(const double *W, int64_t n, int c0, int k, double *U64,
                                   float *Uf, float *Ut, __bf16 *Uh, __bf16 *Ul, int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * k) return;
  const int64_t i = idx % n;
  const int c = (int)(idx / n);
  const double w = W[i + n * c];
  const int64_t col = c0 + c;
  U64[i + n * col] = w;
  const float f = (float)w;
  Uf[i + n * col] = f;
  Ut[i * n + col] = f;
  const __bf16 h = (__bf16)f;
  Uh[col * ldb + i] = h;
  Ul[col * ldb + i] = (__bf16)(f - (float)h);
}

hipError_t launch_append_cols(const double *W, int64_t n, int c0, int k, double *U64, float *Uf,
                              float *Ut, __bf16 *Uh, __bf16 *Ul, int64_t ldb, hipStream_t s) {
  const int64_t nk = n * k;
  hipLaunchKernelGGL(append_cols_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s, W, n,
                     c0, k, U64, Uf, Ut, Uh, Ul, ldb);
  return hipGetLastError();
}

// Per-block FP64 sum of squares (pairs layout: {sum, 0}).
__global__ void sumsq_kernel(const float *x, int64_t count, double *partials) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s;
    partials[2 * blockIdx.x + 1] = 0.0;
  }
}

hipError_t launch_sumsq(const float *x, int64_t count, double *partials, int nblocks,
                        hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(nblocks), dim3(256), 0, s, x, count, partials);
  return hipGetLastError();
}

// FP64 -> FP32 row of U_d for slice reconstruction: w[m] = U_d[t + ld*m].
__global__ void ud_row_kernel(const double *Ud, int64_t ld, int64_t t, int rd, float *w) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < rd) w[m] = (float)Ud[t + ld * m];
}

hipError_t launch_ud_row(const double *Ud, int64_t ld, int64_t t, int rd, float *w,
                         hipStream_t s) {
  hipLaunchKernelGGL(ud_row_kernel, dim3((rd + 255) / 256), dim3(256), 0, s, Ud, ld, t, rd, w);
  return hipGetLastError();
}

// bf16 split of a row-major FP32 matrix: hi = bf16(w), lo = bf16(w - hi).
__global__ void split_rows_kernel(const float *w, int64_t rows, int64_t n, int64_t ldw,
                                  __bf16 *hi, __bf16 *lo, int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ldb) return;
  const int64_t i = idx / ldb, j = idx % ldb;
  const float f = j < n ? w[i * ldw + j] : 0.0f;
  const __bf16 h = (__bf16)f;
  hi[idx] = h;
  lo[idx] = (__bf16)(f - (float)h);
}

hipError_t launch_split_rows(const float *w, int64_t rows, int64_t n, int64_t ldw, __bf16 *hi,
                             __bf16 *lo, int64_t ldb, hipStream_t s) {
  const int64_t total = rows * ldb;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w,
                     rows, n, ldw, hi, lo, ldb);
  return hipGetLastError();
}

__global__ void f32_to_f64_kernel(const float *x, int64_t n, double *y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

hipError_t launch_f32_to_f64(const float *x, int64_t n, double *y, hipStream_t s) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Factored streaming mode: V = V0 M with V0 (R x r) only ever appended to and
// the small orthogonal M (r x r) rotated (Sec. 3.2's auxiliary V kept as a
// product; the core is C = V x_d S).
// ---------------------------------------------------------------------------
// y = M x or M^T x (M n x n), and y2 = y + add when y2 is set: one wave per
// output (its lanes stride the sum, then a DPP wave sum), four per block. y
// must not overlap x.
__global__ __launch_bounds__(256) void small_gemv_kernel(const double *M, int n, const double *x,
                                                         int trans, double *y, const double *add,
                                                         double *y2) {
  const int lane = threadIdx.x & 63, i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;  // (uniform per wave)
  double acc = 0.0;
  if (trans)
    for (int l = lane; l < n; l += 64) acc += M[l + (size_t)n * i] * x[l];
  else
    for (int l = lane; l < n; l += 64) acc += M[i + (size_t)n * l] * x[l];
  acc = dpp_wave_sum(acc);
  if (lane == 0) {
    y[i] = acc;
    if (y2) y2[i] = acc + add[i];
  }
}

hipError_t launch_small_gemv(const double *M, int n, const double *x, int trans, double *y,
                             const double *add, double *y2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(small_gemv_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, M, n, x,
                     trans, y, add, y2);
  return hipGetLastError();
}

__global__ void vcol_kernel(const double *V0, int64_t R, int r, const double *w,
                            const double *base, double scale, double *out64, float *out32) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= R) return;
  double acc = 0.0;
  for (int l = 0; l < r; ++l) acc += V0[row + R * l] * w[l];
  const double v = scale * ((base ? base[row] : 0.0) - acc);
  if (out64) out64[row] = v;
  if (out32) out32[row] = (float)v;
}

hipError_t launch_vcol(const double *V0, int64_t R, int r, const double *w, const double *base,
                       double scale, double *out64, float *out32, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(vcol_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, V0, R, r,
                     w, base, scale, out64, out32);
  return hipGetLastError();
}

__global__ void m_update_kernel(const double *M, int r, const double *V2, int c, int grow,
                                double *Mn) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx % c, j = idx / c;
  const double *v2c = V2 + (size_t)(r + 1) * j;
  double acc;
  if (i < r) {
    acc = 0.0;
#pragma unroll 8
    for (int l = 0; l < r; ++l) acc += M[i + (size_t)r * l] * v2c[l];
  } else {  // grow: the appended direction of blockdiag(M, 1)
    acc = grow ? v2c[r] : 0.0;
  }
  Mn[i + (size_t)c * j] = acc;
}

hipError_t launch_m_update(const double *M, int r, const double *V2, int c, int grow,
                           double *Mn, hipStream_t s) {
  const int total = c * c;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(m_update_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, M,
                     r, V2, c, grow, Mn);
  return hipGetLastError();
}

__global__ void remap_rows_kernel(const double *src, int64_t ld_src, RowMap map, int64_t Rn,
                                  int cols, double *dst) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= Rn) return;
  const int64_t o = map_new_to_old(map, row);
  for (int j = 0; j < cols; ++j) dst[row + Rn * j] = (o >= 0) ? src[o + ld_src * j] : 0.0;
}

hipError_t launch_remap_rows(const double *src, int64_t ld_src, RowMap map, int64_t Rn,
                             int cols, double *dst, hipStream_t s) {
  if (Rn <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(remap_rows_kernel, dim3((unsigned)((Rn + 255) / 256)), dim3(256), 0, s, src,
                     ld_src, map, Rn, cols, dst);
  return hipGetLastError();
}

__global__ void mt_rows_kernel(const double *M, int n, const double *S, double *W, int64_t ldw) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int m = idx / n, k = idx % n;
  W[m * ldw + k] = M[k + (size_t)n * m] * (S ? S[m] : 1.0);
}

hipError_t launch_mt_rows(const double *M, int n, const double *S, double *W, int64_t ldw,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mt_rows_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, M, n,
                     S, W, ldw);
  return hipGetLastError();
}

__global__ void f64_to_f32_kernel(const double *x, int64_t n, float *y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

hipError_t launch_f64_to_f32(const double *x, int64_t n, float *y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     y);
  return hipGetLastError();
}

__global__ void identity_kernel(double *M, int n) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n * n) M[idx] = (idx % n == idx / n) ? 1.0 : 0.0;
}

hipError_t launch_identity(double *M, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(identity_kernel, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, s, M,
                     n);
  return hipGetLastError();
}

__global__ void ud_row64_kernel(const double *Ud, int64_t ld, int64_t t, int rd, const double *S,
                                double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < rd) out[j] = Ud[t + ld * j] * S[j];
}

hipError_t launch_ud_row64(const double *Ud, int64_t ld, int64_t t, int rd, const double *S,
                           double *out, hipStream_t s) {
  if (rd <= 0) return hipSuccess;
  hipLaunchKernelGGL(ud_row64_kernel, dim3((unsigned)((rd + 63) / 64)), dim3(64), 0, s, Ud, ld, t,
                     rd, S, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// V0^T x for a tall column-major V0 (R x r): lanes run over rows (coalesced
// column segments, no LDS). Block (bx, by) covers rows [kGemvRows bx,
// kGemvRows (bx + 1)) and columns [16 by, 16 by + 16), four per wave; each lane
// accumulates its kGemvRPL rows of every chunk in registers, so one wave
// reduction per column and block serves kGemvRows rows. The block writes
// part[j * nb + bx] (j < r), and blocks with by == 0 also part[r * nb + bx] =
// sum of x^2 over their rows.
// ---------------------------------------------------------------------------
constexpr int kGemvRPL = 8;                          // rows per lane and chunk
constexpr int kGemvChunks = 4;                       // chunks per block
constexpr int kGemvRows = 64 * kGemvRPL * kGemvChunks;  // 2048 rows per block

// MAPPED: V0 is stored at the old ranks (ld = ldv rows) and row i of the new
// layout reads old row map(i), or is zero for a padded row.
template <bool MAPPED>
__global__ __launch_bounds__(256) void gemv_t_kernel(const double *V0, int64_t ldv, RowMap map,
                                                     int64_t R, int r, const double *x,
                                                     double *part) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nb = gridDim.x;
  const int j0 = ((int)blockIdx.y * 4 + wid) * 4;  // this wave's four columns
  const bool norms = blockIdx.y == 0 && wid == 0;
  if (j0 >= r && !norms) return;
  const int64_t rowb = (int64_t)blockIdx.x * kGemvRows;
  const bool full = !MAPPED && rowb + kGemvRows <= R;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  double xx = 0.0;
  for (int ch = 0; ch < kGemvChunks; ++ch) {
    const int64_t row0 = rowb + (int64_t)ch * 64 * kGemvRPL + lane;
    double xv[kGemvRPL];
    int64_t src[kGemvRPL];
#pragma unroll
    for (int i = 0; i < kGemvRPL; ++i) {
      const int64_t row = row0 + 64 * i;
      const double v = x[row < R ? row : 0];
      xv[i] = row < R ? v : 0.0;
      src[i] = row < R ? (MAPPED ? map_new_to_old(map, row) : row) : -1;
    }
    if (norms) {
#pragma unroll
      for (int i = 0; i < kGemvRPL; ++i) xx += xv[i] * xv[i];
    }
    if (j0 >= r) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // columns past r repeat column j0 and are not stored
      const int j = (j0 + c < r) ? j0 + c : j0;
      const double *col = V0 + ldv * (int64_t)j;
      if (full) {
#pragma unroll
        for (int i = 0; i < kGemvRPL; ++i) s[c] += col[row0 + 64 * i] * xv[i];
      } else {
#pragma unroll
        for (int i = 0; i < kGemvRPL; ++i) {
          const double v = col[src[i] >= 0 ? src[i] : 0];
          s[c] += (src[i] >= 0 ? v : 0.0) * xv[i];
        }
      }
    }
  }
  if (j0 < r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double t = wave_sum(s[c]);
      if (lane == 0 && j0 + c < r) part[(size_t)(j0 + c) * nb + blockIdx.x] = t;
    }
  }
  if (norms) {
    xx = wave_sum(xx);
    if (lane == 0) part[(size_t)r * nb + blockIdx.x] = xx;
  }
}

// delta = a - b over n rows, and per block the pair (sum b * delta, sum
// delta^2) into part[2 * block]; reduced afterwards in a fixed order. Used to
// move the ISVD quantities of a slice from coordinates b (reduced-precision
// products) to the exact coordinates a without a second pass over V.
__global__ __launch_bounds__(256) void delta_kernel(const double *a, const double *b, int64_t n,
                                                    double *delta, double *part) {
  __shared__ double red[16];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double bi = b[i];
    const double dl = a[i] - bi;
    delta[i] = dl;
    s1 += bi * dl;
    s2 += dl * dl;
  }
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

hipError_t launch_delta(const double *a, const double *b, int64_t n, double *delta, double *part,
                        int nblocks, hipStream_t s) {
  if (nblocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(delta_kernel, dim3((unsigned)nblocks), dim3(256), 0, s, a, b, n, delta,
                     part);
  return hipGetLastError();
}

int gemv_t_blocks(int64_t R) {
  const int64_t t = (R + kGemvRows - 1) / kGemvRows;
  return (int)(t > 0 ? t : 1);
}

hipError_t launch_gemv_t(const double *V0, int64_t R, int r, const double *x, double *part,
                         int nb, hipStream_t s) {
  RowMap ident{};
  ident.identity = 1;
  hipLaunchKernelGGL(gemv_t_kernel<false>, dim3((unsigned)nb, (unsigned)(r > 0 ? (r + 15) / 16 : 1)), dim3(256),
                     0, s, V0, R, ident, R, r, x, part);
  return hipGetLastError();
}

hipError_t launch_gemv_t_mapped(const double *V, int64_t ldv, const RowMap &map, int64_t R, int r,
                                const double *x, double *part, int nb, hipStream_t s) {
  if (map.identity) return launch_gemv_t(V, R, r, x, part, nb, s);
  hipLaunchKernelGGL(gemv_t_kernel<true>, dim3((unsigned)nb, (unsigned)(r > 0 ? (r + 15) / 16 : 1)), dim3(256),
                     0, s, V, ldv, map, R, r, x, part);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The r x r part of the two Gram-Schmidt passes in the factored form, with
// G0 = V0^T V0 kept up to date so the second pass needs no sweep over V0:
//   p1 = M^T t1, w1 = M p1, t2 = t1 - G0 w1          (t2 = V0^T e1)
//   ||e1||^2 = ||d||^2 - 2 w1.t1 + w1.G0 w1
//   p2 = M^T t2, w2 = M p2, p = p1 + p2, ws = w1 + w2
//   q^2 = ||e1||^2 - 2 w2.t2 + w2.G0 w2              (e = e1 - V0 w2)
// With `given`, t2 and ||e1||^2 (sc[0]) come from an exact sweep instead.
// sc: [0] ||e1||^2, [1] q^2, [2] magnitude of the terms cancelled in q^2.
// One block; r x r products split over its threads.
// ---------------------------------------------------------------------------
// y = M^T x: one wave per output, lanes along the (contiguous) column of M
// (M null: the identity)
__device__ inline void mv_trans(const double *M, int r, const double *x, double *y) {
  if (!M) {
    for (int i = threadIdx.x; i < r; i += blockDim.x) y[i] = x[i];
    return;
  }
  // four outputs per wave and iteration: their loads are in flight together
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i0 = 4 * wid; i0 < r; i0 += 4 * nw) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = lane; l < r; l += 64) {
      const double xl = x[l];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = (i0 + c < r) ? i0 + c : i0;
        a[c] += M[l + (size_t)r * i] * xl;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double t = dpp_wave_sum(a[c]);
      if (lane == 0 && i0 + c < r) y[i0 + c] = t;
    }
  }
}

// Block-wide sum with DPP wave sums (every thread active), the result in every
// thread; scratch holds one double per wave.
__device__ inline double block_sum_dpp(double v, double *scratch) {
  const int nw = (int)(blockDim.x >> 6);
  v = dpp_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t += scratch[w];
  return t;
}

// y = M x (M column-major r x r). For r <= kMvRows the block's 16 waves split
// the columns l (wave w takes l = w, w + 16, ...) and the lanes the rows, so
// all loads of a wave are independent; the 16 partial vectors are summed in
// LDS. Larger r: one thread per output row.
constexpr int kMvRows = 256;
__device__ inline void mv_plain(const double *M, int r, const double *x, double *y,
                                double (*part)[kMvRows]) {
  if (!M) {
    for (int i = threadIdx.x; i < r; i += blockDim.x) y[i] = x[i];
    return;
  }
  if (r <= kMvRows && blockDim.x == 1024) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double a[kMvRows / 64];
#pragma unroll
    for (int c = 0; c < kMvRows / 64; ++c) a[c] = 0.0;
    for (int l = wid; l < r; l += 16) {
      const double xl = x[l];
      const double *mc = M + (size_t)r * l;
#pragma unroll
      for (int c = 0; c < kMvRows / 64; ++c) {
        const int i = lane + 64 * c;
        if (i < r) a[c] += mc[i] * xl;
      }
    }
#pragma unroll
    for (int c = 0; c < kMvRows / 64; ++c) {
      const int i = lane + 64 * c;
      if (i < r) part[wid][i] = a[c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += blockDim.x) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < 16; ++w) t += part[w][i];
      y[i] = t;
    }
    __syncthreads();
    return;
  }
  for (int i = threadIdx.x; i < r; i += blockDim.x) {
    double a = 0.0;
    for (int l = 0; l < r; ++l) a += M[i + (size_t)r * l] * x[l];
    y[i] = a;
  }
}

__global__ __launch_bounds__(1024) void isvd_gram_kernel(const double *M, const double *G0, int r,
                                                         const double *t1, const double *dd,
                                                         int given, double *p1, double *w1,
                                                         double *t2, double *p2, double *w2,
                                                         double *p, double *ws, double *sc,
                                                         double *g, double *ge) {
  __shared__ double red[16];
  __shared__ double part[16][kMvRows];
  const int tid = threadIdx.x;
  mv_trans(M, r, t1, p1);
  __syncthreads();
  mv_plain(M, r, p1, w1, part);
  __syncthreads();
  mv_plain(G0, r, w1, g, part);  // G0 is symmetric
  __syncthreads();
  double a1 = 0.0, a2 = 0.0;
  for (int i = tid; i < r; i += blockDim.x) {
    if (!given) t2[i] = t1[i] - g[i];
    a1 += w1[i] * t1[i];
    a2 += w1[i] * g[i];
  }
  a1 = block_sum_dpp(a1, red);
  a2 = block_sum_dpp(a2, red);
  const double e1sq = given ? sc[0] : dd[0] - 2.0 * a1 + a2;
  __syncthreads();
  mv_trans(M, r, t2, p2);
  __syncthreads();
  for (int i = tid; i < r; i += blockDim.x) p[i] = p1[i] + p2[i];
  mv_plain(M, r, p2, w2, part);
  __syncthreads();
  mv_plain(G0, r, w2, g, part);
  __syncthreads();
  double b1 = 0.0, b2 = 0.0;
  for (int i = tid; i < r; i += blockDim.x) {
    ws[i] = w1[i] + w2[i];
    if (ge) ge[i] = t2[i] - g[i];  // V0^T e with e = e1 - V0 w2
    b1 += w2[i] * t2[i];
    b2 += w2[i] * g[i];
  }
  b1 = block_sum_dpp(b1, red);
  b2 = block_sum_dpp(b2, red);
  if (tid == 0) {
    sc[0] = e1sq;
    sc[1] = e1sq - 2.0 * b1 + b2;
    sc[2] = (given ? e1sq : dd[0] + 2.0 * fabs(a1) + fabs(a2)) + 2.0 * fabs(b1) + fabs(b2);
  }
}

hipError_t launch_isvd_gram(const double *M, const double *G0, int r, const double *t1,
                            const double *dd, int given, double *p1, double *w1, double *t2,
                            double *p2, double *w2, double *p, double *ws, double *sc,
                            double *g, double *ge, hipStream_t s) {
  hipLaunchKernelGGL(isvd_gram_kernel, dim3(1), dim3(1024), 0, s, M, G0, r, t1, dd, given, p1,
                     w1, t2, p2, w2, p, ws, sc, g, ge);
  return hipGetLastError();
}

// Gn ((r + 1) x (r + 1)) = [[G0, g / q], [g^T / q, ee / q^2]] after appending
// v = e / q to V0 (g = V0^T e, ee = ||e||^2, q = sqrt(ee) read on the device, so
// the appended column has unit norm whatever q decided the growth); or Gn = G0
// (grow = 0).
__global__ void g0_update_kernel(const double *G0, int r, const double *g, const double *ee,
                                 int grow, double *Gn) {
  const int c = r + grow;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= c * c) return;
  const int i = idx % c, j = idx / c;
  double v;
  if (i < r && j < r) {
    v = G0[i + (size_t)r * j];
  } else {
    const double inv_q = 1.0 / sqrt(ee[0]);
    if (i < r) v = g[i] * inv_q;
    else if (j < r) v = g[j] * inv_q;
    else v = ee[0] * inv_q * inv_q;
  }
  Gn[i + (size_t)c * j] = v;
}

hipError_t launch_g0_update(const double *G0, int r, const double *g, const double *ee, int grow,
                            double *Gn, hipStream_t s) {
  const int c = r + grow;
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(g0_update_kernel, dim3((unsigned)((c * c + 255) / 256)), dim3(256), 0, s,
                     G0, r, g, ee, grow, Gn);
  return hipGetLastError();
}

// out[i] = sum_b part[b * n + i] (b < nb), one thread per entry, in a fixed
// order: four interleaved partial sums, then their pairwise sum.
// Blocks of 64 outputs and 16 waves: wave w sums the partials w, w + 16, ...
// (rows of 64 consecutive doubles, two chains), then the 16 wave sums are
// added in a fixed order. Spreading the partials over the waves keeps many
// loads in flight even when there are few outputs (a small Gram over many
// row chunks).
__global__ __launch_bounds__(1024) void batch_sum_kernel(const double *part, int nb, int64_t n,
                                                         double *out) {
  __shared__ double ws[16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double a0 = 0.0, a1 = 0.0;
  if (i < n) {
    int b = w;
    for (; b + 16 < nb; b += 32) {
      a0 += part[(size_t)b * n + i];
      a1 += part[(size_t)(b + 16) * n + i];
    }
    if (b < nb) a0 += part[(size_t)b * n + i];
  }
  ws[w][lane] = a0 + a1;
  __syncthreads();
  if (w == 0 && i < n) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += ws[q][lane];
    out[i] = t;
  }
}

hipError_t launch_batch_sum(const double *part, int nb, int64_t n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_sum_kernel, dim3((unsigned)((n + 63) / 64)), dim3(1024), 0, s, part,
                     nb, n, out);
  return hipGetLastError();
}

// out = a + b (n entries; out may alias a or b)
__global__ void vadd_kernel(const double *a, const double *b, int64_t n, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

hipError_t launch_vadd(const double *a, const double *b, int64_t n, double *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(vadd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n,
                     out);
  return hipGetLastError();
}

// x /= sqrt(ss[0]) (ss on the device: a sum of squares formed by an earlier launch)
__global__ void scale_rsqrt_kernel(double *x, int64_t n, const double *ss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= 1.0 / sqrt(ss[0]);
}

hipError_t launch_scale_rsqrt(double *x, int64_t n, const double *ss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_rsqrt_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     ss);
  return hipGetLastError();
}

// C (m x n, ld ldc) = op(A) B with op(A) = A (m x k, ld lda) or A^T (A k x m),
// B k x n (ld ldb); one thread per output (small r x r products).
__global__ void small_gemm_kernel(int transA, const double *A, int64_t lda, const double *B,
                                  int64_t ldb, double *C, int64_t ldc, int m, int n, int k) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int i = idx % m, j = idx / m;
  const double *bc = B + ldb * j;
  double acc = 0.0;
  if (transA) {
    const double *ac = A + lda * i;
#pragma unroll 8
    for (int l = 0; l < k; ++l) acc += ac[l] * bc[l];
  } else {
#pragma unroll 8
    for (int l = 0; l < k; ++l) acc += A[i + lda * l] * bc[l];
  }
  C[i + ldc * j] = acc;
}

hipError_t launch_small_gemm(int transA, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, int m, int n, int k,
                             hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s,
                     transA, A, lda, B, ldb, C, ldc, m, n, k);
  return hipGetLastError();
}

}  // namespace st
