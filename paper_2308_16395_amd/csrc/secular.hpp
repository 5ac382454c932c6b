// SVD of the small ISVD middle matrix S' (Alg. 3) through its secular equation.
//
// S' is diagonal plus one row: S' = [[diag(s), 0], [p^T, q]] when the new
// direction is kept (q > eps) and S' = [diag(s); p^T] when it is ignored. With
// the p-row moved to the top, the q-column to the front and the s-entries sorted
// ascending, S' becomes the upper arrow matrix
//     M = e_0 z^T + diag(d),  d_0 = 0 < d_1 <= ... <= d_r,  z = (q, p...),
// whose Gram is M^T M = diag(d)^2 + z z^T (diagonal plus rank one). Its singular
// values solve f(sigma) = 1 + sum_t z_t^2 / (d_t^2 - sigma^2) = 0, one root in
// each gap between consecutive poles and one above the largest, and
//     v = (z_t / (d_t^2 - sigma^2))_t,   u = (-1, d_1 v_1, ..., d_r v_r)
// are its singular vectors up to normalisation (Golub 1973; Bunch, Nielsen and
// Sorensen 1978). For orthogonal vectors in floating point, z is replaced by
// the z^ for which the computed roots are exact (Gu and Eisenstat 1995):
//     z^_t^2 = prod_i (lambda_i - d_t^2) / prod_{j != t} (d_j^2 - d_t^2).
// Entries with |z_t| below the tolerance, and the lower of two poles closer than
// the tolerance (after a Givens rotation that moves its weight to the upper
// one), deflate to the singular triplet (d_t, e_t, e_t).
//
// Every difference lambda_i - d_t^2 is formed from the root's offset mu_i to
// its nearest pole o_i as (d_o - d_t)(d_o + d_t) + mu_i, which keeps it
// accurate to a few ulps. The functions are templated on a reducer so that the
// same code runs with lane-parallel sums in a wavefront and with plain loops on
// the host.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define ST_HD __host__ __device__
#else
#define ST_HD
#endif

namespace st {

struct SecData {
  int n;           // r + 1
  int r;
  double *d;       // [n] poles, ascending, d[0] = 0
  double *z;       // [n] weights after deflation rotations
  double *zh;      // [n] z^ (0 for deflated entries)
  int *active;     // [n]
  int *K;          // [n] active indices ascending (first m used)
  int *defl;       // [n] deflated indices t >= 1 ascending
  int *org;        // [n] origin pole of each root
  double *mu;      // [n] root offset from its origin pole (in squared units)
  int *rot_t;      // [2n] rotation index pairs (lower, upper)
  double *rot_cs;  // [2n] rotation (c, s)
  int *counts;     // [3] m, number of deflated t >= 1, number of rotations
  double *zz;      // [1] sum of z_t^2 over active t
};

// Build poles, weights and deflation (single thread).
ST_HD inline void sec_prep(SecData s, const double *S, const double *p, double q, int grow,
                           double tol) {
  const int r = s.r;
  s.d[0] = 0.0;
  s.z[0] = grow ? q : 0.0;
  for (int t = 1; t <= r; ++t) {
    s.d[t] = S[r - t];
    s.z[t] = p[r - t];
  }
  s.active[0] = grow ? 1 : 0;
  for (int t = 1; t <= r; ++t) s.active[t] = fabs(s.z[t]) > tol ? 1 : 0;
  int nrot = 0, prev = -1;
  for (int t = 1; t <= r; ++t) {
    if (!s.active[t]) continue;
    if (prev >= 1 && s.d[t] - s.d[prev] <= tol) {
      const double za = s.z[prev], zb = s.z[t];
      const double rho = hypot(za, zb);
      const double c = zb / rho, sn = za / rho;
      s.z[t] = rho;
      s.z[prev] = 0.0;
      s.active[prev] = 0;
      s.rot_t[2 * nrot] = prev;
      s.rot_t[2 * nrot + 1] = t;
      s.rot_cs[2 * nrot] = c;
      s.rot_cs[2 * nrot + 1] = sn;
      ++nrot;
    }
    prev = t;
  }
  int m = 0, nd = 0;
  double zz = 0.0;
  for (int t = 0; t <= r; ++t) {
    if (s.active[t]) {
      s.K[m++] = t;
      zz += s.z[t] * s.z[t];
    } else if (t >= 1) {
      s.defl[nd++] = t;
    }
  }
  s.counts[0] = m;
  s.counts[1] = nd;
  s.counts[2] = nrot;
  s.zz[0] = zz;
}

// f(mu) at sigma^2 = d_o^2 + mu, summed over the active poles.
template <class Red>
ST_HD inline double sec_f(const SecData &s, int m, double dor, double mu, const Red &red) {
  return 1.0 + red.sum(m, [&](int j) {
    const int t = s.K[j];
    const double dt = s.d[t];
    const double del = (dt - dor) * (dt + dor);
    return s.z[t] * s.z[t] / (del - mu);
  });
}

// Root i (ascending) by bracketing bisection on the offset from the nearer pole:
// geometric steps while the bracket spans more than a factor of two, then halving.
template <class Red>
ST_HD inline void sec_root(const SecData &s, int i, const Red &red, int *org, double *mu) {
  const int m = s.counts[0];
  const int lo = s.K[i];
  const double dlo = s.d[lo];
  int o = lo;
  double sgn = 1.0, h;
  if (i + 1 < m) {
    const int hi = s.K[i + 1];
    const double dhi = s.d[hi];
    const double mid = 0.5 * (dhi - dlo) * (dhi + dlo);
    const double fm = sec_f(s, m, dlo, mid, red);
    if (fm < 0.0) {
      o = hi;
      sgn = -1.0;
    }
    h = mid;
  } else {
    h = s.zz[0];
  }
  const double dor = s.d[o];
  // F(nu) = sgn * f(sgn * nu) increases from -inf at nu = 0+ and F(h) >= 0.
  double a = h * 0x1p-120, b = h;
  if (sgn * sec_f(s, m, dor, sgn * a, red) >= 0.0) {
    *org = o;
    *mu = sgn * a;
    return;
  }
  for (int it = 0; it < 400; ++it) {
    const double c = (b > 2.0 * a) ? sqrt(a * b) : 0.5 * (a + b);
    if (!(c > a && c < b)) break;
    if (sgn * sec_f(s, m, dor, sgn * c, red) < 0.0)
      a = c;
    else
      b = c;
  }
  *org = o;
  *mu = sgn * 0.5 * (a + b);
}

// lambda_i - d_t^2 for root i.
ST_HD inline double sec_lam_minus(const SecData &s, int i, double dt) {
  const double dor = s.d[s.org[i]];
  return (dor - dt) * (dor + dt) + s.mu[i];
}

// z^ of the active pole K[jt] (Gu-Eisenstat), with factors paired so that
// every ratio lies in (0, 1].
template <class Red>
ST_HD inline double sec_zhat(const SecData &s, int jt, const Red &red) {
  const int m = s.counts[0];
  const int t = s.K[jt];
  const double dt = s.d[t];
  const double prod = red.prod(m, [&](int i) {
    const double num = sec_lam_minus(s, i, dt);
    if (i == m - 1) return num;
    const int pole = (i < jt) ? s.K[i] : s.K[i + 1];
    const double dp = s.d[pole];
    return num / ((dp - dt) * (dp + dt));
  });
  const double mag = sqrt(prod > 0.0 ? prod : 0.0);
  return s.z[t] < 0.0 ? -mag : mag;
}

// Singular value of triplet `trip` (roots first, then deflated poles).
ST_HD inline double sec_sigma(const SecData &s, int trip) {
  const int m = s.counts[0];
  if (trip < m) {
    const double dor = s.d[s.org[trip]];
    const double l = dor * dor + s.mu[trip];
    return sqrt(l > 0.0 ? l : 0.0);
  }
  return s.d[s.defl[trip - m]];
}

// Unnormalised singular vectors of triplet `trip` in the arrow-matrix index
// space, with the deflation rotations applied (last one first); returns the
// singular value and writes the two norms. `red` supplies for_each (parallel
// over t), sync, single, sum.
template <class Red>
ST_HD inline double sec_vectors(const SecData &s, int trip, double *u, double *v,
                                const Red &red, double *nu, double *nv) {
  const int m = s.counts[0];
  const int n = s.n;
  const double sigma = sec_sigma(s, trip);
  if (trip < m) {
    const int o = s.org[trip];
    const double dor = s.d[o], mu = s.mu[trip];
    red.for_each(n, [&](int t) {
      double vt = 0.0;
      if (s.active[t]) {
        const double dt = s.d[t];
        const double den = -((dor - dt) * (dor + dt) + mu);  // d_t^2 - lambda
        vt = s.zh[t] / den;
      }
      v[t] = vt;
      u[t] = (t == 0) ? -1.0 : s.d[t] * vt;
    });
  } else {
    const int td = s.defl[trip - m];
    red.for_each(n, [&](int t) {
      v[t] = (t == td) ? 1.0 : 0.0;
      u[t] = (t == td) ? 1.0 : 0.0;
    });
  }
  red.sync();
  red.single([&]() {
    for (int k = s.counts[2] - 1; k >= 0; --k) {
      const int ta = s.rot_t[2 * k], tb = s.rot_t[2 * k + 1];
      const double c = s.rot_cs[2 * k], sn = s.rot_cs[2 * k + 1];
      double a = u[ta], b = u[tb];
      u[ta] = c * a + sn * b;
      u[tb] = -sn * a + c * b;
      a = v[ta];
      b = v[tb];
      v[ta] = c * a + sn * b;
      v[tb] = -sn * a + c * b;
    }
  });
  red.sync();
  *nu = sqrt(red.sum(n, [&](int t) { return u[t] * u[t]; }));
  *nv = sqrt(red.sum(n, [&](int t) { return v[t] * v[t]; }));
  return sigma;
}

// Output column of triplet `trip`: singular values in descending order, ties
// broken by triplet index.
template <class Red>
ST_HD inline int sec_rank(const SecData &s, int trip, int ntrip, const Red &red) {
  const double me = sec_sigma(s, trip);
  const double cnt = red.sum(ntrip, [&](int j) {
    const double o = sec_sigma(s, j);
    return (o > me || (o == me && j < trip)) ? 1.0 : 0.0;
  });
  return (int)(cnt + 0.5);
}

}  // namespace st
