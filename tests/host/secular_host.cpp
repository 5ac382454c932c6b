// Host build of the library's secular-equation SVD (secular.hpp) with plain
// loops in place of wavefront reductions, for CPU unit tests.
#include <cmath>
#include <vector>

#include "secular.hpp"

namespace {
struct HostRed {
  template <class F>
  double sum(int m, F f) const {
    double a = 0.0;
    for (int j = 0; j < m; ++j) a += f(j);
    return a;
  }
  template <class F>
  double prod(int m, F f) const {
    double a = 1.0;
    for (int j = 0; j < m; ++j) a *= f(j);
    return a;
  }
  template <class F>
  void for_each(int m, F f) const {
    for (int j = 0; j < m; ++j) f(j);
  }
  void sync() const {}
  template <class F>
  void single(F f) const {
    f();
  }
};
}  // namespace

extern "C" int sec_svd_host(int r, const double *S, const double *p, double q, int grow,
                            double tol, double *U2, double *V2, double *Snew, int *counts_out) {
  const int n = r + 1;
  std::vector<double> d(n), z(n), zh(n, 0.0), mu(n), rcs(2 * n), zz(1);
  std::vector<int> act(n), K(n), defl(n), org(n), rt(2 * n), counts(3);
  st::SecData s{};
  s.n = n;
  s.r = r;
  s.d = d.data();
  s.z = z.data();
  s.zh = zh.data();
  s.active = act.data();
  s.K = K.data();
  s.defl = defl.data();
  s.org = org.data();
  s.mu = mu.data();
  s.rot_t = rt.data();
  s.rot_cs = rcs.data();
  s.counts = counts.data();
  s.zz = zz.data();
  st::sec_prep(s, S, p, q, grow, tol);
  HostRed red;
  const int m = counts[0];
  for (int i = 0; i < m; ++i) st::sec_root(s, i, red, &org[i], &mu[i]);
  for (int jt = 0; jt < m; ++jt) zh[K[jt]] = st::sec_zhat(s, jt, red);
  const int ntrip = grow ? n : n - 1;
  std::vector<double> u(n), v(n);
  for (int trip = 0; trip < ntrip; ++trip) {
    double nu, nv;
    const double sigma = st::sec_vectors(s, trip, u.data(), v.data(), red, &nu, &nv);
    const int col = st::sec_rank(s, trip, ntrip, red);
    for (int t = 0; t < n; ++t) {
      const int orig = (t == 0) ? r : r - t;
      U2[orig + (size_t)n * col] = u[t] / nu;
      V2[orig + (size_t)n * col] = v[t] / nv;
    }
    Snew[col] = sigma;
  }
  for (int i = 0; i < 3; ++i) counts_out[i] = counts[i];
  return ntrip;
}
