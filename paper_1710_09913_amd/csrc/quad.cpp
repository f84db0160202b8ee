// Reference quadrature and basis tables of the conventional quadrature-point apply
// (the matrix-free evaluation over integration points that the paper compares
// DoGIP with, Section 3.3).
#include <cmath>

#include "internal.hpp"
#include "reftab.hpp"

namespace dogip {

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_n in long double).
static void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double t = std::cos(pi * (i + 0.75L) / (n + 0.5L)), dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = t;  // P_0, P_1
      for (int m = 2; m <= n; ++m) {
        const long double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0L;
      dp = n * (t * p1 - p0) / (t * t - 1.0L);  // P_n'
      const long double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-30L) break;
    }
    // recompute P_n' at the converged node
    long double p0 = 1.0L, p1 = t;
    for (int m = 2; m <= n; ++m) {
      const long double p2 = ((2 * m - 1) * t * p1 - (m - 1) * p0) / m;
      p0 = p1;
      p1 = p2;
    }
    dp = n == 1 ? 1.0L : n * (t * p1 - p0) / (t * t - 1.0L);
    x[n - 1 - i] = double((1.0L + t) / 2.0L);  // ascending
    w[n - 1 - i] = double(1.0L / ((1.0L - t * t) * dp * dp));  // 2 / ((1-t^2) P'^2) / 2
  }
}

void collapsed_rule(int d, int n, std::vector<double>& pts, std::vector<double>& wts) {
  DOGIP_CHECK(d == 2 || d == 3, DOGIP_E_RANGE, "dim must be 2 or 3");
  DOGIP_CHECK(n >= 1 && n <= 16, DOGIP_E_RANGE, "points per direction must be 1..16");
  std::vector<double> g, w;
  gauss_legendre01(n, g, w);
  pts.clear();
  wts.clear();
  if (d == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double s = g[i], t = g[j];
        pts.push_back(s);
        pts.push_back(t * (1.0 - s));
        wts.push_back(w[i] * w[j] * (1.0 - s));
      }
  } else {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
          const double s = g[i], t = g[j], v = g[l];
          pts.push_back(s);
          pts.push_back(t * (1.0 - s));
          pts.push_back(v * (1.0 - s) * (1.0 - t));
          wts.push_back(w[i] * w[j] * w[l] * (1.0 - s) * (1.0 - s) * (1.0 - t));
        }
  }
}

// R_m(lam) = prod_{s<m} (k lam - s)/(s+1) and its derivative (Silvester's product form).
static long double pf(int k, int m, long double t) {
  long double v = 1.0L;
  for (int s = 0; s < m; ++s) v *= (k * t - s) / (s + 1);
  return v;
}
static long double pf_der(int k, int m, long double t) {
  long double tot = 0.0L;
  for (int s = 0; s < m; ++s) {
    long double term = (long double)k / (s + 1);
    for (int s2 = 0; s2 < m; ++s2)
      if (s2 != s) term *= (k * t - s2) / (s2 + 1);
    tot += term;
  }
  return tot;
}

void basis_table(int d, int k, int kind, const std::vector<double>& pts, std::vector<double>& tab) {
  const int vt = dim_p(d, k), nq = int(pts.size()) / d, nb = kind == KIND_SE ? d : 1;
  tab.assign(size_t(nq) * nb * vt, 0.0);
  for (int q = 0; q < nq; ++q) {
    long double lam[4] = {1.0L, 0.0L, 0.0L, 0.0L};
    for (int r = 0; r < d; ++r) {
      lam[r + 1] = pts[size_t(q) * d + r];
      lam[0] -= lam[r + 1];
    }
    for (int l = 0; l < vt; ++l) {
      int b[4] = {0, 0, 0, 0};
      ref::bary_index(d, k, l, b);
      if (kind == KIND_WP) {
        long double v = 1.0L;
        for (int j = 0; j <= d; ++j) v *= pf(k, b[j], lam[j]);
        tab[size_t(q) * vt + l] = double(v);
      } else {
        auto dlam = [&](int jj) {
          long double v = pf_der(k, b[jj], lam[jj]);
          for (int j = 0; j <= d; ++j)
            if (j != jj) v *= pf(k, b[j], lam[j]);
          return v;
        };
        for (int r = 0; r < d; ++r) tab[(size_t(q) * nb + r) * vt + l] = double(dlam(r + 1) - dlam(0));
      }
    }
  }
}

void coarse_basis_at_nodes(int d, int kf, std::vector<double>& tab) {
  const int kc = kf - 1, vf = dim_p(d, kf), vc = dim_p(d, kc);
  tab.assign(size_t(vf) * vc, 0.0);
  for (int l = 0; l < vf; ++l) {
    int bf[4] = {0, 0, 0, 0};
    ref::bary_index(d, kf, l, bf);
    long double lam[4];
    for (int j = 0; j <= d; ++j) lam[j] = (long double)bf[j] / kf;
    for (int c = 0; c < vc; ++c) {
      int b[4] = {0, 0, 0, 0};
      if (kc > 0) ref::bary_index(d, kc, c, b);
      long double v = 1.0L;
      for (int j = 0; j <= d; ++j) v *= pf(kc, b[j], lam[j]);
      tab[size_t(l) * vc + c] = std::fabs(double(v)) < 1e-13 ? 0.0 : double(v);
    }
  }
}

}  // namespace dogip
