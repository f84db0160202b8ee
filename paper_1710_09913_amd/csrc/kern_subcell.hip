// D for a coefficient with jumps inside the cells (inclusions: a_in inside a union of
// balls, a_out elsewhere) by sub-cell quadrature, one thread per cell:
//   int_T a phi^W_i = a_out |T| w^_i + (a_in - a_out) int_T 1_B phi^W_i,
// the second integral over the red refinement of the reference cell, refined only
// where a sub-simplex is cut by a ball boundary, down to `depth` levels.  A sub-simplex
// whose vertices all lie in one ball is inside (balls are convex); one whose bounding
// sphere misses every ball is outside.  Inside sub-simplices and cut ones at the last
// level are integrated with the collapsed Gauss rule mapped onto them; on cut ones the
// indicator is evaluated at the points.  D_T,i then follows Theorem 2 or 4.
#include "kern_common.hpp"

namespace dogip {
namespace dev {

template <int D>
__device__ __forceinline__ int classify_sub(const double (&P)[D + 1][D], const double* __restrict__ balls, int nb) {
  double g[D] = {};
  for (int v = 0; v <= D; ++v)
    for (int x = 0; x < D; ++x) g[x] += P[v][x];
  for (int x = 0; x < D; ++x) g[x] /= double(D + 1);
  double rho = 0.0;
  for (int v = 0; v <= D; ++v) {
    double s = 0.0;
    for (int x = 0; x < D; ++x) s += (P[v][x] - g[x]) * (P[v][x] - g[x]);
    rho = fmax(rho, sqrt(s));
  }
  bool outside = true;
  for (int j = 0; j < nb; ++j) {
    const double* c = balls + j * (D + 1);
    const double r = c[D];
    bool all_in = true;
    for (int v = 0; v <= D; ++v) {
      double s = 0.0;
      for (int x = 0; x < D; ++x) s += (P[v][x] - c[x]) * (P[v][x] - c[x]);
      all_in = all_in && sqrt(s) < r;
    }
    if (all_in) return 1;
    double s = 0.0;
    for (int x = 0; x < D; ++x) s += (c[x] - g[x]) * (c[x] - g[x]);
    outside = outside && (sqrt(s) - rho >= r);
  }
  return outside ? 0 : 2;
}

// Child `c` of the red refinement of v (in place); the children order of the oracle.
template <int D>
__device__ __forceinline__ void red_child(double (&v)[D + 1][D], int c) {
  double m[D + 1][D + 1][D];
  for (int i = 0; i <= D; ++i)
    for (int j = i + 1; j <= D; ++j)
      for (int x = 0; x < D; ++x) m[i][j][x] = (v[i][x] + v[j][x]) * 0.5;
  double o[D + 1][D];
  auto put = [&](int slot, const double* p) {
    for (int x = 0; x < D; ++x) o[slot][x] = p[x];
  };
  if constexpr (D == 2) {
    switch (c) {
      case 0: put(0, v[0]); put(1, m[0][1]); put(2, m[0][2]); break;
      case 1: put(0, m[0][1]); put(1, v[1]); put(2, m[1][2]); break;
      case 2: put(0, m[0][2]); put(1, m[1][2]); put(2, v[2]); break;
      default: put(0, m[0][1]); put(1, m[1][2]); put(2, m[0][2]); break;
    }
  } else {
    switch (c) {
      case 0: put(0, v[0]); put(1, m[0][1]); put(2, m[0][2]); put(3, m[0][3]); break;
      case 1: put(0, m[0][1]); put(1, v[1]); put(2, m[1][2]); put(3, m[1][3]); break;
      case 2: put(0, m[0][2]); put(1, m[1][2]); put(2, v[2]); put(3, m[2][3]); break;
      case 3: put(0, m[0][3]); put(1, m[1][3]); put(2, m[2][3]); put(3, v[3]); break;
      case 4: put(0, m[0][1]); put(1, m[0][2]); put(2, m[0][3]); put(3, m[1][3]); break;
      case 5: put(0, m[0][1]); put(1, m[0][2]); put(2, m[1][2]); put(3, m[1][3]); break;
      case 6: put(0, m[0][2]); put(1, m[0][3]); put(2, m[1][3]); put(3, m[2][3]); break;
      default: put(0, m[0][2]); put(1, m[1][2]); put(2, m[1][3]); put(3, m[2][3]); break;
    }
  }
  for (int i = 0; i <= D; ++i)
    for (int x = 0; x < D; ++x) v[i][x] = o[i][x];
}

template <int D>
__device__ __forceinline__ double det_abs(const double (&M)[D][D]) {
  if constexpr (D == 2) return fabs(M[0][0] * M[1][1] - M[0][1] * M[1][0]);
  return fabs(M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
              M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]));
}

// Barycentric multi-indices of the W nodes (order Q) as a device table.
template <int D, int Q>
struct CBary {
  static constexpr int WT = dim_p(D, Q);
  uint8_t b[WT][D + 1];
  constexpr CBary() : b{} {
    for (int i = 0; i < WT; ++i) {
      int t[4] = {0, 0, 0, 0};
      if (Q > 0) ref::bary_index(D, Q, i, t);
      for (int j = 0; j <= D; ++j) b[i][j] = uint8_t(t[j]);
    }
  }
};
template <int D, int Q>
__constant__ CBary<D, Q> cbary{};

template <int D, int Q>
__global__ __launch_bounds__(128) void k_build_d_sub(SubLaunch a) {
  constexpr int WT = dim_p(D, Q), NCH = 1 << D;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= a.nel) return;
  double X[D + 1][D];
  for (int j = 0; j <= D; ++j) {
    const int64_t v = a.cells[e * (D + 1) + j];
    for (int x = 0; x < D; ++x) X[j][x] = a.xyz[v * D + x];
  }
  double R[D][D];  // columns X_r - X_0
  for (int x = 0; x < D; ++x)
    for (int r = 0; r < D; ++r) R[x][r] = X[r + 1][x] - X[0][x];
  double acc[WT];
  for (int i = 0; i < WT; ++i) acc[i] = 0.0;
  int64_t total = 1;
  for (int l = 0; l < a.depth; ++l) total *= NCH;
  int64_t npts = 0;
  for (int64_t idx = 0; idx < total;) {
    double v[D + 1][D] = {};
    for (int r = 0; r < D; ++r) v[r + 1][r] = 1.0;
    int l = 0, cls = 0;
    int64_t span = total;  // leaves under the current sub-simplex
    for (;;) {
      double P[D + 1][D];
      for (int i = 0; i <= D; ++i)
        for (int x = 0; x < D; ++x) {
          double s = X[0][x];
          for (int r = 0; r < D; ++r) s += R[x][r] * v[i][r];
          P[i][x] = s;
        }
      cls = classify_sub<D>(P, a.balls, a.nballs);
      if (cls != 2 || l == a.depth) break;
      span /= NCH;
      red_child<D>(v, int((idx / span) % NCH));
      ++l;
    }
    if (cls != 0) {
      double Rs[D][D];
      for (int x = 0; x < D; ++x)
        for (int r = 0; r < D; ++r) Rs[x][r] = v[r + 1][x] - v[0][x];
      const double js = det_abs<D>(Rs);
      for (int g = 0; g < a.ng; ++g) {
        double xh[D];
        for (int x = 0; x < D; ++x) {
          double s = v[0][x];
          for (int r = 0; r < D; ++r) s += Rs[x][r] * a.gpts[g * D + r];
          xh[x] = s;
        }
        ++npts;
        if (cls == 2) {
          bool in = false;
          for (int j = 0; j < a.nballs && !in; ++j) {
            const double* c = a.balls + j * (D + 1);
            double s = 0.0;
            for (int x = 0; x < D; ++x) {
              double p = X[0][x];
              for (int r = 0; r < D; ++r) p += R[x][r] * xh[r];
              s += (p - c[x]) * (p - c[x]);
            }
            in = sqrt(s) < c[D];
          }
          if (!in) continue;
        }
        const double w = a.gwts[g] * js;
        // Silvester factors P[j][m] = prod_{s<m} (Q lam_j - s)/(s+1)
        double lam[D + 1];
        lam[0] = 1.0;
        for (int r = 0; r < D; ++r) {
          lam[r + 1] = xh[r];
          lam[0] -= xh[r];
        }
        double pf[D + 1][Q + 1];
        for (int j = 0; j <= D; ++j) {
          pf[j][0] = 1.0;
          for (int m = 1; m <= Q; ++m) pf[j][m] = pf[j][m - 1] * (Q * lam[j] - (m - 1)) / m;
        }
        for (int i = 0; i < WT; ++i) {
          double phi = 1.0;
          for (int j = 0; j <= D; ++j) phi *= pf[j][cbary<D, Q>.b[i][j]];
          acc[i] = fma(w, phi, acc[i]);
        }
      }
    }
    idx += span;
  }
  if (a.npts) a.npts[e] = double(npts);
  // D_T,i (Theorems 2 and 4 with the scalar coefficient)
  const double J = det_abs<D>(R), vol = J / (D == 2 ? 2.0 : 6.0);
  const int64_t w = e >> 6, lane = e & 63;
  auto store = [&](int f, double val) {
    a.d64[(w * a.nch64 + (f >> 1)) * 128 + lane * 2 + (f & 1)] = val;
    if (a.d32) a.d32[d32_pos(w, int(lane), f, a.nch32)] = float(val);
  };
  double K[6] = {};
  if (a.kind == KIND_SE) {
    double Ri[D][D];
    if constexpr (D == 2) {
      const double det = R[0][0] * R[1][1] - R[0][1] * R[1][0];
      Ri[0][0] = R[1][1] / det;
      Ri[0][1] = -R[0][1] / det;
      Ri[1][0] = -R[1][0] / det;
      Ri[1][1] = R[0][0] / det;
    } else {
      const double c00 = R[1][1] * R[2][2] - R[1][2] * R[2][1];
      const double c01 = R[1][2] * R[2][0] - R[1][0] * R[2][2];
      const double c02 = R[1][0] * R[2][1] - R[1][1] * R[2][0];
      const double det = R[0][0] * c00 + R[0][1] * c01 + R[0][2] * c02;
      Ri[0][0] = c00 / det;
      Ri[1][0] = c01 / det;
      Ri[2][0] = c02 / det;
      Ri[0][1] = (R[0][2] * R[2][1] - R[0][1] * R[2][2]) / det;
      Ri[1][1] = (R[0][0] * R[2][2] - R[0][2] * R[2][0]) / det;
      Ri[2][1] = (R[0][1] * R[2][0] - R[0][0] * R[2][1]) / det;
      Ri[0][2] = (R[0][1] * R[1][2] - R[0][2] * R[1][1]) / det;
      Ri[1][2] = (R[0][2] * R[1][0] - R[0][0] * R[1][2]) / det;
      Ri[2][2] = (R[0][0] * R[1][1] - R[0][1] * R[1][0]) / det;
    }
    int c = 0;
    for (int r = 0; r < D; ++r)
      for (int s = r; s < D; ++s) {
        double t = 0.0;
        for (int p = 0; p < D; ++p) t += Ri[r][p] * Ri[s][p];
        K[c++] = t;
      }
  }
  const int ns = a.kind == KIND_SE ? n_sym(D) : 1;
  for (int i = 0; i < WT; ++i) {
    const double integ = a.a_out * vol * a.what[i] + (a.a_in - a.a_out) * J * acc[i];
    if (a.kind == KIND_SE)
      for (int c = 0; c < ns; ++c) store(i * ns + c, integ * K[c]);
    else
      store(i, integ);
  }
}

template <int D, int Q>
void sub_t(const SubLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((k_build_d_sub<D, Q>), dim3(unsigned((a.nel + 127) / 128)), dim3(128), 0, st, a);
}

}  // namespace dev

void launch_build_d_sub(int dim, int q, const SubLaunch& a, hipStream_t st) {
  if (a.nel <= 0) return;
  switch (dim * 100 + q) {
    case 200: dev::sub_t<2, 0>(a, st); break;
    case 202: dev::sub_t<2, 2>(a, st); break;
    case 204: dev::sub_t<2, 4>(a, st); break;
    case 206: dev::sub_t<2, 6>(a, st); break;
    case 208: dev::sub_t<2, 8>(a, st); break;
    case 300: dev::sub_t<3, 0>(a, st); break;
    case 302: dev::sub_t<3, 2>(a, st); break;
    case 304: dev::sub_t<3, 4>(a, st); break;
    case 306: dev::sub_t<3, 6>(a, st); break;
    default: throw Error(DOGIP_E_RANGE, "no sub-cell quadrature kernel for this double-grid order");
  }
}

}  // namespace dogip
