// Reference-element tables of the element-wise DoGIP operator, computed in exact
// rational arithmetic (usable at compile time and at run time, host and device).
//
// Reference simplex T^ = conv{0, e_1, ..., e_d} (Section 2.1).  Lagrange nodes of
// P_p are the lattice a/p, |a| <= p, enumerated lexicographically in (a_1..a_d);
// their barycentric multi-index is b = (p - |a|, a_1, ..., a_d).  The nodal basis
// uses the product form over barycentric coordinates
//     phi_b(lambda) = prod_j P^p_{b_j}(lambda_j),  P^p_m(t) = prod_{s<m} (p t - s)/(s + 1),
// which is 1 at its own node and 0 at every other lattice node.
//
// * Weighted projection (Theorem 2): B^[i][l] = phi^V_l(x^W_i), W = C_{N,2k}.
// * Elliptic problem (Theorem 4): B^[r][i][l] = d phi^V_l / d x^_r (x^W_i),
//   W = D_{N,2k-2}, the derivative taken in reference coordinates
//   (d/dx^_r = d/dlambda_r - d/dlambda_0); the inverse Jacobians live in D.
// * w^_i = (1/|T^|) int_T^ phi^W_i, by expanding each factor P^q_m into powers of
//   lambda_j and integrating with  int_T^ prod lambda_j^e_j = d! |T^| prod e_j! / (|e| + d)!.
//   The double-grid order is q = 2k or 2k - 2; q = 0 is a single node at the
//   centroid with weight 1.
#pragma once

#include <stdint.h>

namespace dogip {

enum Kind : int { KIND_WP = 0, KIND_SE = 1 };

constexpr int binom(int n, int r) {
  if (r < 0 || r > n) return 0;
  long long v = 1;
  for (int i = 1; i <= r; ++i) v = v * (n - r + i) / i;
  return (int)v;
}
constexpr int dim_p(int d, int p) { return binom(p + d, d); }
constexpr int w_order(int k, int kind) { return kind == KIND_WP ? 2 * k : 2 * k - 2; }
constexpr int n_sym(int d) { return d * (d + 1) / 2; }

namespace ref {

using i128 = __int128;

constexpr i128 iabs(i128 a) { return a < 0 ? -a : a; }
constexpr i128 igcd(i128 a, i128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b != 0) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Exact rational with positive denominator in lowest terms.
struct Q {
  i128 n = 0, d = 1;
  constexpr Q() = default;
  constexpr Q(i128 num, i128 den = 1) : n(num), d(den) {
    if (d < 0) { n = -n; d = -d; }
    i128 g = igcd(n, d);
    if (g > 1) { n /= g; d /= g; }
    if (n == 0) d = 1;
  }
};
constexpr Q operator+(Q a, Q b) {
  i128 g = igcd(a.d, b.d);
  return Q(a.n * (b.d / g) + b.n * (a.d / g), a.d / g * b.d);
}
constexpr Q operator-(Q a, Q b) { return a + Q(-b.n, b.d); }
constexpr Q operator*(Q a, Q b) {
  i128 g1 = igcd(a.n, b.d), g2 = igcd(b.n, a.d);
  if (g1 == 0) g1 = 1;
  if (g2 == 0) g2 = 1;
  return Q((a.n / g1) * (b.n / g2), (a.d / g2) * (b.d / g1));
}
constexpr bool is_zero(Q a) { return a.n == 0; }
constexpr double to_double(Q a) { return (double)a.n / (double)a.d; }

// Lattice enumeration: the t-th multi-index a in N^d, |a| <= p, lexicographic.
constexpr void lattice_index(int d, int p, int t, int* a) {
  int cnt = 0;
  int x[3] = {0, 0, 0};
  // lexicographic walk
  for (x[0] = 0; x[0] <= p; ++x[0]) {
    if (d == 2) {
      for (x[1] = 0; x[0] + x[1] <= p; ++x[1]) {
        if (cnt == t) { a[0] = x[0]; a[1] = x[1]; return; }
        ++cnt;
      }
    } else {
      for (x[1] = 0; x[0] + x[1] <= p; ++x[1])
        for (x[2] = 0; x[0] + x[1] + x[2] <= p; ++x[2]) {
          if (cnt == t) { a[0] = x[0]; a[1] = x[1]; a[2] = x[2]; return; }
          ++cnt;
        }
    }
  }
}

// Barycentric multi-index b[0..d] of lattice node t of P_p.
constexpr void bary_index(int d, int p, int t, int* b) {
  int a[3] = {0, 0, 0};
  lattice_index(d, p, t, a);
  int s = 0;
  for (int r = 0; r < d; ++r) { b[r + 1] = a[r]; s += a[r]; }
  b[0] = p - s;
}

// Sub-simplex of the reference cell whose relative interior holds lattice node t of
// P_p, as a bit index: 2D vertices 0-2, edges 3-5, interior 6; 3D vertices 0-3,
// edges 4-9, faces 10-13 (face j opposite vertex j), interior 14.  Edges (a, b),
// a < b, are numbered lexicographically.
constexpr int node_entity(int d, int p, int t) {
  int b[4] = {0, 0, 0, 0};
  bary_index(d, p, t, b);
  int sup[4] = {0, 0, 0, 0}, ns = 0, opp = 0;
  for (int j = 0; j <= d; ++j) {
    if (b[j] > 0)
      sup[ns++] = j;
    else
      opp = j;
  }
  if (ns == 1) return sup[0];
  if (ns == 2) {
    int idx = 0;
    for (int i = 0; i < sup[0]; ++i) idx += d - i;
    return d + 1 + idx + (sup[1] - sup[0] - 1);
  }
  if (ns == 3 && d == 3) return 10 + opp;
  return d == 2 ? 6 : 14;
}

// Number of lattice nodes of P_p inside sub-simplex slot e, and the rank of node t
// among the nodes of its slot (lattice order).
constexpr int entity_nodes(int d, int p, int e) {
  int n = 0;
  for (int t = 0; t < dim_p(d, p); ++t) n += node_entity(d, p, t) == e ? 1 : 0;
  return n;
}
constexpr int entity_rank(int d, int p, int t) {
  int r = 0;
  const int e = node_entity(d, p, t);
  for (int s = 0; s < t; ++s) r += node_entity(d, p, s) == e ? 1 : 0;
  return r;
}

// Barycentric coordinates (exact) of W node i for double-grid order q.
constexpr void w_node_bary(int d, int q, int i, Q* lam) {
  if (q == 0) {
    for (int j = 0; j <= d; ++j) lam[j] = Q(1, d + 1);
    return;
  }
  int b[4] = {0, 0, 0, 0};
  bary_index(d, q, i, b);
  for (int j = 0; j <= d; ++j) lam[j] = Q(b[j], q);
}

// P^p_m(t) and its derivative at rational t.
constexpr Q pfac(int p, int m, Q t) {
  Q v(1);
  for (int s = 0; s < m; ++s) v = v * ((Q(p) * t - Q(s)) * Q(1, s + 1));
  return v;
}
constexpr Q pfac_der(int p, int m, Q t) {
  Q tot(0);
  for (int s = 0; s < m; ++s) {
    Q term(p, s + 1);
    for (int s2 = 0; s2 < m; ++s2)
      if (s2 != s) term = term * ((Q(p) * t - Q(s2)) * Q(1, s2 + 1));
    tot = tot + term;
  }
  return tot;
}

// phi^V_l (order k) at barycentric point lam.
constexpr Q basis_value(int d, int k, int l, const Q* lam) {
  int b[4] = {0, 0, 0, 0};
  bary_index(d, k, l, b);
  Q v(1);
  for (int j = 0; j <= d; ++j) v = v * pfac(k, b[j], lam[j]);
  return v;
}

// d phi^V_l / d x^_r (r = 0..d-1) at barycentric point lam.
constexpr Q basis_grad(int d, int k, int l, int r, const Q* lam) {
  int b[4] = {0, 0, 0, 0};
  bary_index(d, k, l, b);
  auto dlam = [&](int jj) {
    Q v = pfac_der(k, b[jj], lam[jj]);
    for (int j = 0; j <= d; ++j)
      if (j != jj) v = v * pfac(k, b[j], lam[j]);
    return v;
  };
  return dlam(r + 1) - dlam(0);
}

// Entry of B^ (kind, order k): index (r, i, l); r ignored for the projection.
constexpr Q bhat_entry(int d, int k, int kind, int r, int i, int l) {
  Q lam[4];
  w_node_bary(d, w_order(k, kind), i, lam);
  return kind == KIND_WP ? basis_value(d, k, l, lam) : basis_grad(d, k, l, r, lam);
}

constexpr i128 fact(int n) {
  i128 v = 1;
  for (int i = 2; i <= n; ++i) v *= i;
  return v;
}

// w^_i for the P_q lattice.
constexpr Q what_entry(int d, int q, int i) {
  if (q == 0) return Q(1);
  int b[4] = {0, 0, 0, 0};
  bary_index(d, q, i, b);
  // power coefficients of each factor P^q_{b_j}(t) = sum_e c[j][e] t^e
  Q c[4][17];
  for (int j = 0; j <= d; ++j) {
    for (int e = 0; e <= 16; ++e) c[j][e] = Q(0);
    c[j][0] = Q(1);
    for (int s = 0; s < b[j]; ++s) {
      // multiply by (q t - s)/(s+1)
      Q nc[17];
      for (int e = 0; e <= 16; ++e) nc[e] = Q(0);
      for (int e = 0; e <= s; ++e) {
        nc[e + 1] = nc[e + 1] + c[j][e] * Q(q, s + 1);
        nc[e] = nc[e] - c[j][e] * Q(s, s + 1);
      }
      for (int e = 0; e <= 16; ++e) c[j][e] = nc[e];
    }
  }
  Q tot(0);
  int e[4] = {0, 0, 0, 0};
  for (e[0] = 0; e[0] <= b[0]; ++e[0])
    for (e[1] = 0; e[1] <= b[1]; ++e[1])
      for (e[2] = 0; e[2] <= b[2]; ++e[2])
        for (e[3] = 0; e[3] <= (d == 3 ? b[3] : 0); ++e[3]) {
          Q coef(1);
          i128 num = fact(d);
          int se = 0;
          for (int j = 0; j <= d; ++j) {
            coef = coef * c[j][e[j]];
            num *= fact(e[j]);
            se += e[j];
          }
          if (!is_zero(coef)) tot = tot + coef * Q(num, fact(se + d));
        }
  return tot;
}

// Table of B^ as doubles, [NB][WT][VT] with NB = d (elliptic) or 1.  The 1D
// factors P^k_m and their derivatives are tabulated once at the W lattice
// abscissae t = b/q (or at the centroid coordinate 1/(d+1) when q = 0), so every
// entry is a product of d+1 table values.
template <int D, int K, int KIND>
struct BTable {
  static constexpr int VT = dim_p(D, K);
  static constexpr int Qo = w_order(K, KIND);
  static constexpr int WT = dim_p(D, Qo);
  static constexpr int NB = KIND == KIND_SE ? D : 1;
  static constexpr int NT = Qo == 0 ? 1 : Qo + 1;
  double v[NB][WT][VT] = {};
  constexpr BTable() {
    Q P[K + 1][NT], PD[K + 1][NT];
    for (int m = 0; m <= K; ++m)
      for (int t = 0; t < NT; ++t) {
        Q x = Qo == 0 ? Q(1, D + 1) : Q(t, Qo);
        P[m][t] = pfac(K, m, x);
        PD[m][t] = pfac_der(K, m, x);
      }
    int bv[VT][4] = {}, bw[WT][4] = {};
    for (int l = 0; l < VT; ++l) bary_index(D, K, l, bv[l]);
    for (int i = 0; i < WT; ++i) {
      if (Qo == 0) {
        for (int j = 0; j <= D; ++j) bw[i][j] = 0;
      } else {
        bary_index(D, Qo, i, bw[i]);
      }
    }
    for (int i = 0; i < WT; ++i)
      for (int l = 0; l < VT; ++l) {
        if (KIND == KIND_WP) {
          Q val(1);
          for (int j = 0; j <= D; ++j) val = val * P[bv[l][j]][bw[i][j]];
          v[0][i][l] = to_double(val);
        } else {
          Q dl[4];
          for (int jj = 0; jj <= D; ++jj) {
            Q val = PD[bv[l][jj]][bw[i][jj]];
            for (int j = 0; j <= D; ++j)
              if (j != jj) val = val * P[bv[l][j]][bw[i][j]];
            dl[jj] = val;
          }
          for (int r = 0; r < D; ++r) v[r][i][l] = to_double(dl[r + 1] - dl[0]);
        }
      }
  }
};

// Factored elliptic B^ (k >= 2): the gradient of u in P_k is a vector field in P_{k-1},
// so B^ = (I_d (x) B2) B1 exactly, with
//   B1[r][j][l] = d phi^V_l / d x^_r at node j of the P_{k-1} lattice, and
//   B2[i][j]    = phi^{k-1}_j (x^W_i), the P_{k-1} Lagrange basis at the W nodes (P_{2k-2}).
// W nodes that are P_{k-1} nodes give unit rows of B2.  At 3D P3 the two factors have 216
// + 3 x 106 nonzeros (against 1014 in B^), at 2D P5 436 + 2 x 255 (against 1516).
template <int D, int K>
struct FTable {
  static constexpr int VT = dim_p(D, K);
  static constexpr int NJ = dim_p(D, K - 1);
  static constexpr int WT = dim_p(D, 2 * K - 2);
  double b1[D][NJ][VT] = {};
  double b2[WT][NJ] = {};
  constexpr FTable() {
    static_assert(K >= 2, "the factored form needs k >= 2");
    for (int j = 0; j < NJ; ++j) {
      Q lam[4];
      int b[4] = {0, 0, 0, 0};
      bary_index(D, K - 1, j, b);
      for (int t = 0; t <= D; ++t) lam[t] = Q(b[t], K - 1);
      for (int l = 0; l < VT; ++l)
        for (int r = 0; r < D; ++r) b1[r][j][l] = to_double(basis_grad(D, K, l, r, lam));
    }
    for (int i = 0; i < WT; ++i) {
      Q lam[4];
      w_node_bary(D, 2 * K - 2, i, lam);
      for (int j = 0; j < NJ; ++j) b2[i][j] = to_double(basis_value(D, K - 1, j, lam));
    }
  }
};

}  // namespace ref
}  // namespace dogip
