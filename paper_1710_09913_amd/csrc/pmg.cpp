// p-multigrid preconditioned flexible CG.
//
// The paper leaves the solver open and names multigrid that fits the DoGIP structure as
// future work (Section 4).  Here: the operator's order k is coarsened on the same mesh,
// P_k -> P_{k-1} -> ... -> P_1, each level a DoGIP operator rebuilt from the fine
// operator's coefficient.  The prolongation from P_{j-1} to P_j is the embedding of the
// coarse space: a fine dof takes the coarse function's value at its node, evaluated in
// one cell holding it (all agree, the functions being continuous); the restriction is its
// transpose.  A V-cycle smooths with Chebyshev polynomials in D^-1 A (degree 3 on
// [lmax/8, 1.1 lmax], lmax by power iteration) before and after the coarse correction,
// and solves a large coarsest level by Jacobi-PCG to a relative residual of 0.1.  That
// inner solve makes the preconditioner vary between applications, hence the flexible
// CG outside: each new direction is made A-orthogonal to the previous one,
// beta = -(z_{k+1} . A p_k) / (p_k . A p_k), which stays right when the preconditioner
// changes from one application to the next (r_{k+1} . z_k, the form that assumes a fixed
// symmetric preconditioner, does not).
//
// On a unit-cube mesh of Kuhn simplices (n^d cubes) the halved mesh is nested in it: each
// coarse simplex is the union of 2^d fine ones, and every fine vertex is a coarse vertex or
// the midpoint of a coarse edge.  There the hierarchy continues below P_1 with P_1 on the
// meshes n/2, n/4, ... for the elliptic problem (degree-4 smoothing on [lmax/20, 1.1 lmax])
// until the coarsest has at most 400 interior dofs: the coefficient of a coarse cell is
// the mean over its children (of the logarithm for a log-coefficient; for inclusions the
// geometric mean of a at points of the cell), and the prolongation is P_1 interpolation (a midpoint
// takes the mean of the edge's ends).  A coarsest level that small is solved exactly by
// its dense inverse.
//
// The transfer weights are a few constants, so a transfer entry is stored as its column
// and the index of its weight in a small table.  In the FP32 mode the finest level's
// smoother keeps its residual and direction in FP32 vectors.
#include "pmg.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <set>
#include <utility>

#include "solve.hpp"

namespace dogip {

namespace {

// Chebyshev smoothing: degree and range for the order levels and for the geometric ones
// (tuned on 3D 64^3 P3 with the lognormal coefficient)
constexpr int CHEB_DEGREE = 3;
constexpr double CHEB_RANGE = 8.0;
constexpr int CHEB_DEGREE_H = 4;
constexpr double CHEB_RANGE_H = 20.0;
// geometric coarsening continues while the coarsest level has more interior dofs than
// DENSE_TARGET; a coarsest level with at most DENSE_MAX interior dofs is solved with its
// dense inverse (Cholesky on the host at set-up), a larger one by Jacobi-PCG
constexpr int64_t DENSE_TARGET = 400;
constexpr int64_t DENSE_MAX = 1000;

// Host arrays of the transfers that are written in full after allocation: default-initialised
// elements (no zeroing).  Zeroing the ~1.2 GB of them at 3D 64^3 P3 on one thread, only to
// overwrite every element from host threads, took about a fifth of the set-up.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <class T>
using RawVec = std::vector<T, NoInit<T>>;
constexpr double COARSE_TOL = 0.1;
constexpr int COARSE_MAXIT = 400;
constexpr int POWER_ITERS = 15;
constexpr int MAX_RESTARTS = 3;

struct Dots {
  double* part;
  double* out;
};

double dot(Dots& d, const double* a, const double* b, int64_t n, hipStream_t st) {
  vk_dot(a, b, n, d.part, d.out, st);
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, d.out, sizeof v, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return v;
}

void copy(double* dst, const double* src, int64_t n, hipStream_t st) {
  if (n > 0) HIPCHK(hipMemcpyAsync(dst, src, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
}

// the prolongation's CSR (fine rows) and its transpose (coarse rows), uploaded to level C
template <class RowV, class ColV, class ValV>
void set_transfer(PmgLevel& C, int64_t nfine, int64_t ncoarse, const RowV& prow, const ColV& pcol,
                  const ValV& pval) {
  // transpose, entries of a coarse row in ascending fine row: the fine rows are cut into nr
  // ranges, each range counts its entries per coarse row, the counts become offsets (coarse
  // row major, range minor) and each range fills its entries in order, on host threads
  const int64_t nr = 8, fchunk = (nfine + nr - 1) / nr;
  std::vector<RawVec<int64_t>> cnt(static_cast<size_t>(nr));
  parallel_tasks(nr, [&](int64_t t) {
    auto& k = cnt[size_t(t)];
    k.resize(size_t(ncoarse));
    std::fill(k.begin(), k.end(), int64_t(0));
    for (int64_t f = t * fchunk; f < std::min(nfine, (t + 1) * fchunk); ++f)
      for (int64_t j = prow[f]; j < prow[f + 1]; ++j) k[size_t(pcol[j])]++;
  });
  std::vector<int64_t> rrow(ncoarse + 1, 0);
  parallel_for(ncoarse, [&](int64_t c) {
    int64_t tot = 0;
    for (int64_t t = 0; t < nr; ++t) tot += cnt[size_t(t)][size_t(c)];
    rrow[c + 1] = tot;
  });
  for (int64_t i = 0; i < ncoarse; ++i) rrow[i + 1] += rrow[i];
  parallel_for(ncoarse, [&](int64_t c) {
    int64_t at = rrow[c];
    for (int64_t t = 0; t < nr; ++t) {
      const int64_t n = cnt[size_t(t)][size_t(c)];
      cnt[size_t(t)][size_t(c)] = at;
      at += n;
    }
  });
  RawVec<int32_t> rcol(pcol.size());
  RawVec<double> rval(pcol.size());
  parallel_tasks(nr, [&](int64_t t) {
    auto& fill = cnt[size_t(t)];
    for (int64_t f = t * fchunk; f < std::min(nfine, (t + 1) * fchunk); ++f)
      for (int64_t j = prow[f]; j < prow[f + 1]; ++j) {
        const int64_t at = fill[size_t(pcol[j])]++;
        rcol[size_t(at)] = int32_t(f);
        rval[size_t(at)] = pval[size_t(j)];
      }
  });
  cnt.clear();
  auto up = [](DevBuf& b, const auto& v) {
    using T = typename std::decay_t<decltype(v)>::value_type;
    b.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  };
  up(C.prow, prow);
  up(C.rrow, rrow);
  // value table, keyed by bit pattern so that packing changes no value; a value's index is
  // its rank among the distinct bit patterns
  auto bits = [](double v) {
    uint64_t k;
    std::memcpy(&k, &v, sizeof k);
    return k;
  };
  // distinct values per chunk on host threads (a sorted list that stops past 256), merged
  const int64_t nval = int64_t(pval.size()), nt = 16, chunk = (nval + nt - 1) / nt;
  std::vector<std::vector<uint64_t>> part(nt);
  parallel_tasks(nt, [&](int64_t t) {
    auto& u = part[size_t(t)];
    for (int64_t j = t * chunk; j < std::min(nval, (t + 1) * chunk) && u.size() <= 256; ++j) {
      const uint64_t k = bits(pval[size_t(j)]);
      const auto at = std::lower_bound(u.begin(), u.end(), k);
      if (at == u.end() || *at != k) u.insert(at, k);
    }
  });
  std::set<uint64_t> seen;
  for (const auto& u : part) seen.insert(u.begin(), u.end());
  C.packed = seen.size() <= 256 && nfine < (int64_t(1) << 24) && ncoarse < (int64_t(1) << 24);
  if (C.packed) {
    const std::vector<uint64_t> keys(seen.begin(), seen.end());
    std::vector<double> tab(256, 0.0);
    for (size_t c = 0; c < keys.size(); ++c) std::memcpy(&tab[c], &keys[c], sizeof(double));
    auto pack = [&](const auto& col, const auto& val) {
      RawVec<uint32_t> e(col.size());
      parallel_for(int64_t(col.size()), [&](int64_t j) {
        const auto at = std::lower_bound(keys.begin(), keys.end(), bits(val[size_t(j)])) - keys.begin();
        e[size_t(j)] = uint32_t(col[size_t(j)]) | (uint32_t(at) << 24);
      });
      return e;
    };
    up(C.ppk, pack(pcol, pval));
    up(C.rpk, pack(rcol, rval));
    up(C.ptab, tab);
  } else {
    up(C.pcol, pcol);
    up(C.pval, pval);
    up(C.rcol, rcol);
    up(C.rval, rval);
  }
  C.nfine = nfine;
  C.nnz = int64_t(pcol.size());
}

// order levels: P_{k-1} embedded in P_k on the same mesh
void build_transfer(const Space& F, const Space& Cs, PmgLevel& C) {
  const int d = F.dim, vf = F.vt, vc = Cs.vt;
  std::vector<double> tab;
  coarse_basis_at_nodes(d, F.k, tab);
  // each fine dof's row comes from its first cell node in cell order (the smallest
  // c * vf + l holding it); cells are scanned in parallel with an atomic minimum
  std::unique_ptr<std::atomic<int64_t>[]> first(new std::atomic<int64_t>[size_t(F.ndofs)]);
  parallel_for(F.ndofs, [&](int64_t f) { first[size_t(f)].store(INT64_MAX, std::memory_order_relaxed); });
  parallel_for(F.nc, [&](int64_t c) {
    for (int l = 0; l < vf; ++l) {
      const int64_t v = c * vf + l;
      std::atomic<int64_t>& a = first[size_t(F.cell_dofs[c * vf + l])];
      int64_t cur = a.load(std::memory_order_relaxed);
      while (v < cur && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
      }
    }
  });
  std::vector<int> nnz_l(size_t(vf), 0);
  for (int l = 0; l < vf; ++l)
    for (int cc = 0; cc < vc; ++cc) nnz_l[size_t(l)] += tab[size_t(l) * vc + cc] != 0.0 ? 1 : 0;
  RawVec<int64_t> prow(size_t(F.ndofs) + 1);
  prow[0] = 0;
  for (int64_t f = 0; f < F.ndofs; ++f) {
    const int64_t v = first[size_t(f)].load(std::memory_order_relaxed);
    DOGIP_CHECK(v != INT64_MAX, DOGIP_E_INVALID, "dof held by no cell");
    prow[f + 1] = prow[f] + nnz_l[size_t(v % vf)];
  }
  const size_t nnz = static_cast<size_t>(prow[F.ndofs]);
  RawVec<int32_t> pcol(nnz);
  RawVec<double> pval(nnz);
  parallel_for(F.ndofs, [&](int64_t f) {
    const int64_t v = first[size_t(f)].load(std::memory_order_relaxed);
    const int64_t c = v / vf;
    const int l = int(v % vf);
    int64_t at = prow[f];
    for (int cc = 0; cc < vc; ++cc) {
      const double w = tab[size_t(l) * vc + cc];
      if (w == 0.0) continue;
      pcol[size_t(at)] = Cs.cell_dofs[c * vc + cc];
      pval[size_t(at++)] = w;
    }
  });
  set_transfer(C, F.ndofs, Cs.ndofs, prow, pcol, pval);
}

// geometric levels: P_1 on the unit mesh nf/2 interpolated on the unit mesh nf (both
// spaces P_1, dofs located by their lattice coordinates)
void build_h_transfer(const Space& F, const Space& Cs, int nf, PmgLevel& C) {
  const int d = F.dim, nc = nf / 2;
  const int64_t m = nc + 1;
  std::vector<int32_t> at(size_t(d == 2 ? m * m : m * m * m), -1);
  for (int64_t i = 0; i < Cs.ndofs; ++i) {
    int64_t key = 0;
    for (int x = d - 1; x >= 0; --x) key = key * m + std::llround(Cs.dof_xyz[i * d + x] * nc);
    DOGIP_CHECK(key >= 0 && key < int64_t(at.size()), DOGIP_E_INVALID, "coarse vertex off the lattice");
    at[size_t(key)] = int32_t(i);
  }
  std::vector<int64_t> prow(F.ndofs + 1, 0);
  std::vector<int32_t> pcol;
  std::vector<double> pval;
  pcol.reserve(size_t(F.ndofs) * 2);
  pval.reserve(size_t(F.ndofs) * 2);
  for (int64_t f = 0; f < F.ndofs; ++f) {
    int64_t I[3] = {0, 0, 0}, off[3] = {0, 0, 0};
    int nodd = 0;
    for (int x = 0; x < d; ++x) {
      I[x] = std::llround(F.dof_xyz[f * d + x] * nf);
      off[x] = I[x] & 1;
      nodd += int(off[x]);
    }
    // a vertex of the coarse mesh, or the midpoint of the coarse edge from (I - off) / 2
    // to (I + off) / 2 (Kuhn edges run in the + direction of every axis they span)
    auto coarse = [&](int sgn) {
      int64_t key = 0;
      for (int x = d - 1; x >= 0; --x) key = key * m + (I[x] + sgn * off[x]) / 2;
      const int32_t c = at[size_t(key)];
      DOGIP_CHECK(c >= 0, DOGIP_E_INVALID, "fine vertex without coarse neighbours");
      return c;
    };
    if (nodd == 0) {
      pcol.push_back(coarse(0));
      pval.push_back(1.0);
    } else {
      pcol.push_back(coarse(-1));
      pval.push_back(0.5);
      pcol.push_back(coarse(1));
      pval.push_back(0.5);
    }
    prow[f + 1] = int64_t(pcol.size());
  }
  set_transfer(C, F.ndofs, Cs.ndofs, prow, pcol, pval);
}

// for each cell of the unit mesh nf, the cell of the unit mesh nf/2 holding it: the coarse
// cube of its centroid, and the Kuhn simplex of that cube given by the descending order of
// the centroid's coordinates inside it (the cell order of make_unit_mesh)
std::vector<int32_t> parent_cells(const Mesh& mf, int nf) {
  const int d = mf.dim, d1 = d + 1, nc = nf / 2;
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<int32_t> par(size_t(mf.nc));
  for (int64_t c = 0; c < mf.nc; ++c) {
    double g[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < d1; ++j)
      for (int x = 0; x < d; ++x) g[x] += mf.xyz[int64_t(mf.cells[c * d1 + j]) * d + x] / d1;
    int64_t ci[3] = {0, 0, 0};
    double xi[3] = {0.0, 0.0, 0.0};
    for (int x = 0; x < d; ++x) {
      const double t = g[x] * nc;
      ci[x] = std::min<int64_t>(std::max<int64_t>(int64_t(std::floor(t)), 0), nc - 1);
      xi[x] = t - double(ci[x]);
    }
    int sub = -1;
    if (d == 2) {
      sub = xi[0] >= xi[1] ? 0 : 1;
      par[c] = int32_t((ci[1] * nc + ci[0]) * 2 + sub);
    } else {
      for (int p = 0; p < 6 && sub < 0; ++p)
        if (xi[perms[p][0]] >= xi[perms[p][1]] && xi[perms[p][1]] >= xi[perms[p][2]]) sub = p;
      par[c] = int32_t(((ci[2] * nc + ci[1]) * nc + ci[0]) * 6 + sub);
    }
  }
  return par;
}

// the mean of each coarse cell's children (per values per cell)
std::vector<double> restrict_coef(const std::vector<double>& cf, const std::vector<int32_t>& par, int per,
                                  int64_t ncoarse) {
  std::vector<double> out(size_t(ncoarse) * per, 0.0);
  std::vector<int32_t> cnt(size_t(ncoarse), 0);
  for (size_t c = 0; c < par.size(); ++c) {
    cnt[size_t(par[c])]++;
    for (int v = 0; v < per; ++v) out[size_t(par[c]) * per + v] += cf[c * per + v];
  }
  for (int64_t c = 0; c < ncoarse; ++c) {
    DOGIP_CHECK(cnt[size_t(c)] > 0, DOGIP_E_INVALID, "coarse cell without children");
    for (int v = 0; v < per; ++v) out[size_t(c) * per + v] /= cnt[size_t(c)];
  }
  return out;
}

void upload(DevBuf& b, const std::vector<double>& v) {
  b.alloc(std::max<size_t>(v.size(), 1) * sizeof(double));
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
}

double power_lmax(Op& op, PmgLevel& L, Dots& dd, hipStream_t st) {
  const int64_t n = L.n;
  double* v = L.d.as<double>();
  double* t = L.t.as<double>();
  const double* invd = op.invdiag.as<double>();
  vk_hash_fill(v, n, st);
  double nrm = std::sqrt(dot(dd, v, v, n, st));
  double lam = 1.0;
  for (int it = 0; it <= POWER_ITERS; ++it) {
    vk_axpby(0.0, v, 1.0 / nrm, v, n, st);  // normalize
    op_apply(op, v, t, DOGIP_F64, st);
    vk_cheb_init(t, invd, v, 1.0, n, st);  // v = D^-1 A v
    nrm = std::sqrt(dot(dd, v, v, n, st));
    DOGIP_CHECK(std::isfinite(nrm) && nrm > 0.0, DOGIP_E_NONFINITE, "power iteration failed");
    lam = nrm;
  }
  return lam;
}

// D of a coarser level from the fine operator's coefficient (or inclusions)
void level_d(const Op& op, Op& lop, hipStream_t st) {
  if (op.inc_depth >= 0) {
    // the same inclusions, integrated by the same sub-cell rule for this level's W
    op_set_inclusions(lop, int(op.inc_balls.size() / size_t(op.space->dim + 1)), op.inc_balls.data(), op.inc_in,
                      op.inc_out, op.inc_depth, op.inc_ng, nullptr, st);
  } else {
    op_set_coef(lop, op.coef_kind_copy, op.coef_copy.as<double>(), st);
  }
}

int coef_per_cell(const Op& op) { return op.coef_kind_copy == DOGIP_COEF_SYM ? op.space->nsym : 1; }

// the fine operator's coefficient on the host
std::vector<double> host_coef(const Op& op, hipStream_t st) {
  std::vector<double> cf(size_t(coef_per_cell(op)) * size_t(op.space->nc));
  HIPCHK(hipStreamSynchronize(st));
  if (!cf.empty()) HIPCHK(hipMemcpy(cf.data(), op.coef_copy.p, cf.size() * sizeof(double), hipMemcpyDeviceToHost));
  return cf;
}

// Coefficient of a geometric level's cells for inclusions: the geometric mean of a over
// the order-6 barycentric lattice of each cell (28 points in 2D, 84 in 3D).  Integrating
// the inclusions again (the arithmetic mean) makes a coarse cell that a ball only partly
// covers too stiff; on 3D 64^3 P3 with a = 100 in 64 balls the geometric mean takes 29
// outer iterations against 35, the harmonic mean 43.
std::vector<double> inclusion_mean(const Op& op, const Mesh& m) {
  constexpr int M = 6;
  const int d = m.dim;
  std::vector<std::array<double, 4>> bary;
  for (int i = 0; i <= M; ++i)
    for (int j = 0; i + j <= M; ++j) {
      if (d == 2)
        bary.push_back({double(i) / M, double(j) / M, double(M - i - j) / M, 0.0});
      else
        for (int k = 0; i + j + k <= M; ++k)
          bary.push_back({double(i) / M, double(j) / M, double(k) / M, double(M - i - j - k) / M});
    }
  const size_t nb = op.inc_balls.size() / size_t(d + 1);
  const double lin = std::log(op.inc_in), lout = std::log(op.inc_out);
  std::vector<double> out(size_t(m.nc));
  parallel_for(m.nc, [&](int64_t c) {
    const int32_t* cv = m.cells.data() + size_t(c) * size_t(d + 1);
    double acc = 0.0;
    for (const auto& b : bary) {
      double x[3] = {0.0, 0.0, 0.0};
      for (int v = 0; v <= d; ++v)
        for (int r = 0; r < d; ++r) x[r] += b[size_t(v)] * m.xyz[size_t(cv[v]) * size_t(d) + size_t(r)];
      bool in = false;
      for (size_t q = 0; q < nb && !in; ++q) {
        const double* ball = op.inc_balls.data() + q * size_t(d + 1);
        double r2 = 0.0;
        for (int r = 0; r < d; ++r) r2 += (x[r] - ball[r]) * (x[r] - ball[r]);
        in = r2 < ball[d] * ball[d];
      }
      acc += in ? lin : lout;
    }
    out[size_t(c)] = std::exp(acc / double(bary.size()));
  });
  return out;
}

// D of the geometric levels (P.lv[first..]) from the fine coefficient, restricted level by
// level, or from the inclusions
void h_levels_d(const Op& op, Pmg& P, size_t first, hipStream_t st) {
  if (first >= P.lv.size()) return;
  std::vector<double> cf;
  if (op.inc_depth < 0) cf = host_coef(op, st);
  for (size_t j = first; j < P.lv.size(); ++j) {
    PmgLevel& L = *P.lv[j];
    if (op.inc_depth >= 0) {
      const std::vector<double> cm = inclusion_mean(op, *L.space->mesh);
      DevBuf dc;
      upload(dc, cm);
      op_set_coef(*L.op, DOGIP_COEF_SCALAR, dc.as<double>(), st);
      HIPCHK(hipStreamSynchronize(st));
    } else {
      cf = restrict_coef(cf, L.parent, coef_per_cell(op), L.space->nc);
      DevBuf dc;
      upload(dc, cf);
      op_set_coef(*L.op, op.coef_kind_copy, dc.as<double>(), st);
      HIPCHK(hipStreamSynchronize(st));
    }
  }
}

// geometric levels below P_1 when the mesh is a unit-cube Kuhn mesh
void add_h_levels(Op& op, Pmg& P, hipStream_t st) {
  const Space& s0 = *op.space;
  int n = s0.mesh->unit_n;
  // the projection's (mass) matrix has a condition number bounded in h, so coarser
  // meshes have nothing to correct there (64^2 P3 with inclusions: 62 outer iterations
  // with or without them); the order levels are kept
  if (n <= 0 || s0.kind != DOGIP_SE) return;
  const size_t first = P.lv.size();
  std::shared_ptr<const Mesh> mf = s0.mesh;
  auto interior = [](const Space& s) { return s.ndofs - int64_t(s.boundary.size()); };
  while (n % 2 == 0 && n / 2 >= 2 && interior(*P.lv.back()->op->space) > DENSE_TARGET) {
    std::shared_ptr<const Mesh> mc = make_unit_mesh(s0.dim, n / 2);
    auto sc = make_space(mc, 1, s0.kind, s0.bc);
    auto L = std::make_unique<PmgLevel>();
    L->hlevel = true;
    L->parent = parent_cells(*mf, n);
    // created with a = 1; h_levels_d sets the coefficient below
    DevBuf ones(size_t(std::max<int64_t>(mc->nc, 1)) * sizeof(double));
    vk_fill(ones.as<double>(), 1.0, mc->nc, st);
    L->own = make_op(sc, DOGIP_COEF_SCALAR, ones.as<double>(), op.has32 ? DOGIP_OP_FP32 : 0u, 0, DOGIP_VARIANT_AUTO,
                     st);
    HIPCHK(hipStreamSynchronize(st));
    build_h_transfer(*P.lv.back()->op->space, *sc, n, *L);
    L->space = sc;
    L->op = L->own.get();
    L->n = sc->ndofs;
    L->range = CHEB_RANGE_H;
    P.lv.push_back(std::move(L));
    mf = mc;
    n /= 2;
  }
  h_levels_d(op, P, first, st);
}

// the coarsest level's A on its interior dofs, column by column (A e_j), factored
// A = L L^T on the host and inverted; leaves nint = 0 (Jacobi-PCG instead) when the level
// is too large or the factorization meets a non-positive pivot
void build_dense(PmgLevel& L, hipStream_t st) {
  L.nint = 0;
  const Space& s = *L.op->space;
  std::vector<uint8_t> isb(size_t(s.ndofs), 0);
  for (int32_t b : s.boundary) isb[size_t(b)] = 1;
  std::vector<int32_t> idx;
  for (int64_t i = 0; i < s.ndofs; ++i)
    if (!isb[size_t(i)]) idx.push_back(int32_t(i));
  const int64_t m = int64_t(idx.size());
  if (m == 0 || m > DENSE_MAX) return;
  // columns by probing: dofs of one colour share no cell neighbour (distance-2 colouring
  // of the cell graph), so A applied to the sum of their unit vectors gives each column on
  // its own rows (the dofs sharing a cell with it)
  const int vt = s.vt;
  std::vector<std::vector<int64_t>> cells_of(size_t(s.ndofs));
  for (int64_t c = 0; c < s.nc; ++c)
    for (int l = 0; l < vt; ++l) cells_of[size_t(s.cell_dofs[c * vt + l])].push_back(c);
  std::vector<int32_t> colour(size_t(s.ndofs), -1), pos(size_t(s.ndofs), -1);
  for (int64_t i = 0; i < m; ++i) pos[size_t(idx[size_t(i)])] = int32_t(i);
  std::vector<int32_t> stamp;
  int ncol = 0;
  for (int64_t j = 0; j < m; ++j) {
    const int32_t dj = idx[size_t(j)];
    // colours taken by the dofs within distance 2 (sharing a cell with a neighbour)
    std::vector<int32_t> nb;
    for (int64_t c : cells_of[size_t(dj)])
      for (int l = 0; l < vt; ++l) nb.push_back(s.cell_dofs[c * vt + l]);
    stamp.assign(size_t(ncol) + 1, 0);
    for (int32_t a : nb)
      for (int64_t c : cells_of[size_t(a)])
        for (int l = 0; l < vt; ++l) {
          const int32_t o = colour[size_t(s.cell_dofs[c * vt + l])];
          if (o >= 0) stamp[size_t(o)] = 1;
        }
    int k = 0;
    while (k < ncol && stamp[size_t(k)]) ++k;
    colour[size_t(dj)] = k;
    ncol = std::max(ncol, k + 1);
  }
  std::vector<double> A(static_cast<size_t>(m * m), 0.0);
  std::vector<double> col(static_cast<size_t>(s.ndofs));
  std::vector<double> probe(static_cast<size_t>(s.ndofs));
  DevBuf e(size_t(s.ndofs) * sizeof(double)), y(size_t(s.ndofs) * sizeof(double));
  for (int k = 0; k < ncol; ++k) {
    for (int64_t i = 0; i < s.ndofs; ++i) probe[size_t(i)] = colour[size_t(i)] == k ? 1.0 : 0.0;
    HIPCHK(hipMemcpy(e.p, probe.data(), probe.size() * sizeof(double), hipMemcpyHostToDevice));
    op_apply(*L.op, e.as<double>(), y.as<double>(), DOGIP_F64, st);
    HIPCHK(hipMemcpyAsync(col.data(), y.p, col.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // row i of column j (colour k): the dofs sharing a cell with j
    for (int64_t j = 0; j < m; ++j) {
      const int32_t dj = idx[size_t(j)];
      if (colour[size_t(dj)] != k) continue;
      for (int64_t c : cells_of[size_t(dj)])
        for (int l = 0; l < vt; ++l) {
          const int32_t di = s.cell_dofs[c * vt + l];
          if (pos[size_t(di)] >= 0) A[size_t(int64_t(pos[size_t(di)]) * m + j)] = col[size_t(di)];
        }
    }
  }
  // Cholesky (lower triangle of A overwritten by L) from the symmetric part
  for (int64_t j = 0; j < m; ++j) {
    double d = 0.5 * (A[size_t(j * m + j)] + A[size_t(j * m + j)]);
    for (int64_t k = 0; k < j; ++k) d -= A[size_t(j * m + k)] * A[size_t(j * m + k)];
    if (!(d > 0.0) || !std::isfinite(d)) return;
    const double ljj = std::sqrt(d);
    A[size_t(j * m + j)] = ljj;
    for (int64_t i = j + 1; i < m; ++i) {
      double v = 0.5 * (A[size_t(i * m + j)] + A[size_t(j * m + i)]);
      for (int64_t k = 0; k < j; ++k) v -= A[size_t(i * m + k)] * A[size_t(j * m + k)];
      A[size_t(i * m + j)] = v / ljj;
    }
  }
  // inverse column by column: L z = e_c, L^T x = z
  std::vector<double> inv(static_cast<size_t>(m * m));
  std::vector<double> z(static_cast<size_t>(m));
  for (int64_t c = 0; c < m; ++c) {
    for (int64_t i = 0; i < m; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int64_t k = c; k < i; ++k) v -= A[size_t(i * m + k)] * z[size_t(k)];
      z[size_t(i)] = i < c ? 0.0 : v / A[size_t(i * m + i)];
    }
    for (int64_t i = m - 1; i >= 0; --i) {
      double v = z[size_t(i)];
      for (int64_t k = i + 1; k < m; ++k) v -= A[size_t(k * m + i)] * inv[size_t(k * m + c)];
      inv[size_t(i * m + c)] = v / A[size_t(i * m + i)];
    }
  }
  upload(L.dinv, inv);
  L.didx.alloc(size_t(m) * sizeof(int32_t));
  HIPCHK(hipMemcpy(L.didx.p, idx.data(), size_t(m) * sizeof(int32_t), hipMemcpyHostToDevice));
  L.nint = m;
}

void check_source(const Op& op) {
  DOGIP_CHECK((op.coef_kind_copy >= 0 || op.inc_depth >= 0) && !op.global_w && op.nq == 0, DOGIP_E_STATE,
              "the multigrid solve needs an element-wise operator built from a coefficient form or inclusions");
}

void build(Op& op, hipStream_t st) {
  const Space& s0 = *op.space;
  check_source(op);
  DevBuf ones(size_t(std::max<int64_t>(s0.nc, 1)) * sizeof(double));
  vk_fill(ones.as<double>(), 1.0, s0.nc, st);
  auto P = std::make_unique<Pmg>();
  for (int j = 0; j < s0.k; ++j) P->lv.push_back(std::make_unique<PmgLevel>());
  P->lv[0]->op = &op;
  P->lv[0]->n = s0.ndofs;
  for (int j = 1; j < s0.k; ++j) {
    auto sp = make_space(s0.mesh, s0.k - j, s0.kind, s0.bc);
    PmgLevel& L = *P->lv[size_t(j)];
    const unsigned fl = op.has32 ? DOGIP_OP_FP32 : 0u;
    if (op.inc_depth >= 0) {
      L.own = make_op(sp, DOGIP_COEF_SCALAR, ones.as<double>(), fl, 0, DOGIP_VARIANT_AUTO, st);
      level_d(op, *L.own, st);
    } else {
      L.own = make_op(sp, op.coef_kind_copy, op.coef_copy.as<double>(), fl, 0, DOGIP_VARIANT_AUTO, st);
    }
    L.space = sp;
    L.op = L.own.get();
    L.n = sp->ndofs;
  }
  for (size_t j = 0; j + 1 < P->lv.size(); ++j)
    build_transfer(*P->lv[j]->op->space, *P->lv[j + 1]->op->space, *P->lv[j + 1]);
  for (auto& L : P->lv) L->range = CHEB_RANGE;
  add_h_levels(op, *P, st);
  for (auto& Lp : P->lv) {
    PmgLevel& L = *Lp;
    const size_t vb = std::max<int64_t>(L.n, 1) * sizeof(double);
    if (Lp != P->lv.front()) {
      L.x.alloc(vb);
      L.b.alloc(vb);
    }
    L.r.alloc(vb);
    L.d.alloc(vb);
    L.t.alloc(vb);
  }
  const size_t vb = std::max<int64_t>(s0.ndofs, 1) * sizeof(double);
  P->r.alloc(vb);
  P->z.alloc(vb);
  P->p.alloc(vb);
  P->q.alloc(vb);
  P->dots.alloc(size_t(RED_BLOCKS + 8) * sizeof(double));
  P->fcg.alloc(8 * sizeof(double));
  if (op_has_v32(op)) P->e32.alloc(size_t(op.plan.ntiles + op_finish_energy_count(op)) * sizeof(double));
  Dots dd{P->dots.as<double>(), P->dots.as<double>() + RED_BLOCKS};
  for (auto& L : P->lv) L->lmax = power_lmax(*L->op, *L, dd, st);
  build_dense(*P->lv.back(), st);
  op.pmg = std::move(P);
}

// after a coefficient change: each level's D, diagonal and lmax again; the spaces, tiles
// and transfers stay
void refresh(Op& op, hipStream_t st) {
  check_source(op);
  Pmg& P = *op.pmg;
  size_t first_h = P.lv.size();
  for (size_t j = 1; j < P.lv.size(); ++j) {
    if (P.lv[j]->hlevel) {
      first_h = j;
      break;
    }
    level_d(op, *P.lv[j]->op, st);
  }
  h_levels_d(op, P, first_h, st);
  Dots dd{P.dots.as<double>(), P.dots.as<double>() + RED_BLOCKS};
  for (auto& L : P.lv) L->lmax = power_lmax(*L->op, *L, dd, st);
  build_dense(*P.lv.back(), st);
  P.stale = false;
}

// Chebyshev smoothing of A x = b at level L (from x = 0 when first).  On return r holds
// the recursively updated residual b - A x (each step subtracts A d as it adds d to x).
void smooth(PmgLevel& L, double* x, const double* b, int prec, bool first, hipStream_t st) {
  Op& A = *L.op;
  const int64_t n = L.n;
  double *r = L.r.as<double>(), *d = L.d.as<double>(), *t = L.t.as<double>();
  const double* invd = A.invdiag.as<double>();
  const bool stream = stream_vectors(n, 40, int64_t(A.lidx.bytes + A.tile_dofs.bytes));  // x, r, d, t, D^-1
  const double hi = 1.1 * L.lmax, lo = L.lmax / L.range;
  const int degree = L.hlevel ? CHEB_DEGREE_H : CHEB_DEGREE;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  if (first) {
    vk_fill(x, 0.0, n, st);
    copy(r, b, n, st);
  } else {
    op_apply(A, x, t, prec, st);
    vk_sub(b, t, r, n, st);
  }
  vk_cheb_init(r, invd, d, 1.0 / theta, n, st);
  double rho = 1.0 / sigma;
  for (int i = 0; i < degree; ++i) {
    op_apply(A, d, t, prec, st);
    const double rn = 1.0 / (2.0 * sigma - rho);
    vk_cheb_step(x, r, d, t, invd, rn * rho, 2.0 * rn / delta, n, stream, st);
    rho = rn;
  }
}

// smooth() for the FP32 mode on the finest level: r, d and A d are stored in FP32 (in the
// first half of the level's FP64 work vectors) and A d comes from the FP32-vector apply,
// which halves the vector traffic of the smoothing steps; x, b and the arithmetic of the
// updates stay FP64
void smooth32(PmgLevel& L, double* x, const double* b, bool first, double* energy, hipStream_t st) {
  Op& A = *L.op;
  const int64_t n = L.n;
  float *r = L.r.as<float>(), *d = L.d.as<float>(), *t = L.t.as<float>();
  const double* invd = A.invdiag.as<double>();
  const bool stream = stream_vectors(n, 28, int64_t(A.lidx.bytes + A.tile_dofs.bytes));  // x, D^-1 FP64; r, d, t
  const double hi = 1.1 * L.lmax, lo = L.lmax / L.range;
  const int degree = L.hlevel ? CHEB_DEGREE_H : CHEB_DEGREE;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  if (first) {
    vk_fill(x, 0.0, n, st);
    launch_to_f32(b, r, n, st);
  } else {
    // the FP64 t is read before the FP32 t (its first half) is written
    op_apply(A, x, L.t.as<double>(), DOGIP_F32, st);
    vk_sub_to32(b, L.t.as<double>(), r, n, st);
  }
  vk_cheb_init32(r, invd, d, 1.0 / theta, n, st);
  double rho = 1.0 / sigma;
  for (int i = 0; i < degree; ++i) {
    op_apply_v32(A, d, t, st, energy);
    const double rn = 1.0 / (2.0 * sigma - rho);
    vk_cheb_step32(x, r, d, t, invd, rn * rho, 2.0 * rn / delta, n, stream, st);
    rho = rn;
  }
}

// x ~= A^-1 b at level j
void vcycle(Pmg& P, size_t j, const double* b, double* x, int prec, hipStream_t st) {
  PmgLevel& L = *P.lv[j];
  Op& A = *L.op;
  const int64_t n = L.n;
  if (j + 1 == P.lv.size()) {
    vk_fill(x, 0.0, n, st);
    if (L.nint > 0) {
      // exact: A^-1 on the interior, identity rows on the Dirichlet boundary
      vk_dense_solve(L.dinv.as<double>(), L.didx.as<int32_t>(), L.nint, b, x, st);
      vk_copy_indexed(x, b, A.bnd.as<int32_t>(), int64_t(A.space->boundary.size()), st);
    } else {
      cg_inner(A, b, x, P.coarse_tol, COARSE_MAXIT, prec, st);
    }
    return;
  }
  const bool v32 = j == 0 && prec == DOGIP_F32 && P.e32.bytes > 0;
  if (v32)
    smooth32(L, x, b, true, P.e32.as<double>(), st);
  else
    smooth(L, x, b, prec, true, st);
  // restrict the residual the smoother leaves in r; zero the coarse Dirichlet rows
  PmgLevel& C = *P.lv[j + 1];
  if (C.packed && v32)
    vk_csr_pk_x32(C.rrow.as<int64_t>(), C.rpk.as<uint32_t>(), C.ptab.as<double>(), L.r.as<float>(), C.b.as<double>(),
                  C.n, C.nnz, st);
  else if (C.packed)
    vk_csr_pk(C.rrow.as<int64_t>(), C.rpk.as<uint32_t>(), C.ptab.as<double>(), L.r.as<double>(), C.b.as<double>(),
              C.n, C.nnz, false, st);
  else if (v32)
    vk_csr_x32(C.rrow.as<int64_t>(), C.rcol.as<int32_t>(), C.rval.as<double>(), L.r.as<float>(), C.b.as<double>(),
               C.n, C.nnz, st);
  else
    vk_csr(C.rrow.as<int64_t>(), C.rcol.as<int32_t>(), C.rval.as<double>(), L.r.as<double>(), C.b.as<double>(), C.n,
           C.nnz, false, st);
  launch_zero_indexed(C.b.as<double>(), C.op->bnd.as<int32_t>(), int64_t(C.op->space->boundary.size()), st);
  vcycle(P, j + 1, C.b.as<double>(), C.x.as<double>(), prec, st);
  // x += P x_c
  if (C.packed)
    vk_csr_pk(C.prow.as<int64_t>(), C.ppk.as<uint32_t>(), C.ptab.as<double>(), C.x.as<double>(), x, n, C.nnz, true,
              st);
  else
    vk_csr(C.prow.as<int64_t>(), C.pcol.as<int32_t>(), C.pval.as<double>(), C.x.as<double>(), x, n, C.nnz, true, st);
  if (v32)
    smooth32(L, x, b, false, P.e32.as<double>(), st);
  else
    smooth(L, x, b, prec, false, st);
}

}  // namespace

int op_pcg_pmg(Op& op, const double* b, double* x, const dogip_solve_opts& o, dogip_solve_stats& stats, int prec,
               hipStream_t st) {
  if (!op.pmg)
    build(op, st);
  else if (op.pmg->stale)
    refresh(op, st);
  Pmg& P = *op.pmg;
  P.coarse_tol = (o.inner_tol > 0.0 && o.inner_tol < 1.0) ? o.inner_tol : COARSE_TOL;
  const int64_t n = op.space->ndofs;
  Dots dd{P.dots.as<double>(), P.dots.as<double>() + RED_BLOCKS};
  double *r = P.r.as<double>(), *p = P.p.as<double>(), *q = P.q.as<double>();
  double* z = P.z.as<double>();
  const double bb = dot(dd, b, b, n, st);
  if (!std::isfinite(bb)) return DOGIP_E_NONFINITE;
  if (bb == 0.0) {
    vk_fill(x, 0.0, n, st);
    stats.relres = 0.0;
    return DOGIP_OK;
  }
  const double thr = o.tol * o.tol * bb;
  if (o.x0_given) {
    op_apply(op, x, q, DOGIP_F64, st);
    vk_sub(b, q, r, n, st);
  } else {
    vk_fill(x, 0.0, n, st);
    copy(r, b, n, st);
  }
  int it = 0, restarts = 0, status = DOGIP_E_NOT_CONVERGED;
  double rr = dot(dd, r, r, n, st);
  stats.relres = std::sqrt(rr / bb);
  if (rr <= thr) return DOGIP_OK;
  // the iteration keeps its scalars on the device (one host synchronization per
  // iteration, for r.r and the flag)
  double* S = P.fcg.as<double>();
  vk_fill(S, 0.0, 8, st);
  vcycle(P, 0, r, z, prec, st);
  copy(p, z, n, st);
  vk_dot(r, z, n, dd.part, S + 0, st);
  while (it < o.maxit) {
    op_apply(op, p, q, DOGIP_F64, st);
    vk_dot(p, q, n, dd.part, S + 1, st);
    vk_fcg_alpha(S, st);
    vk_axpy_s(x, p, S, 2, 1.0, n, st);
    vk_axpy_s(r, q, S, 2, -1.0, n, st);
    vk_dot(r, r, n, dd.part, S + 3, st);
    double h[8];
    HIPCHK(hipMemcpyAsync(h, S, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h[7] != 0.0) {
      status = h[7] == 1.0 ? DOGIP_E_BREAKDOWN : DOGIP_E_NONFINITE;
      break;
    }
    ++it;
    rr = h[3];
    stats.relres = std::sqrt(rr / bb);
    if (!std::isfinite(rr)) {
      status = DOGIP_E_NONFINITE;
      break;
    }
    if (rr <= thr) {
      // verify on the true residual; otherwise continue from it with a fresh direction
      op_apply(op, x, q, DOGIP_F64, st);
      vk_sub(b, q, r, n, st);
      rr = dot(dd, r, r, n, st);
      stats.relres = std::sqrt(rr / bb);
      if (rr <= thr) {
        status = DOGIP_OK;
        break;
      }
      if (++restarts > MAX_RESTARTS) break;
      vcycle(P, 0, r, z, prec, st);
      copy(p, z, n, st);
      vk_dot(r, z, n, dd.part, S + 0, st);
      continue;
    }
    vcycle(P, 0, r, z, prec, st);
    vk_dot(r, z, n, dd.part, S + 4, st);
    vk_dot(z, q, n, dd.part, S + 5, st);  // q still holds A p_k
    vk_fcg_beta(S, st);
    vk_xpby_s(p, z, S, 6, n, st);
  }
  stats.iters = it;
  stats.outer = it + restarts;
  return status;
}

}  // namespace dogip
