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
// and solves the P_1 level by Jacobi-PCG to a relative residual of 0.1.  The inner solve
// makes the preconditioner vary between applications, hence the flexible
// (Polak-Ribiere) CG outside.
#include "pmg.hpp"

#include <cmath>
#include <utility>

#include "solve.hpp"

namespace dogip {

namespace {

constexpr int CHEB_DEGREE = 3;
constexpr double CHEB_RANGE = 8.0;
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

// CSR of the prolongation (fine rows) and of its transpose (coarse rows)
void build_transfer(const Space& F, const Space& Cs, PmgLevel& C) {
  const int d = F.dim, vf = F.vt, vc = Cs.vt;
  std::vector<double> tab;
  coarse_basis_at_nodes(d, F.k, tab);
  std::vector<int64_t> first(F.ndofs, -1);
  for (int64_t c = 0; c < F.nc; ++c)
    for (int l = 0; l < vf; ++l) {
      const int32_t f = F.cell_dofs[c * vf + l];
      if (first[f] < 0) first[f] = c * vf + l;
    }
  std::vector<int64_t> prow(F.ndofs + 1, 0);
  std::vector<int32_t> pcol;
  std::vector<double> pval;
  for (int64_t f = 0; f < F.ndofs; ++f) {
    DOGIP_CHECK(first[f] >= 0, DOGIP_E_INVALID, "dof held by no cell");
    const int64_t c = first[f] / vf;
    const int l = int(first[f] % vf);
    for (int cc = 0; cc < vc; ++cc) {
      const double w = tab[size_t(l) * vc + cc];
      if (w == 0.0) continue;
      pcol.push_back(Cs.cell_dofs[c * vc + cc]);
      pval.push_back(w);
    }
    prow[f + 1] = int64_t(pcol.size());
  }
  // transpose, entries of a coarse row in ascending fine row
  std::vector<int64_t> rrow(Cs.ndofs + 1, 0);
  for (int32_t c : pcol) rrow[c + 1]++;
  for (int64_t i = 0; i < Cs.ndofs; ++i) rrow[i + 1] += rrow[i];
  std::vector<int32_t> rcol(pcol.size());
  std::vector<double> rval(pcol.size());
  std::vector<int64_t> fill(rrow.begin(), rrow.end() - 1);
  for (int64_t f = 0; f < F.ndofs; ++f)
    for (int64_t j = prow[f]; j < prow[f + 1]; ++j) {
      const int64_t at = fill[pcol[j]]++;
      rcol[at] = int32_t(f);
      rval[at] = pval[j];
    }
  auto up = [](DevBuf& b, const auto& v) {
    using T = typename std::decay_t<decltype(v)>::value_type;
    b.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  };
  up(C.prow, prow);
  up(C.pcol, pcol);
  up(C.pval, pval);
  up(C.rrow, rrow);
  up(C.rcol, rcol);
  up(C.rval, rval);
  C.nfine = F.ndofs;
  C.nnz = int64_t(pcol.size());
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
  P->zo.alloc(vb);
  P->p.alloc(vb);
  P->q.alloc(vb);
  P->dots.alloc(size_t(RED_BLOCKS + 8) * sizeof(double));
  Dots dd{P->dots.as<double>(), P->dots.as<double>() + RED_BLOCKS};
  for (auto& L : P->lv) L->lmax = power_lmax(*L->op, *L, dd, st);
  op.pmg = std::move(P);
}

// after a coefficient change: each level's D, diagonal and lmax again; the spaces, tiles
// and transfers stay
void refresh(Op& op, hipStream_t st) {
  check_source(op);
  Pmg& P = *op.pmg;
  for (size_t j = 1; j < P.lv.size(); ++j) level_d(op, *P.lv[j]->op, st);
  Dots dd{P.dots.as<double>(), P.dots.as<double>() + RED_BLOCKS};
  for (auto& L : P.lv) L->lmax = power_lmax(*L->op, *L, dd, st);
  P.stale = false;
}

// Chebyshev smoothing of A x = b at level L (from x = 0 when first).  On return r holds
// the recursively updated residual b - A x (each step subtracts A d as it adds d to x).
void smooth(PmgLevel& L, double* x, const double* b, int prec, bool first, hipStream_t st) {
  Op& A = *L.op;
  const int64_t n = L.n;
  double *r = L.r.as<double>(), *d = L.d.as<double>(), *t = L.t.as<double>();
  const double* invd = A.invdiag.as<double>();
  const double hi = 1.1 * L.lmax, lo = L.lmax / CHEB_RANGE;
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
  for (int i = 0; i < CHEB_DEGREE; ++i) {
    op_apply(A, d, t, prec, st);
    const double rn = 1.0 / (2.0 * sigma - rho);
    vk_cheb_step(x, r, d, t, invd, rn * rho, 2.0 * rn / delta, n, st);
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
    cg_inner(A, b, x, P.coarse_tol, COARSE_MAXIT, prec, st);
    return;
  }
  smooth(L, x, b, prec, true, st);
  // restrict the residual the smoother leaves in r; zero the coarse Dirichlet rows
  PmgLevel& C = *P.lv[j + 1];
  vk_csr(C.rrow.as<int64_t>(), C.rcol.as<int32_t>(), C.rval.as<double>(), L.r.as<double>(), C.b.as<double>(), C.n,
         C.nnz, false, st);
  launch_zero_indexed(C.b.as<double>(), C.op->bnd.as<int32_t>(), int64_t(C.op->space->boundary.size()), st);
  vcycle(P, j + 1, C.b.as<double>(), C.x.as<double>(), prec, st);
  // x += P x_c
  vk_csr(C.prow.as<int64_t>(), C.pcol.as<int32_t>(), C.pval.as<double>(), C.x.as<double>(), x, n, C.nnz, true, st);
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
  double* zo = P.zo.as<double>();
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
  vcycle(P, 0, r, z, prec, st);
  copy(p, z, n, st);
  double rz = dot(dd, r, z, n, st);
  while (it < o.maxit) {
    op_apply(op, p, q, DOGIP_F64, st);
    const double pq = dot(dd, p, q, n, st);
    if (!std::isfinite(pq) || !std::isfinite(rz)) {
      status = DOGIP_E_NONFINITE;
      break;
    }
    if (!(pq > 0.0)) {
      status = DOGIP_E_BREAKDOWN;
      break;
    }
    const double alpha = rz / pq;
    vk_axpby(alpha, p, 1.0, x, n, st);
    vk_axpby(-alpha, q, 1.0, r, n, st);
    ++it;
    rr = dot(dd, r, r, n, st);
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
      rz = dot(dd, r, z, n, st);
      continue;
    }
    std::swap(z, zo);
    vcycle(P, 0, r, z, prec, st);
    const double rzn = dot(dd, r, z, n, st), rzo = dot(dd, r, zo, n, st);
    const double beta = (rzn - rzo) / rz;
    vk_axpby(1.0, z, beta, p, n, st);
    rz = rzn;
  }
  stats.iters = it;
  stats.outer = it + restarts;
  return status;
}

}  // namespace dogip
