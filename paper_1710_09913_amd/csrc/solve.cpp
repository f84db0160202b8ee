// Jacobi-preconditioned conjugate gradients and FP64 iterative refinement around
// an FP32-apply inner CG.  The paper leaves the solver open (Section 1: a
// suitable iterative solver); CG fits because A is symmetric positive definite.
//
// All scalars live on the device; the host only reads the residual history
// every check_every iterations, so iterations are queued back to back.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.hpp"
#include "pmg.hpp"
#include "solve.hpp"

namespace dogip {

static PcgWork& work(Op& op, int maxit) {
  const int64_t n = op.space->ndofs;
  if (!op.pcg || op.pcg->maxit < maxit) {
    auto w = std::make_unique<PcgWork>();
    w->n = n;
    w->maxit = maxit;
    const size_t vb = size_t(n) * sizeof(double);
    w->r.alloc(vb);
    w->p.alloc(vb);
    w->q.alloc(vb);
    w->rout.alloc(vb);
    w->dx.alloc(vb);
    w->yout.alloc(vb);
    w->part.alloc(size_t(3) * RED_BLOCKS * sizeof(double));
    w->energy.alloc(size_t(op.plan.ntiles + op_finish_energy_count(op)) * sizeof(double));
    w->scal.alloc(sizeof(PcgScalars));
    w->nrm.alloc(sizeof(double));
    w->hist.alloc(size_t(maxit + 2) * sizeof(double));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&w->hhist), size_t(maxit + 2) * sizeof(double), hipHostMallocDefault));
    op.pcg = std::move(w);
  }
  return *op.pcg;
}

struct CgResult {
  int status = DOGIP_OK;
  int iters = 0;
  double relres = 0.0;
  double bnorm = 0.0;
  bool stalled = false;
};

// One Jacobi-PCG run on A x = b (x holds the initial guess when x0_given).
// prec selects the apply used for the search directions.  With reliable, the
// recursive residual is replaced by the true FP64 residual b - A64 x whenever it
// has fallen by the factor delta since the last replacement, and at apparent
// convergence; the search direction is kept (residual replacement in the sense of
// van der Vorst and Ye), so the iteration continues without a restart.
// Stops when the tracked residual (true residual under reliable) is <= tol ||b||.
struct CgParams {
  double tol = 1e-8;
  int maxit = 1000;
  int prec = DOGIP_F64;
  bool reliable = false;
  double delta = 0.1;
  int check_every = 16;
  bool v32 = false;  // with the FP32 apply: r, p, q stored in FP32 (x and inner products FP64)
};

static CgResult cg_run(Op& op, const double* b, double* x, bool x0_given, const CgParams& cp, hipStream_t st) {
  PcgWork& w = work(op, std::max(cp.maxit, 1));
  const int64_t n = op.space->ndofs;
  double* r = w.r.as<double>();
  double* p = w.p.as<double>();
  double* q = w.q.as<double>();
  double* part = w.part.as<double>();
  double* hist = w.hist.as<double>();
  auto* sc = w.scal.as<PcgScalars>();
  const double* invd = op.invdiag.as<double>();
  const bool v32 = cp.v32 && cp.prec == DOGIP_F32 && op_has_v32(op);
  if (v32 && !w.r32.p) {
    w.r32.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(float));
    w.p32.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(float));
    w.q32.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(float));
  }
  float* r32 = w.r32.as<float>();
  float* p32 = w.p32.as<float>();
  float* q32 = w.q32.as<float>();
  const float* invd32 = op.invdiag32.as<float>();
  // per dof: x, r, p, A p and the inverse diagonal (FP64, or r, p, A p, inverse diagonal FP32)
  const bool stream = stream_vectors(n, v32 ? 24 : 40, int64_t(op.lidx.bytes + op.tile_dofs.bytes));
  if (x0_given) {
    op_apply(op, x, q, DOGIP_F64, st);
    if (v32)
      vk_pcg_init32(b, q, invd32, r32, p32, n, part, sc, hist, st);
    else
      vk_pcg_init(b, q, invd, r, p, n, part, sc, hist, st);
  } else {
    vk_fill(x, 0.0, n, st);
    if (v32)
      vk_pcg_init32(b, nullptr, invd32, r32, p32, n, part, sc, hist, st);
    else
      vk_pcg_init(b, nullptr, invd, r, p, n, part, sc, hist, st);
  }
  PcgScalars hs{};
  HIPCHK(hipMemcpyAsync(&hs, sc, sizeof hs, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  CgResult res;
  res.bnorm = std::sqrt(hs.bb);
  if (hs.flags) {
    res.status = DOGIP_E_NONFINITE;
    return res;
  }
  if (hs.bb == 0.0) {
    vk_fill(x, 0.0, n, st);
    return res;
  }
  const double thr = cp.tol * cp.tol * hs.bb;
  res.relres = std::sqrt(hs.rr / hs.bb);
  if (hs.rr <= thr) return res;
  double rr_true = hs.rr;  // residual norm^2 at the last exact (re)computation
  double rr_min = hs.rr;   // smallest true residual norm^2 so far
  int stalls = 0;
  int last_rep = 0;  // iteration of the last replacement
  int it = 0;
  int step = std::max(1, cp.check_every);
  for (;;) {
    const int todo = std::min(step, cp.maxit - it);
    for (int j = 0; j < todo; ++j) {
      if (v32) {
        op_apply_v32(op, p32, q32, st, w.energy.as<double>());
        vk_fin_pq(w.energy.as<double>(), op.plan.ntiles + op_finish_energy_count(op), sc, st);
        vk_pcg_xr32(x, r32, p32, q32, invd32, sc, n, part, stream, st);
        vk_fin_rz(part, sc, hist, it + j + 1, st);
        vk_pcg_p32(p32, r32, invd32, sc, n, st);
      } else {
        op_apply(op, p, q, cp.prec, st, w.energy.as<double>());
        vk_fin_pq(w.energy.as<double>(), op.plan.ntiles + op_finish_energy_count(op), sc, st);
        vk_pcg_xr(x, r, p, q, invd, sc, n, part, stream, st);
        vk_fin_rz(part, sc, hist, it + j + 1, st);
        vk_pcg_p(p, r, invd, sc, n, stream, st);
      }
    }
    HIPCHK(hipMemcpyAsync(w.hhist + it + 1, hist + it + 1, sizeof(double) * todo, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool conv = false;
    for (int j = 1; j <= todo; ++j) {
      const double rr = w.hhist[it + j];
      if (rr < 0.0 || !std::isfinite(rr)) {
        HIPCHK(hipMemcpy(&hs, sc, sizeof hs, hipMemcpyDeviceToHost));
        res.status = (hs.flags & PCG_BREAKDOWN) ? DOGIP_E_BREAKDOWN : DOGIP_E_NONFINITE;
        res.iters = it + j;
        return res;
      }
      if (rr <= thr) {
        conv = true;
        break;
      }
    }
    const double first = w.hhist[it + 1];
    it += todo;
    double last = w.hhist[it];
    res.iters = it;
    const bool forced = cp.prec == DOGIP_F32 && it - last_rep >= 512;  // keep the true residual in view
    if (cp.reliable && (conv || forced || last <= cp.delta * cp.delta * rr_true)) {
      last_rep = it;
      // residual replacement with the FP64 operator
      // at apparent convergence the direction restarts from the true residual; the
      // replacements triggered by delta keep it
      op_apply(op, x, q, DOGIP_F64, st);
      const bool restarted = conv;
      if (v32)
        vk_replace32(b, q, invd32, r32, restarted ? p32 : nullptr, n, part, sc, st);
      else
        vk_replace(b, q, invd, r, restarted ? p : nullptr, n, part, sc, st);
      HIPCHK(hipMemcpyAsync(&hs, sc, sizeof hs, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (hs.flags || !std::isfinite(hs.rr)) {
        res.status = DOGIP_E_NONFINITE;
        return res;
      }
      const bool gap = hs.rr > GAP_RR * std::max(last, 1e-300);
      if (cp.prec == DOGIP_F32) {
        // the FP32 error dominates when the true residual is well above the recursive
        // one; far above its minimum, the iteration diverges: hand over at once
        const bool diverged = hs.rr > DIVERGE_RR * rr_min;
        stalls = diverged ? 3 : (gap ? stalls + 1 : 0);
      } else {
        stalls = hs.rr > 0.25 * rr_true ? stalls + 1 : 0;
      }
      if (gap && !restarted) {
        // a recursive residual far below the true one no longer describes the iterate: it
        // lost its accuracy, or the Krylov space ran out (a right-hand side in a few
        // eigenvectors) and the last steps ran on rounding noise.  The kept direction
        // belongs to that residual; keeping it took a huge step along noise (alpha =
        // r.z / p.Ap with a tiny p) and diverged.  Restart the direction from the true
        // residual (q still holds A64 x; the same r and r.z are recomputed).
        if (v32)
          vk_replace32(b, q, invd32, r32, p32, n, part, sc, st);
        else
          vk_replace(b, q, invd, r, p, n, part, sc, st);
      }
      rr_min = std::min(rr_min, hs.rr);
      rr_true = hs.rr;
      last = hs.rr;
      conv = hs.rr <= thr;
      if (!conv && stalls >= (cp.prec == DOGIP_F32 ? 3 : 2)) {
        // the true residual stopped decreasing: with the FP32 operator the caller
        // finishes in FP64; with FP64 the tolerance is below the attainable accuracy
        res.relres = std::sqrt(hs.rr / hs.bb);
        res.status = DOGIP_E_NOT_CONVERGED;
        res.stalled = cp.prec == DOGIP_F32;
        return res;
      }
    }
    res.relres = std::sqrt(std::max(last, 0.0) / hs.bb);
    if (conv) return res;
    if (it >= cp.maxit) {
      res.status = DOGIP_E_NOT_CONVERGED;
      return res;
    }
    // predict the iterations still needed from the recent convergence rate
    if (todo > 1 && last > 0 && first > last) {
      const double rate = std::log(last / first) / (todo - 1);
      double target = thr;
      if (cp.reliable) target = std::max(thr, cp.delta * cp.delta * rr_true);
      const double need = std::log(target / last) / rate;
      step = int(std::min<double>(std::max<double>(need * 0.9, 1.0), double(std::max(8, cp.check_every * 4))));
    } else {
      step = std::max(1, cp.check_every);
    }
  }
}

int cg_inner(Op& op, const double* b, double* x, double tol, int maxit, int prec, hipStream_t st) {
  CgParams cp;
  cp.tol = tol;
  cp.maxit = std::max(1, maxit);
  cp.prec = prec;
  cp.reliable = false;
  return cg_run(op, b, x, false, cp, st).iters;
}

// ||b - A x|| with the FP64 apply; writes the residual into r.
static double true_residual(Op& op, const double* b, const double* x, double* r, hipStream_t st) {
  PcgWork& w = *op.pcg;
  op_apply(op, x, w.yout.as<double>(), DOGIP_F64, st);
  vk_resid(b, w.yout.as<double>(), r, op.space->ndofs, w.part.as<double>(), w.nrm.as<double>(), st);
  double rr = 0.0;
  HIPCHK(hipMemcpyAsync(&rr, w.nrm.p, sizeof rr, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return std::sqrt(rr);
}

// ||a||^2 (deterministic reduction).
static double norm2(Op& op, const double* a, hipStream_t st) {
  PcgWork& w = *op.pcg;
  vk_dot(a, a, op.space->ndofs, w.part.as<double>(), w.nrm.as<double>(), st);
  double v = 0.0;
  HIPCHK(hipMemcpyAsync(&v, w.nrm.p, sizeof v, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return v;
}

int op_pcg(Op& op, const double* b, double* x, const dogip_solve_opts& o, dogip_solve_stats& stats, hipStream_t st) {
  DOGIP_CHECK(b && x, DOGIP_E_NULL, "null vector");
  DOGIP_CHECK(b != x, DOGIP_E_INVALID, "b and x must differ");
  DOGIP_CHECK(o.tol > 0.0 && o.maxit >= 1, DOGIP_E_RANGE, "tol must be > 0 and maxit >= 1");
  DOGIP_CHECK(o.mode >= DOGIP_SOLVE_F64 && o.mode <= DOGIP_SOLVE_MIXED_V64, DOGIP_E_RANGE, "unknown solve mode");
  DOGIP_CHECK(o.mode == DOGIP_SOLVE_F64 || o.mode == DOGIP_SOLVE_PMG || op.has32, DOGIP_E_STATE,
              "mixed mode needs DOGIP_OP_FP32");
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(&stats, 0, sizeof stats);
  const int check = o.check_every > 0 ? o.check_every : 16;
  PcgWork& w = work(op, o.maxit);
  int status = DOGIP_OK;
  CgParams cp;
  cp.tol = o.tol;
  cp.maxit = o.maxit;
  cp.check_every = check;
  if (o.mode == DOGIP_SOLVE_PMG || o.mode == DOGIP_SOLVE_PMG_MIXED) {
    // flexible CG preconditioned by p-multigrid V-cycles (FP64 outside; the V-cycle's
    // applies in FP32 for PMG_MIXED)
    status = op_pcg_pmg(op, b, x, o, stats, o.mode == DOGIP_SOLVE_PMG ? DOGIP_F64 : DOGIP_F32, st);
  } else if (o.mode == DOGIP_SOLVE_F64 || o.mode == DOGIP_SOLVE_MIXED || o.mode == DOGIP_SOLVE_MIXED_V64) {
    // FP64: plain Jacobi-PCG.  MIXED: the same iteration with the FP32 apply, the
    // vectors r, p, q in FP32 (x and the inner products FP64), and FP64 residual
    // replacement (reliable updates); MIXED_V64 keeps r, p, q in FP64.  In every mode
    // apparent convergence is verified on the true FP64 residual (a replacement); the
    // mixed modes also replace whenever the residual has dropped by delta, which
    // re-rounds r from the FP64 residual.
    cp.prec = o.mode == DOGIP_SOLVE_F64 ? DOGIP_F64 : DOGIP_F32;
    cp.reliable = true;
    cp.delta = o.mode == DOGIP_SOLVE_F64 ? 0.0 : ((o.inner_tol > 0 && o.inner_tol < 1) ? o.inner_tol : 0.1);
    cp.v32 = o.mode == DOGIP_SOLVE_MIXED;
    CgResult c = cg_run(op, b, x, o.x0_given != 0, cp, st);
    status = c.status;
    stats.iters = c.iters;
    stats.outer = 1;
    stats.relres = c.relres;
    if (c.stalled && c.iters < o.maxit) {
      // finish with the FP64 operator from the current iterate
      CgParams f = cp;
      f.prec = DOGIP_F64;
      f.reliable = true;  // convergence still verified on the true residual
      f.delta = 0.0;
      f.v32 = false;
      f.maxit = o.maxit - c.iters;
      CgResult g = cg_run(op, b, x, true, f, st);
      status = g.status;
      stats.iters += g.iters;
      stats.outer = 2;
      stats.relres = g.relres;
    }
  } else {
    // MIXED_RESTART: FP64 iterative refinement r = b - A64 x; A32 d ~= r by a restarted
    // inner PCG to inner_tol; x += d.
    const int64_t n = op.space->ndofs;
    double* rout = w.rout.as<double>();
    double* dx = w.dx.as<double>();
    const double bn = std::sqrt(norm2(op, b, st));
    if (o.x0_given) {
      stats.relres = bn > 0 ? true_residual(op, b, x, rout, st) / bn : 0.0;
    } else {
      vk_fill(x, 0.0, n, st);
      HIPCHK(hipMemcpyAsync(rout, b, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
      stats.relres = bn > 0 ? 1.0 : 0.0;
    }
    const double inner_tol = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
    int total = 0;
    for (int outer = 0; outer < max_outer; ++outer) {
      if (bn == 0.0 || stats.relres <= o.tol) break;
      CgParams in = cp;
      in.prec = DOGIP_F32;
      in.tol = std::max(inner_tol, 0.3 * o.tol / stats.relres);
      in.maxit = std::max(1, o.maxit - total);
      CgResult c = cg_run(op, rout, dx, false, in, st);
      total += c.iters;
      stats.outer = outer + 1;
      if (c.status == DOGIP_E_BREAKDOWN || c.status == DOGIP_E_NONFINITE) {
        status = c.status;
        break;
      }
      vk_axpy1(x, dx, n, st);
      const double rn = true_residual(op, b, x, rout, st);
      const double prev = stats.relres;
      stats.relres = rn / bn;
      if (!std::isfinite(stats.relres)) {
        status = DOGIP_E_NONFINITE;
        break;
      }
      if (total >= o.maxit && stats.relres > o.tol) {
        status = DOGIP_E_NOT_CONVERGED;
        break;
      }
      if (stats.relres > 0.9 * prev && stats.relres > o.tol) {
        // stagnation of the refinement: finish with FP64 CG from the current x
        CgParams f = cp;
        f.prec = DOGIP_F64;
        f.reliable = true;
        f.delta = 0.0;
        f.maxit = std::max(1, o.maxit - total);
        CgResult g = cg_run(op, b, x, true, f, st);
        total += g.iters;
        status = g.status;
        stats.relres = g.relres;
        break;
      }
    }
    stats.iters = total;
    if (status == DOGIP_OK && stats.relres > o.tol) status = DOGIP_E_NOT_CONVERGED;
  }
  // verified residual with the FP64 apply
  if (status == DOGIP_OK || status == DOGIP_E_NOT_CONVERGED) {
    const double bn = std::sqrt(norm2(op, b, st));
    // (op.pcg, not w: an inner solve of the multigrid's coarsest level on this same
    // operator may have regrown the work buffers)
    stats.relres_true = bn > 0 ? true_residual(op, b, x, op.pcg->rout.as<double>(), st) / bn : 0.0;
  }
  HIPCHK(hipStreamSynchronize(st));
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  stats.status = status;
  return status;
}

}  // namespace dogip
