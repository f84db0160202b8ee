// Batched operators: one persistent launch per apply over all problems, and a
// Jacobi-PCG per problem driven by segmented vector kernels (one CG each, with its
// own scalars and stopping test, all problems advancing in the same launches).
#include "batch.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace dogip {

struct BatchWork {
  int maxit = 0;
  DevBuf r32, p32, q32;  // FP32 vectors of the mixed iteration
  DevBuf r, p, q, yout, part, energy, sc, rr_true, rr_min, iters, need, stalls, active, res, state, use64, last_rep;
  DevBuf act, rep, items_a, items_b, items_r;  // compacted problem and work-item lists
  int* h_lists = nullptr;                      // pinned: active, use64, need, act, rep
  uint64_t* h_items = nullptr;                 // pinned: three item lists
  ~BatchWork() {
    if (h_lists) (void)hipHostFree(h_lists);
    if (h_items) (void)hipHostFree(h_items);
  }
};

Batch::~Batch() = default;

template <class T>
static void upload_vec(DevBuf& b, const std::vector<T>& v) {
  b.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

std::unique_ptr<Batch> make_batch(const std::vector<std::shared_ptr<Op>>& ops, hipStream_t st) {
  auto b = std::make_unique<Batch>();
  b->ops = ops;
  const Space& s0 = *ops[0]->space;
  b->dim = s0.dim;
  b->kind = s0.kind;
  DOGIP_CHECK(b->dim == 2, DOGIP_E_RANGE, "batched launches are built for 2D problems");
  const int np = int(ops.size());
  std::vector<BatchDesc> desc(np);
  std::vector<int64_t> voff(np + 1, 0), tile_base(np + 1, 0), bnd_off(np + 1, 0);
  std::vector<int32_t> shared, bnd;
  std::vector<int64_t> sh_off(np + 1, 0);
  std::vector<uint32_t> rowptr(1, 0), slots;
  std::vector<std::pair<double, uint64_t>> items;
  int64_t stage_total = 0;
  int64_t max32 = 0, max64 = 0;
  bool all32 = true;
  for (int p = 0; p < np; ++p) {
    const Op& op = *ops[p];
    const Space& s = *op.space;
    DOGIP_CHECK(s.dim == b->dim && s.kind == b->kind, DOGIP_E_INVALID, "batch problems must share dim and kind");
    DOGIP_CHECK(s.k >= 1 && s.k <= 4, DOGIP_E_RANGE, "batched launches cover k = 1..4");
    DOGIP_CHECK(op.variant == DOGIP_VARIANT_UNROLLED, DOGIP_E_INVALID, "batch operators must use the unrolled kernels");
    DOGIP_CHECK(!op.global_w && op.nq == 0, DOGIP_E_INVALID, "batch operators must use the element-wise D");
    DOGIP_CHECK(op.plan.te <= 256, DOGIP_E_RANGE, "batch tiles must have at most 256 cells");
    all32 = all32 && op.has32;
    BatchDesc& d = desc[p];
    d.D64 = op.d64.p;
    d.D32 = op.d32.p;
    d.lidx = op.lidx.as<uint16_t>();
    d.tile_off = op.tile_off.as<int64_t>();
    d.tile_dofs = op.tile_dofs.as<uint32_t>();
    d.stage_off = op.stage_off.as<int64_t>();
    d.nel = s.nc;
    d.ntiles = op.plan.ntiles;
    d.nch64 = op.nch64;
    d.nch32 = op.nch32;
    d.voff = voff[p];
    d.stage_base = stage_total;
    d.tile_base = tile_base[p];
    d.nlc = op.plan.nlc;
    d.te = op.plan.te;
    d.lds_slots = int(op.plan.max_tile_dofs);
    d.k = s.k;
    max64 = std::max<int64_t>(max64, d.lds_slots);
    max32 = std::max<int64_t>(max32, d.lds_slots);
    voff[p + 1] = voff[p] + s.ndofs;
    tile_base[p + 1] = tile_base[p] + op.plan.ntiles;
    // work items: cost ~ D bytes of the tile's cells
    for (int64_t t = 0; t < op.plan.ntiles; ++t) {
      const int64_t cells = std::min<int64_t>(op.plan.te, s.nc - t * op.plan.te);
      items.push_back({-double(cells) * double(op.nch64 + op.plan.nlc), (uint64_t(p) << 32) | uint64_t(t)});
    }
    // combined second-pass lists (indices into the concatenated vectors / staging buffer)
    for (size_t i = 0; i < op.plan.shared.size(); ++i) {
      shared.push_back(int32_t(voff[p] + op.plan.shared[i]));
      for (uint32_t j = op.plan.sh_rowptr[i]; j < op.plan.sh_rowptr[i + 1]; ++j)
        slots.push_back(uint32_t(stage_total + op.plan.sh_slots[j]));
      rowptr.push_back(uint32_t(slots.size()));
    }
    sh_off[p + 1] = int64_t(shared.size());
    for (int32_t v : s.boundary) bnd.push_back(int32_t(voff[p] + v));
    bnd_off[p + 1] = int64_t(bnd.size());
    stage_total += op.plan.stage_off.back();
  }
  DOGIP_CHECK(voff[np] < (int64_t(1) << 31) && stage_total < (int64_t(1) << 32), DOGIP_E_RANGE, "batch too large");
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, uint64_t>& a, const std::pair<double, uint64_t>& c) { return a.first < c.first; });
  std::vector<uint64_t> it(items.size());
  for (size_t i = 0; i < items.size(); ++i) it[i] = items[i].second;
  b->offsets = voff;
  b->ntiles_total = tile_base[np];
  b->nitems = int64_t(it.size());
  b->nshared = int64_t(shared.size());
  b->nbnd = int64_t(bnd.size());
  upload_vec(b->desc, desc);
  upload_vec(b->items, it);
  upload_vec(b->voff, voff);
  upload_vec(b->tile_base, tile_base);
  upload_vec(b->shared, shared);
  upload_vec(b->rowptr, rowptr);
  upload_vec(b->slots, slots);
  {
    std::vector<uint32_t> pair, more_off, more;
    pair_lists(rowptr, slots, pair, more_off, more);
    upload_vec(b->pair, pair);
    upload_vec(b->more_off, more_off);
    upload_vec(b->more, more);
  }
  upload_vec(b->bnd, bnd);
  upload_vec(b->bnd_off, bnd_off);
  upload_vec(b->sh_off, sh_off);
  b->items_host = it;
  b->counter.alloc(sizeof(uint32_t));
  b->stage.alloc(size_t(std::max<int64_t>(stage_total, 1)) * sizeof(double));
  b->invd.alloc(size_t(voff[np]) * sizeof(double));
  for (int p = 0; p < np; ++p)
    HIPCHK(hipMemcpyAsync(b->invd.as<double>() + voff[p], ops[p]->invdiag.p, size_t(voff[p + 1] - voff[p]) * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
  if (all32) {
    b->invd32.alloc(size_t(std::max<int64_t>(voff[np], 1)) * sizeof(float));
    launch_to_f32(b->invd.as<double>(), b->invd32.as<float>(), voff[np], st);
  }
  HIPCHK(hipStreamSynchronize(st));
  // persistent grid: as many workgroups as fit on the device at once
  b->lds64 = size_t(max64) * (sizeof(double) + sizeof(double));
  b->lds32 = size_t(max32) * (sizeof(double) + sizeof(float));
  int dev = 0, ncu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int o64 = std::max(1, batch_blocks_per_cu(b->dim, b->kind, DOGIP_F64, b->lds64));
  const int o32 = all32 ? std::max(1, batch_blocks_per_cu(b->dim, b->kind, DOGIP_F32, b->lds32)) : 1;
  b->grid64 = unsigned(std::max(1, ncu * o64));
  b->grid32 = unsigned(std::max(1, ncu * o32));
  b->w = std::make_unique<BatchWork>();
  return b;
}

static BatchLaunch launch_args(Batch& b, const double* u, double* y, int prec) {
  BatchLaunch bl{};
  bl.desc = b.desc.as<BatchDesc>();
  bl.items = b.items.as<uint64_t>();
  bl.counter = b.counter.as<uint32_t>();
  bl.nitems = b.nitems;
  bl.u = u;
  bl.y = y;
  bl.stage = b.stage.as<double>();
  bl.prec = prec;
  return bl;
}

static void run_apply(Batch& b, const BatchLaunch& bl, bool energy, hipStream_t st) {
  const bool f64 = bl.prec == DOGIP_F64;
  launch_batch_apply(b.dim, b.kind, bl, f64 ? b.grid64 : b.grid32, f64 ? b.lds64 : b.lds32, energy, st);
  launch_apply_finish(b.stage.as<double>(), b.pair.as<uint32_t>(), b.more_off.as<uint32_t>(), b.more.as<uint32_t>(),
                      b.shared.as<int32_t>(), b.nshared, b.bnd.as<int32_t>(), b.nbnd, bl.u, bl.y, nullptr, st);
  HIPCHK(hipGetLastError());
}

void batch_apply(Batch& b, const double* u, double* y, int prec, hipStream_t st) {
  DOGIP_CHECK(u && y, DOGIP_E_NULL, "null vector");
  DOGIP_CHECK(u != y, DOGIP_E_INVALID, "apply needs u != y");
  DOGIP_CHECK(prec == DOGIP_F64 || prec == DOGIP_F32, DOGIP_E_RANGE, "prec must be DOGIP_F64 or DOGIP_F32");
  if (prec == DOGIP_F32)
    for (auto& o : b.ops) DOGIP_CHECK(o->has32, DOGIP_E_STATE, "FP32 apply needs operators built with DOGIP_OP_FP32");
  run_apply(b, launch_args(b, u, y, prec), false, st);
}

int batch_pcg(Batch& b, const double* rhs, double* x, const dogip_solve_opts& o, dogip_solve_stats* stats,
              hipStream_t st) {
  DOGIP_CHECK(rhs && x, DOGIP_E_NULL, "null vector");
  DOGIP_CHECK(rhs != x, DOGIP_E_INVALID, "b and x must differ");
  DOGIP_CHECK(o.tol > 0.0 && o.maxit >= 1, DOGIP_E_RANGE, "tol must be > 0 and maxit >= 1");
  DOGIP_CHECK(o.mode == DOGIP_SOLVE_F64 || o.mode == DOGIP_SOLVE_MIXED, DOGIP_E_RANGE,
              "batched solves support DOGIP_SOLVE_F64 and DOGIP_SOLVE_MIXED");
  DOGIP_CHECK(!o.x0_given, DOGIP_E_RANGE, "batched solves start from x0 = 0");
  const bool mixed = o.mode == DOGIP_SOLVE_MIXED;
  if (mixed)
    for (auto& op : b.ops) DOGIP_CHECK(op->has32, DOGIP_E_STATE, "mixed mode needs DOGIP_OP_FP32");
  const auto t0 = std::chrono::steady_clock::now();
  const int np = int(b.ops.size());
  const int64_t n = b.offsets.back();
  constexpr int GX_MAX = 1024;  // blocks per problem in the segmented vector kernels
  BatchWork& w = *b.w;
  const size_t ni = b.items_host.size();
  if (mixed && !w.r32.p) {
    const size_t vf = size_t(std::max<int64_t>(n, 1)) * sizeof(float);
    w.r32.alloc(vf);
    w.p32.alloc(vf);
    w.q32.alloc(vf);
  }
  if (!w.r.p) {
    const size_t vb = size_t(n) * sizeof(double);
    w.r.alloc(vb);
    w.p.alloc(vb);
    w.q.alloc(vb);
    w.yout.alloc(vb);
    w.part.alloc(size_t(np) * GX_MAX * 3 * sizeof(double));
    w.energy.alloc(size_t(b.ntiles_total) * sizeof(double));
    w.sc.alloc(size_t(np) * sizeof(PcgScalars));
    w.rr_true.alloc(size_t(np) * sizeof(double));
    w.rr_min.alloc(size_t(np) * sizeof(double));
    w.iters.alloc(size_t(np) * sizeof(int));
    w.need.alloc(size_t(np) * sizeof(int));
    w.stalls.alloc(size_t(np) * sizeof(int));
    w.active.alloc(size_t(np) * sizeof(int));
    w.res.alloc(size_t(np) * sizeof(double));
    w.state.alloc(size_t(np) * sizeof(int));
    w.use64.alloc(size_t(np) * sizeof(int));
    w.last_rep.alloc(size_t(np) * sizeof(int));
    w.act.alloc(size_t(np) * sizeof(int));
    w.rep.alloc(size_t(np) * sizeof(int));
    w.items_a.alloc(ni * sizeof(uint64_t));
    w.items_b.alloc(ni * sizeof(uint64_t));
    w.items_r.alloc(ni * sizeof(uint64_t));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&w.h_lists), size_t(5) * np * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&w.h_items), size_t(3) * ni * sizeof(uint64_t), hipHostMallocDefault));
  }
  BatchVecArgs v{};
  v.voff = b.voff.as<int64_t>();
  v.invd = b.invd.as<double>();
  v.r = w.r.as<double>();
  v.p = w.p.as<double>();
  // mixed: r, p and A p in FP32 (x and the inner products FP64)
  v.v32 = mixed;
  {
    int64_t idx = 0;
    for (const auto& op : b.ops) idx += int64_t(op->lidx.bytes + op->tile_dofs.bytes);
    v.stream = stream_vectors(b.offsets.back(), mixed ? 24 : 40, idx);
  }
  v.invd32 = b.invd32.as<float>();
  v.r32 = w.r32.as<float>();
  v.p32 = w.p32.as<float>();
  v.part = w.part.as<double>();
  v.s = {w.sc.as<PcgScalars>(), w.rr_true.as<double>(), w.iters.as<int>(), w.need.as<int>(), w.stalls.as<int>(),
         w.active.as<int>(), w.state.as<int>(), w.use64.as<int>(), w.last_rep.as<int>(), w.rr_min.as<double>()};
  v.gx = 32;
  v.np = np;
  v.tol = o.tol;
  const double delta = (o.inner_tol > 0 && o.inner_tol < 1) ? o.inner_tol : 0.1;
  const int check = o.check_every > 0 ? o.check_every : 16;
  bk_init(v, rhs, x, st);
  int* h_active = w.h_lists;
  int* h_use64 = w.h_lists + np;
  int* h_need = w.h_lists + 2 * np;
  int* h_act = w.h_lists + 3 * np;
  int* h_rep = w.h_lists + 4 * np;
  uint64_t* h_ia = w.h_items;
  uint64_t* h_ib = w.h_items + ni;
  uint64_t* h_ir = w.h_items + 2 * ni;
  // items of the problems selected by sel(p), in the stored (largest first) order
  auto filter_items = [&](uint64_t* out, auto sel) {
    int64_t c = 0;
    for (uint64_t it : b.items_host)
      if (sel(int(it >> 32))) out[c++] = it;
    return c;
  };
  // u, y: double, or float (the FP32 vectors of the mixed iteration) when f32
  auto apply_list = [&](const void* u, void* y, bool f32, int prec, const uint64_t* items, int64_t nitems,
                        bool energy) {
    if (nitems <= 0) return;
    BatchLaunch bl = launch_args(b, f32 ? nullptr : static_cast<const double*>(u),
                                 f32 ? nullptr : static_cast<double*>(y), prec);
    if (f32) {
      bl.u32 = static_cast<const float*>(u);
      bl.y32 = static_cast<float*>(y);
    }
    bl.items = items;
    bl.nitems = nitems;
    bl.energy = energy ? w.energy.as<double>() : nullptr;
    const bool f64 = prec == DOGIP_F64;
    launch_batch_apply(b.dim, b.kind, bl, f64 ? b.grid64 : b.grid32, f64 ? b.lds64 : b.lds32, energy, st);
  };
  auto finish_list = [&](const int* act, int nact, const void* u, void* y, bool f32) {
    bk_finish(v, act, nact, b.stage.as<double>(), b.rowptr.as<uint32_t>(), b.slots.as<uint32_t>(),
              b.shared.as<int32_t>(), b.sh_off.as<int64_t>(), b.bnd.as<int32_t>(), b.bnd_off.as<int64_t>(), u, y, f32,
              st);
  };
  std::vector<int> iters(np), state(np), use64(np);
  int done_it = 0;
  for (;;) {
    HIPCHK(hipMemcpyAsync(h_active, w.active.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_use64, w.use64.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h_need, w.need.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    {
      // residual replacement r = b - A64 x for the problems that asked for it (at apparent
      // convergence, and in mixed mode also after each reduction by delta)
      int nrep = 0;
      for (int p = 0; p < np; ++p)
        if (h_active[p] && h_need[p]) h_rep[nrep++] = p;
      if (nrep > 0) {
        const int64_t nir = filter_items(h_ir, [&](int p) { return h_active[p] && h_need[p]; });
        HIPCHK(hipMemcpyAsync(w.rep.p, h_rep, sizeof(int) * nrep, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(w.items_r.p, h_ir, sizeof(uint64_t) * nir, hipMemcpyHostToDevice, st));
        apply_list(x, w.yout.as<double>(), false, DOGIP_F64, w.items_r.as<uint64_t>(), nir, false);
        finish_list(w.rep.as<int>(), nrep, x, w.yout.as<double>(), false);
        BatchVecArgs vr = v;
        vr.act = w.rep.as<int>();
        vr.nact = nrep;
        bk_replace(vr, rhs, w.yout.as<double>(), mixed ? 1 : 0, st);
        // the problems whose replacement showed a gap restart their direction from the true
        // residual (need 3; A64 x is still in yout); the others return at once
        bk_replace(vr, rhs, w.yout.as<double>(), mixed ? 1 : 0, st);
        HIPCHK(hipMemcpyAsync(h_active, w.active.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(h_use64, w.use64.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
      }
    }
    int nact = 0;
    for (int p = 0; p < np; ++p)
      if (h_active[p]) h_act[nact++] = p;
    if (nact == 0 || done_it >= o.maxit) break;
    const int64_t nia = filter_items(h_ia, [&](int p) { return h_active[p] && !(mixed && h_use64[p]); });
    const int64_t nib = mixed ? filter_items(h_ib, [&](int p) { return h_active[p] && h_use64[p]; }) : 0;
    HIPCHK(hipMemcpyAsync(w.act.p, h_act, sizeof(int) * nact, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w.items_a.p, h_ia, sizeof(uint64_t) * std::max<int64_t>(nia, 1), hipMemcpyHostToDevice, st));
    if (nib > 0) HIPCHK(hipMemcpyAsync(w.items_b.p, h_ib, sizeof(uint64_t) * nib, hipMemcpyHostToDevice, st));
    v.act = w.act.as<int>();
    v.nact = nact;
    // spread the segmented vector kernels over the whole device whatever the number of problems left
    v.gx = std::min(GX_MAX, std::max(16, 8192 / nact));
    const int todo = std::min(check, o.maxit - done_it);
    for (int j = 0; j < todo; ++j) {
      const void* pv = mixed ? static_cast<const void*>(v.p32) : static_cast<const void*>(v.p);
      void* qv = mixed ? static_cast<void*>(w.q32.p) : static_cast<void*>(w.q.p);
      apply_list(pv, qv, mixed, mixed ? DOGIP_F32 : DOGIP_F64, w.items_a.as<uint64_t>(), nia, true);
      apply_list(pv, qv, mixed, DOGIP_F64, w.items_b.as<uint64_t>(), nib, true);
      finish_list(v.act, nact, pv, qv, mixed);
      HIPCHK(hipGetLastError());
      bk_fin_pq(v, w.energy.as<double>(), b.tile_base.as<int64_t>(), b.bnd.as<int32_t>(), b.bnd_off.as<int64_t>(), st);
      bk_xr(v, x, qv, st);
      bk_fin_rz(v, delta, mixed ? 1 : 0, st);
      bk_p(v, st);
    }
    done_it += todo;
  }
  // verified residuals with the FP64 operator
  run_apply(b, launch_args(b, x, w.yout.as<double>(), DOGIP_F64), false, st);
  bk_resid(v, rhs, w.yout.as<double>(), w.res.as<double>(), st);
  std::vector<double> res(np);
  std::vector<PcgScalars> sc(np);
  HIPCHK(hipMemcpyAsync(res.data(), w.res.p, sizeof(double) * np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(sc.data(), w.sc.p, sizeof(PcgScalars) * np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(iters.data(), w.iters.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(state.data(), w.state.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(use64.data(), w.use64.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = DOGIP_OK;
  for (int p = 0; p < np; ++p) {
    const double bn = std::sqrt(sc[p].bb);
    const double rel = bn > 0 ? std::sqrt(res[p]) / bn : 0.0;
    int status = DOGIP_OK;
    if (sc[p].flags & PCG_BREAKDOWN)
      status = DOGIP_E_BREAKDOWN;
    else if ((sc[p].flags & PCG_NONFINITE) || !std::isfinite(rel))
      status = DOGIP_E_NONFINITE;
    else if (state[p] != 1)
      status = DOGIP_E_NOT_CONVERGED;
    if (status != DOGIP_OK && (worst == DOGIP_OK || status > worst)) worst = status;
    if (stats) {
      dogip_solve_stats& s = stats[p];
      std::memset(&s, 0, sizeof s);
      s.status = status;
      s.iters = iters[p];
      s.outer = use64[p] ? 2 : 1;
      s.relres = bn > 0 ? std::sqrt(std::max(sc[p].rr, 0.0)) / bn : 0.0;
      s.relres_true = rel;
      s.seconds = secs;
    }
  }
  return worst;
}

}  // namespace dogip
