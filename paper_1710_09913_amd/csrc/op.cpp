// Operator construction and the apply / diagonal / gradient entry points.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.hpp"
#include "reftab.hpp"
#include "pmg.hpp"
#include "solve.hpp"

namespace dogip {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? DOGIP_E_NOMEM : DOGIP_E_HIP;
    throw Error(code, std::string(what) + ": " + hipGetErrorString(e));
  }
}

void DevBuf::alloc(size_t n) {
  free();
  if (n == 0) return;
  HIPCHK(hipMalloc(&p, n));
  bytes = n;
}
void DevBuf::free() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

// Events before the tile kernel, between it and the finish kernel, and after the finish.
// Per-apply launch timer: events before the tile kernel, between it and the second pass
// and after it.  The events only time: they are made without the system-scope fence of a
// default event (a writeback and invalidation of the caches at each record, which on
// MI355X lengthened a timed apply by about 10 us), and are kept for reuse.
struct OpTimer {
  bool on = false;
  std::vector<std::array<hipEvent_t, 3>> ev;  // ev[0, used) hold recorded applies
  size_t used = 0;
  std::array<hipEvent_t, 3>& next() {
    if (used == ev.size()) {
      std::array<hipEvent_t, 3> e{};
      for (auto& x : e) HIPCHK(hipEventCreateWithFlags(&x, hipEventDisableSystemFence));
      ev.push_back(e);
    }
    return ev[used++];
  }
  void clear() { used = 0; }
  ~OpTimer() {
    for (auto& e : ev)
      for (auto x : e) (void)hipEventDestroy(x);
  }
};

bool launch_apply_unrolled_2d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st);
bool launch_apply_unrolled_3d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st);
bool launch_apply_factored(int dim, int k, int prec, bool energy, const ApplyLaunch& a, hipStream_t st);
bool launch_apply_looped_2d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st);
bool launch_apply_looped_3d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st);

bool has_unrolled(int dim, int k, int kind) {
  if (dim == 2) return k <= 5;
  return kind == KIND_SE ? k <= 3 : k <= 2;
}

bool has_mfma(int dim, int k, int kind) { return dim == 3 && k == 3 && kind == KIND_SE; }

bool has_factored(int dim, int k, int kind) { return kind == KIND_SE && k >= 2 && k <= (dim == 2 ? 5 : 3); }

bool launch_apply(int dim, int k, int kind, int prec, int variant, const ApplyLaunch& a, hipStream_t st) {
  const bool en = a.energy != nullptr;
  if (variant == DOGIP_VARIANT_MFMA) {
    if (prec == DOGIP_F32) return launch_apply_mfma(en, a, st);
    variant = DOGIP_VARIANT_UNROLLED;  // FP64 applies take the unrolled vector kernel
  }
  if (variant == DOGIP_VARIANT_FACTORED) return launch_apply_factored(dim, k, prec, en, a, st);
  if (variant == DOGIP_VARIANT_UNROLLED)
    return dim == 2 ? launch_apply_unrolled_2d(k, kind, prec, en, a, st)
                    : launch_apply_unrolled_3d(k, kind, prec, en, a, st);
  return dim == 2 ? launch_apply_looped_2d(k, kind, prec, en, a, st) : launch_apply_looped_3d(k, kind, prec, en, a, st);
}

Op::~Op() = default;

template <class T>
static void upload(DevBuf& b, const std::vector<T>& v) {
  b.alloc(v.size() * sizeof(T));
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// inverse of the Jacobi diagonal, and its FP32 copy for the mixed CG
static void set_invdiag(Op& op, const double* diag, hipStream_t st) {
  const int64_t n = op.space->ndofs;
  launch_invert(diag, op.invdiag.as<double>(), n, st);
  if (op.has32) {
    if (!op.invdiag32.p) op.invdiag32.alloc(size_t(std::max<int64_t>(n, 1)) * sizeof(float));
    launch_to_f32(op.invdiag.as<double>(), op.invdiag32.as<float>(), n, st);
  }
}

// Default tile size in waves of 64 cells.  Element-wise operators take large tiles where
// that measured faster, run in passes by fewer lanes: the per-tile gather, accumulation
// and flush are paid once per tile and fewer partial sums are staged (3D 64^3 P3, 1536-cell
// tiles against 512: FP64 apply 0.51 -> 0.46 ms, FP32 0.30 -> 0.29 ms; 3D 64^3 P2, 3072
// against 512: 0.159 -> 0.149 and 0.105 -> 0.094 ms; 2D 512^2 P3, 1024 against 256: 0.061 ->
// 0.054 and 0.0435 -> 0.041 ms).  On the unit-cube meshes 1536 and 3072 cells are aligned
// 8 x 8 x 4 and 8 x 8 x 8 blocks of cubes.  Large tiles are reduced while the mesh would
// give fewer than two tiles per compute unit (2D 256^2 P3: 1024-cell tiles 25% slower
// than 256).  The matrix-core variant and the global form keep at most 8 waves, 3D P4
// 8, other orders 4 (2D 512^2 P5: 8 waves equal to 4 within noise).
static int default_tile_waves(const Space& s, int variant, bool global_w) {
  if (variant == DOGIP_VARIANT_MFMA || global_w) return (s.dim == 3 && s.k >= 2) ? 8 : 4;
  int tw = 4;
  if (s.dim == 3 && s.k == 2) tw = 48;
  if (s.dim == 3 && s.k == 3) tw = 24;
  if (s.dim == 3 && s.k >= 4) tw = 8;
  if (s.dim == 2 && s.k == 3) tw = 16;
  const int64_t min_tiles = 512;  // two per compute unit
  while (tw > 4 && (s.nc + 64 * tw - 1) / (64 * tw) < min_tiles) tw = tw > 8 ? tw / 2 : 4;
  return tw;
}

// The next smaller tile (in waves) tried when a tile's LDS arrays exceed the budget.
static int smaller_tile(int w) {
  static const int sizes[] = {48, 32, 24, 16, 12, 8, 6, 4, 3, 2, 1};
  for (int x : sizes)
    if (x < w) return x;
  return 1;
}

int tile_lanes(const void* kernel, int te, size_t lds, int requested) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t>, std::pair<int, int>> cache;  // (auto lanes, max lanes)
  const auto key = std::make_tuple(kernel, te, lds);
  std::pair<int, int> c{0, 0};
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) c = it->second;
  }
  if (c.first == 0) {
    hipFuncAttributes fa{};
    HIPCHK(hipFuncGetAttributes(&fa, kernel));
    if (lds > 65536) HIPCHK(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    int best = 0, best_waves = 0;
    for (int lanes = 64; lanes <= te && lanes <= fa.maxThreadsPerBlock; lanes += 64) {
      if (te % lanes) continue;
      int blocks = 0;
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, lanes, lds));
      const int waves = blocks * (lanes / 64);
      if (waves > best_waves) best = lanes, best_waves = waves;  // ties keep the fewer lanes
    }
    DOGIP_CHECK(best > 0, DOGIP_E_RANGE, "no workgroup shape fits the tile's LDS arrays");
    c = {best, fa.maxThreadsPerBlock};
    std::lock_guard<std::mutex> g(mu);
    cache[key] = c;
  }
  if (requested <= 0) return c.first;
  DOGIP_CHECK(requested % 64 == 0 && te % requested == 0 && requested <= c.second, DOGIP_E_RANGE,
              "requested lanes do not fit this tile kernel");
  return requested;
}

static void check_coef(const Space& s, int coef_kind) {
  DOGIP_CHECK(coef_kind >= DOGIP_COEF_SCALAR && coef_kind <= DOGIP_COEF_RAW_D, DOGIP_E_RANGE, "unknown coefficient form");
  DOGIP_CHECK(!(coef_kind == DOGIP_COEF_SYM && s.kind == DOGIP_WP), DOGIP_E_RANGE,
              "a tensor coefficient needs the elliptic problem");
}

static void build_d(Op& op, int coef_kind, const double* coef, hipStream_t st) {
  const Space& s = *op.space;
  if (op.pmg) op.pmg->stale = true;  // levels keep their spaces and transfers; D is redone
  op.inc_depth = -1;
  if (coef_kind == DOGIP_COEF_RAW_D || op.global_w) {
    op.coef_kind_copy = -1;
  } else {
    const size_t per = coef_kind == DOGIP_COEF_SYM ? size_t(s.nsym) : 1;
    const size_t bytes = std::max<size_t>(per * size_t(s.nc), 1) * sizeof(double);
    if (op.coef_copy.bytes != bytes) op.coef_copy.alloc(bytes);
    if (s.nc > 0) HIPCHK(hipMemcpyAsync(op.coef_copy.p, coef, per * size_t(s.nc) * sizeof(double),
                                        hipMemcpyDeviceToDevice, st));
    op.coef_kind_copy = coef_kind;
  }
  BuildDLaunch b{};
  b.xyz = op.xyz.as<double>();
  b.cells = op.cells.as<int32_t>();
  b.perm = op.perm.as<int32_t>();
  b.what = op.what.as<double>();
  b.coef = coef;
  b.d64 = op.d64.as<double>();
  b.d32 = op.has32 ? op.d32.as<float>() : nullptr;
  b.nel = s.nc;
  b.nel_pad = op.plan.nel_pad;
  b.nch64 = op.nch64;
  b.nch32 = op.nch32;
  b.dim = s.dim;
  b.kind = s.kind;
  b.coef_kind = coef_kind;
  b.wt = s.wt;
  b.nsym = s.nsym;
  if (op.global_w)
    launch_build_dg(b, op.gw_inc_ptr.as<int64_t>(), op.gw_inc.as<int64_t>(), op.gplan.nw, op.dg64.as<double>(),
                    op.has32 ? op.dg32.as<float>() : nullptr, st);
  else
    launch_build_d(b, st);
  HIPCHK(hipGetLastError());
  // Jacobi diagonal -> inverse
  DevBuf tmp(size_t(s.ndofs) * sizeof(double));
  op_diag(op, tmp.as<double>(), st);
  set_invdiag(op, tmp.as<double>(), st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
}

std::unique_ptr<Op> make_op(std::shared_ptr<const Space> sp, int coef_kind, const double* coef, unsigned flags,
                            int tile_waves, int variant, hipStream_t st) {
  const Space& s = *sp;
  check_coef(s, coef_kind);
  DOGIP_CHECK(coef != nullptr, DOGIP_E_NULL, "null coefficient pointer");
  DOGIP_CHECK(tile_waves >= 0 && tile_waves <= 48, DOGIP_E_RANGE, "tile_waves must be 0..48");
  DOGIP_CHECK(variant >= DOGIP_VARIANT_AUTO && variant <= DOGIP_VARIANT_FACTORED, DOGIP_E_RANGE, "unknown variant");
  DOGIP_CHECK((flags & ~(DOGIP_OP_FP32 | DOGIP_OP_GLOBAL_W)) == 0, DOGIP_E_RANGE, "unknown operator flag");
  auto op = std::make_unique<Op>();
  op->space = sp;
  op->has32 = (flags & DOGIP_OP_FP32) != 0;
  op->global_w = (flags & DOGIP_OP_GLOBAL_W) != 0;
  DOGIP_CHECK(!op->global_w || s.kind == DOGIP_WP, DOGIP_E_RANGE,
              "DOGIP_OP_GLOBAL_W needs a weighted-projection space");
  if (variant == DOGIP_VARIANT_AUTO) variant = has_unrolled(s.dim, s.k, s.kind) ? DOGIP_VARIANT_UNROLLED : DOGIP_VARIANT_LOOPED;
  DOGIP_CHECK(variant == DOGIP_VARIANT_LOOPED || has_unrolled(s.dim, s.k, s.kind), DOGIP_E_RANGE,
              "no unrolled kernel for this (dim, k, kind)");
  DOGIP_CHECK(variant != DOGIP_VARIANT_MFMA || has_mfma(s.dim, s.k, s.kind), DOGIP_E_RANGE,
              "the matrix-core apply covers the 3D P3 elliptic operator only");
  DOGIP_CHECK(variant != DOGIP_VARIANT_MFMA || !op->global_w, DOGIP_E_RANGE,
              "the matrix-core apply needs the element-wise D");
  DOGIP_CHECK(variant != DOGIP_VARIANT_FACTORED || has_factored(s.dim, s.k, s.kind), DOGIP_E_RANGE,
              "the factored B^ covers the elliptic problem with 2 <= k <= 5 (2D), 3 (3D)");
  op->variant = variant;
  // tile size: requested or the default, stepped down until the LDS arrays fit (FP64 tiles
  // hold 16 bytes per dof; the matrix-core FP32 kernel, one cell per lane, 12 bytes per dof
  // and its 19 KB of B^ operand tables within 64 KB)
  const bool mfma = variant == DOGIP_VARIANT_MFMA;
  auto lds = [&](int64_t slots) { return mfma ? std::max<int64_t>(16 * slots, mfma_lds_tables() + 12 * slots) : 16 * slots; };
  const int64_t budget = mfma ? 65536 : LDS_TILE_MAX;
  int tw = tile_waves ? tile_waves : default_tile_waves(s, variant, op->global_w);
  for (;;) {
    op->plan = make_tiles(s, 64 * tw);
    if (lds(op->plan.max_tile_dofs) <= budget || tw == 1) break;
    tw = smaller_tile(tw);
  }
  DOGIP_CHECK(lds(op->plan.max_tile_dofs) <= budget, DOGIP_E_RANGE, "tile dofs exceed the LDS budget");
  DOGIP_CHECK(!mfma || op->plan.te <= 512, DOGIP_E_RANGE, "the matrix-core apply takes tiles of at most 8 waves");
  if (op->global_w) op->gplan = make_global_plan(s, op->plan);
  const TilePlan& p = op->plan;
  op->nch64 = d_chunks(s.wt, s.nsym, 2);
  // the matrix-core variant keeps its FP32 copy of D in its own layout (nch32 < 0)
  op->nch32 = variant == DOGIP_VARIANT_MFMA ? -1 : d_chunks(s.wt, s.nsym, 4);
  if (op->global_w) {
    const GlobalPlan& g = op->gplan;
    upload(op->gw_rec, g.mask);
    upload(op->gw_off, g.woff);
    upload(op->gw_inc_ptr, g.inc_ptr);
    upload(op->gw_inc, g.inc);
    op->dg64.alloc(size_t(g.nw) * sizeof(double));
    if (op->has32) op->dg32.alloc(size_t(g.nw) * sizeof(float));
  } else {
    const size_t ngrp = size_t(p.nel_pad / 64);
    op->d64.alloc(ngrp * op->nch64 * 64 * 2 * sizeof(double));
    HIPCHK(hipMemset(op->d64.p, 0, op->d64.bytes));
    if (op->has32) {
      op->d32.alloc(ngrp * size_t(op->nch32 < 0 ? mfma_d32_per_wave() : op->nch32 * 64 * 4) * sizeof(float));
      HIPCHK(hipMemset(op->d32.p, 0, op->d32.bytes));
    }
  }
  upload(op->lidx, p.lidx);
  upload(op->tile_off, p.tile_off);
  upload(op->tile_dofs, p.tile_dofs);
  upload(op->shared, p.shared);
  upload(op->stage_off, p.stage_off);
  upload(op->sh_pair, p.sh_pair);
  upload(op->sh_more_off, p.sh_more_off);
  upload(op->sh_more, p.sh_more);
  upload(op->bnd, s.boundary);
  op->stage.alloc(size_t(std::max<int64_t>(p.stage_off.back(), 1)) * sizeof(double));
  upload(op->perm, p.perm);
  const Mesh& m = *s.mesh;
  std::vector<int32_t> cint(size_t(s.nc) * (s.dim + 1));
  for (int64_t e = 0; e < s.nc; ++e)
    std::memcpy(&cint[e * (s.dim + 1)], &m.cells[int64_t(p.perm[e]) * (s.dim + 1)], sizeof(int32_t) * (s.dim + 1));
  upload(op->cells, cint);
  upload(op->xyz, m.xyz);
  upload(op->what, s.what);
  op->invdiag.alloc(size_t(s.ndofs) * sizeof(double));
  op->timer = std::make_unique<OpTimer>();
  build_d(*op, coef_kind, coef, st);
  return op;
}

std::unique_ptr<Op> make_op_qp(std::shared_ptr<const Space> sp, int n, const double* coef, unsigned flags,
                               int tile_waves, hipStream_t st) {
  const Space& s = *sp;
  DOGIP_CHECK(coef != nullptr, DOGIP_E_NULL, "null coefficient pointer");
  DOGIP_CHECK(tile_waves >= 0 && tile_waves <= 8, DOGIP_E_RANGE, "tile_waves must be 0..8");
  DOGIP_CHECK((flags & ~DOGIP_OP_FP32) == 0, DOGIP_E_RANGE, "unknown operator flag");
  DOGIP_CHECK(s.k <= (s.dim == 2 ? 5 : (s.kind == DOGIP_SE ? 4 : 3)), DOGIP_E_RANGE,
              "no quadrature-point kernel for this (dim, k, kind)");
  std::vector<double> pts, wts, tab;
  collapsed_rule(s.dim, n, pts, wts);
  basis_table(s.dim, s.k, s.kind, pts, tab);
  auto op = std::make_unique<Op>();
  op->space = sp;
  op->has32 = (flags & DOGIP_OP_FP32) != 0;
  op->variant = DOGIP_VARIANT_LOOPED;
  op->nq = int(wts.size());
  // 4-wave tiles by default: the point loop's registers make larger tiles slower
  // (3D 64^3 P3, n = 6: 2.86 ms with 4 waves, 3.46 ms with 8)
  int te = 64 * (tile_waves ? tile_waves : 4);
  for (;;) {
    op->plan = make_tiles(s, te);
    if (op->plan.max_tile_dofs * 16 <= 65536 || te == 64) break;
    te /= 2;
  }
  DOGIP_CHECK(op->plan.max_tile_dofs * 16 <= 65536, DOGIP_E_RANGE, "tile dofs exceed the LDS budget");
  const TilePlan& p = op->plan;
  upload(op->lidx, p.lidx);
  upload(op->tile_off, p.tile_off);
  upload(op->tile_dofs, p.tile_dofs);
  upload(op->shared, p.shared);
  upload(op->stage_off, p.stage_off);
  upload(op->sh_pair, p.sh_pair);
  upload(op->sh_more_off, p.sh_more_off);
  upload(op->sh_more, p.sh_more);
  upload(op->bnd, s.boundary);
  op->stage.alloc(size_t(std::max<int64_t>(p.stage_off.back(), 1)) * sizeof(double));
  upload(op->perm, p.perm);
  const Mesh& m = *s.mesh;
  std::vector<int32_t> cint(size_t(s.nc) * (s.dim + 1));
  for (int64_t e = 0; e < s.nc; ++e)
    std::memcpy(&cint[e * (s.dim + 1)], &m.cells[int64_t(p.perm[e]) * (s.dim + 1)], sizeof(int32_t) * (s.dim + 1));
  upload(op->cells, cint);
  upload(op->xyz, m.xyz);
  upload(op->qtab64, tab);
  upload(op->qw, wts);
  std::vector<float> tab32(tab.begin(), tab.end());
  if (op->has32) upload(op->qtab32, tab32);
  const size_t ngrp = size_t(p.nel_pad / 64);
  op->qs64.alloc(ngrp * op->nq * 64 * sizeof(double));
  HIPCHK(hipMemset(op->qs64.p, 0, op->qs64.bytes));
  if (op->has32) {
    op->qs32.alloc(ngrp * op->nq * 64 * sizeof(float));
    HIPCHK(hipMemset(op->qs32.p, 0, op->qs32.bytes));
  }
  if (s.kind == DOGIP_SE) {
    op->qk64.alloc(ngrp * s.nsym * 64 * sizeof(double));
    HIPCHK(hipMemset(op->qk64.p, 0, op->qk64.bytes));
    if (op->has32) {
      op->qk32.alloc(ngrp * s.nsym * 64 * sizeof(float));
      HIPCHK(hipMemset(op->qk32.p, 0, op->qk32.bytes));
    }
  }
  op->invdiag.alloc(size_t(s.ndofs) * sizeof(double));
  op->timer = std::make_unique<OpTimer>();
  QpSetupLaunch q{};
  q.xyz = op->xyz.as<double>();
  q.cells = op->cells.as<int32_t>();
  q.perm = op->perm.as<int32_t>();
  q.coef = coef;
  q.w = op->qw.as<double>();
  q.qs64 = op->qs64.as<double>();
  q.qs32 = op->has32 ? op->qs32.as<float>() : nullptr;
  q.qk64 = op->qk64.as<double>();
  q.qk32 = op->has32 ? op->qk32.as<float>() : nullptr;
  q.nel = s.nc;
  q.nq = op->nq;
  q.dim = s.dim;
  q.kind = s.kind;
  launch_qp_setup(q, st);
  HIPCHK(hipGetLastError());
  DevBuf tmp(size_t(s.ndofs) * sizeof(double));
  op_diag(*op, tmp.as<double>(), st);
  set_invdiag(*op, tmp.as<double>(), st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return op;
}

void op_set_coef(Op& op, int coef_kind, const double* coef, hipStream_t st) {
  DOGIP_CHECK(op.nq == 0, DOGIP_E_STATE, "a quadrature-point operator takes its samples at creation");
  check_coef(*op.space, coef_kind);
  DOGIP_CHECK(coef != nullptr, DOGIP_E_NULL, "null coefficient pointer");
  build_d(op, coef_kind, coef, st);
}

void op_set_inclusions(Op& op, int nballs, const double* balls, double a_in, double a_out, int depth, int ng,
                       double* mean_points, hipStream_t st) {
  const Space& s = *op.space;
  DOGIP_CHECK(!op.global_w && op.nq == 0, DOGIP_E_STATE, "sub-cell quadrature builds the element-wise D");
  DOGIP_CHECK(balls != nullptr, DOGIP_E_NULL, "null ball array");
  DOGIP_CHECK(nballs >= 1, DOGIP_E_RANGE, "need at least one ball");
  DOGIP_CHECK(depth >= 0 && depth <= 6, DOGIP_E_RANGE, "depth must be 0..6");
  DOGIP_CHECK(ng >= 1 && ng <= 8, DOGIP_E_RANGE, "points per direction must be 1..8");
  DOGIP_CHECK(std::isfinite(a_in) && std::isfinite(a_out), DOGIP_E_INVALID, "non-finite coefficient");
  // the elliptic form needs a positive coefficient (and the multigrid's coarse levels
  // take its logarithm)
  DOGIP_CHECK(a_in > 0.0 && a_out > 0.0, DOGIP_E_INVALID, "inclusion coefficients must be positive");
  for (int j = 0; j < nballs; ++j) {
    DOGIP_CHECK(balls[j * (s.dim + 1) + s.dim] > 0.0, DOGIP_E_INVALID, "ball radius must be positive");
    for (int x = 0; x <= s.dim; ++x)
      DOGIP_CHECK(std::isfinite(balls[j * (s.dim + 1) + x]), DOGIP_E_INVALID, "non-finite ball");
  }
  if (op.pmg) op.pmg->stale = true;
  op.coef_kind_copy = -1;
  op.inc_depth = -1;
  std::vector<double> pts, wts;
  collapsed_rule(s.dim, ng, pts, wts);
  DevBuf db(size_t(nballs) * (s.dim + 1) * sizeof(double)), dp(pts.size() * sizeof(double)),
      dw(wts.size() * sizeof(double));
  HIPCHK(hipMemcpy(db.p, balls, db.bytes, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dp.p, pts.data(), dp.bytes, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dw.p, wts.data(), dw.bytes, hipMemcpyHostToDevice));
  DevBuf cnt;
  if (mean_points) cnt.alloc(size_t(std::max<int64_t>(s.nc, 1)) * sizeof(double));
  SubLaunch a{};
  a.xyz = op.xyz.as<double>();
  a.cells = op.cells.as<int32_t>();
  a.balls = db.as<double>();
  a.gpts = dp.as<double>();
  a.gwts = dw.as<double>();
  a.what = op.what.as<double>();
  a.d64 = op.d64.as<double>();
  a.d32 = op.has32 ? op.d32.as<float>() : nullptr;
  a.npts = mean_points ? cnt.as<double>() : nullptr;
  a.a_in = a_in;
  a.a_out = a_out;
  a.nel = s.nc;
  a.nch64 = op.nch64;
  a.nch32 = op.nch32;
  a.nballs = nballs;
  a.ng = int(wts.size());
  a.depth = depth;
  a.kind = s.kind;
  launch_build_d_sub(s.dim, w_order(s.k, s.kind), a, st);
  HIPCHK(hipGetLastError());
  DevBuf tmp(size_t(s.ndofs) * sizeof(double));
  op_diag(op, tmp.as<double>(), st);
  set_invdiag(op, tmp.as<double>(), st);
  HIPCHK(hipGetLastError());
  if (mean_points) {
    std::vector<double> h(s.nc);
    HIPCHK(hipMemcpyAsync(h.data(), cnt.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double sum = 0.0;
    for (double v : h) sum += v;
    *mean_points = s.nc ? sum / double(s.nc) : 0.0;
  }
  HIPCHK(hipStreamSynchronize(st));
  op.inc_balls.assign(balls, balls + size_t(nballs) * (s.dim + 1));
  op.inc_in = a_in;
  op.inc_out = a_out;
  op.inc_ng = ng;
  op.inc_depth = depth;
}

static ApplyLaunch apply_args(const Op& op, int prec) {
  const Space& s = *op.space;
  ApplyLaunch a{};
  a.D = prec == DOGIP_F64 ? op.d64.p : op.d32.p;
  a.lidx = op.lidx.as<uint16_t>();
  a.tile_off = op.tile_off.as<int64_t>();
  a.tile_dofs = op.tile_dofs.as<uint32_t>();
  a.nel = s.nc;
  a.ntiles = op.plan.ntiles;
  a.nch = prec == DOGIP_F64 ? op.nch64 : op.nch32;
  a.nlc = op.plan.nlc;
  a.te = op.plan.te;
  const int lanes = prec == DOGIP_F64 ? op.plan.lanes64 : op.plan.lanes32;
  a.cpl = lanes ? op.plan.te / lanes : 0;
  a.lds_slots = int(op.plan.max_tile_dofs);
  a.tile_base = 0;
  a.stage_off = op.stage_off.as<int64_t>();
  a.stage = op.stage.as<double>();
  if (op.nq > 0) {
    const bool f64 = prec == DOGIP_F64;
    a.qtab = f64 ? op.qtab64.p : op.qtab32.p;
    a.qs = f64 ? op.qs64.p : op.qs32.p;
    a.qk = f64 ? op.qk64.p : op.qk32.p;
    a.nq = op.nq;
  }
  if (op.global_w) {
    a.D = prec == DOGIP_F64 ? op.dg64.p : op.dg32.p;
    a.gw_mask = op.gw_rec.as<uint32_t>();
    a.gw_woff = op.gw_off.as<int64_t>();
  }
  return a;
}

// The apply's two launches with the staging buffer `stage` (op.stage, or a caller's buffer
// of at least op_stage_entries(op) doubles); the timer records only with op.stage.
static void apply_impl(Op& op, const double* u, double* y, int prec, hipStream_t st, double* energy, double* stage) {
  const Space& s = *op.space;
  DOGIP_CHECK(u && y, DOGIP_E_NULL, "null vector");
  DOGIP_CHECK(u != y, DOGIP_E_INVALID, "apply needs u != y");
  DOGIP_CHECK(prec == DOGIP_F64 || prec == DOGIP_F32, DOGIP_E_RANGE, "prec must be DOGIP_F64 or DOGIP_F32");
  DOGIP_CHECK(prec == DOGIP_F64 || op.has32, DOGIP_E_STATE, "FP32 apply needs an operator built with DOGIP_OP_FP32");
  ApplyLaunch a = apply_args(op, prec);
  a.u = u;
  a.y = y;
  a.energy = energy;
  a.stage = stage;
  const bool timed = op.timer->on && stage == op.stage.as<double>();
  std::array<hipEvent_t, 3> ev{};
  if (timed) {
    ev = op.timer->next();
    HIPCHK(hipEventRecord(ev[0], st));
  }
  const bool ok = op.nq > 0     ? launch_apply_qp(s.dim, s.k, s.kind, prec, a, st)
                  : op.global_w ? launch_apply_global(s.dim, s.k, prec, op.variant, a, st)
                                : launch_apply(s.dim, s.k, s.kind, prec, op.variant, a, st);
  DOGIP_CHECK(ok, DOGIP_E_RANGE, "no apply kernel for this (dim, k, kind, variant)");
  if (timed) HIPCHK(hipEventRecord(ev[1], st));
  launch_apply_finish(stage, op.sh_pair.as<uint32_t>(), op.sh_more_off.as<uint32_t>(), op.sh_more.as<uint32_t>(),
                      op.shared.as<int32_t>(), int64_t(op.plan.shared.size()), op.bnd.as<int32_t>(),
                      int64_t(s.boundary.size()), u, y, energy ? energy + op.plan.ntiles : nullptr, st);
  HIPCHK(hipGetLastError());
  if (timed) HIPCHK(hipEventRecord(ev[2], st));
}

void op_apply(Op& op, const double* u, double* y, int prec, hipStream_t st, double* energy) {
  apply_impl(op, u, y, prec, st, energy, op.stage.as<double>());
}

int64_t op_stage_entries(const Op& op) { return op.plan.stage_off.empty() ? 0 : op.plan.stage_off.back(); }

void op_apply_staged(Op& op, const double* u, double* y, int prec, double* stage, hipStream_t st) {
  DOGIP_CHECK(stage != nullptr, DOGIP_E_NULL, "null staging buffer");
  apply_impl(op, u, y, prec, st, nullptr, stage);
}

bool op_has_v32(const Op& op) { return op.has32 && !op.global_w && op.nq == 0; }

void op_apply_v32(Op& op, const float* u, float* y, hipStream_t st, double* energy) {
  const Space& s = *op.space;
  DOGIP_CHECK(op_has_v32(op) && u && y && energy, DOGIP_E_STATE, "FP32-vector apply unavailable");
  ApplyLaunch a = apply_args(op, DOGIP_F32);
  a.u32 = u;
  a.y32 = y;
  a.energy = energy;
  DOGIP_CHECK(launch_apply(s.dim, s.k, s.kind, DOGIP_F32, op.variant, a, st), DOGIP_E_RANGE,
              "no apply kernel for this (dim, k, kind, variant)");
  launch_apply_finish32(op.stage.as<double>(), op.sh_pair.as<uint32_t>(), op.sh_more_off.as<uint32_t>(),
                        op.sh_more.as<uint32_t>(), op.shared.as<int32_t>(), int64_t(op.plan.shared.size()),
                        op.bnd.as<int32_t>(), int64_t(s.boundary.size()), u, y, energy + op.plan.ntiles, st);
  HIPCHK(hipGetLastError());
}

void op_diag(Op& op, double* diag, hipStream_t st) {
  const Space& s = *op.space;
  DOGIP_CHECK(diag != nullptr, DOGIP_E_NULL, "null output");
  // the tiles' partial sums of shared dofs go through the staging buffer and are added
  // by the finish kernel in a fixed order (no Dirichlet rows there: the tiles write those)
  auto finish = [&] {
    launch_apply_finish(op.stage.as<double>(), op.sh_pair.as<uint32_t>(), op.sh_more_off.as<uint32_t>(),
                        op.sh_more.as<uint32_t>(), op.shared.as<int32_t>(), int64_t(op.plan.shared.size()), nullptr,
                        0, nullptr, diag, nullptr, st);
    HIPCHK(hipGetLastError());
  };
  if (op.nq > 0) {
    launch_diag_qp(s.dim, s.k, s.kind, apply_args(op, DOGIP_F64), diag, st);
    HIPCHK(hipGetLastError());
    finish();
    return;
  }
  DiagLaunch a{};
  a.D = op.d64.as<double>();
  a.lidx = op.lidx.as<uint16_t>();
  a.tile_off = op.tile_off.as<int64_t>();
  a.tile_dofs = op.tile_dofs.as<uint32_t>();
  a.out = diag;
  a.nel = s.nc;
  a.ntiles = op.plan.ntiles;
  a.nch = op.nch64;
  a.nlc = op.plan.nlc;
  a.te = op.plan.te;
  a.cpl = 0;
  a.lds_slots = int(op.plan.max_tile_dofs);
  a.stage = op.stage.as<double>();
  a.stage_off = op.stage_off.as<int64_t>();
  if (op.global_w) {
    a.D = op.dg64.as<double>();
    a.gw_mask = op.gw_rec.as<uint32_t>();
    a.gw_woff = op.gw_off.as<int64_t>();
    launch_diag_global(s.dim, s.k, a, st);
  } else {
    launch_diag(s.dim, s.k, s.kind, a, st);
  }
  HIPCHK(hipGetLastError());
  finish();
}

void op_set_tile_lanes(Op& op, int lanes64, int lanes32) {
  const int te = op.plan.te;
  for (int l : {lanes64, lanes32})
    DOGIP_CHECK(l == 0 || (l > 0 && l <= 1024 && l % 64 == 0 && te % l == 0), DOGIP_E_RANGE,
                "lanes must be 0 or a multiple of 64 up to 1024 dividing the tile's cells");
  DOGIP_CHECK(op.variant != DOGIP_VARIANT_MFMA || lanes32 == 0 || lanes32 == te, DOGIP_E_RANGE,
              "the matrix-core apply takes one cell per lane");
  op.plan.lanes64 = lanes64;
  op.plan.lanes32 = lanes32;
}

void op_grad(Op& op, const double* u, const double* lam, double* g, hipStream_t st) {
  const Space& s = *op.space;
  DOGIP_CHECK(u && lam && g, DOGIP_E_NULL, "null vector");
  DOGIP_CHECK(!op.global_w && op.nq == 0, DOGIP_E_STATE, "the gradient contraction needs the element-wise D");
  GradLaunch a{};
  a.D = op.d64.as<double>();
  a.lidx = op.lidx.as<uint16_t>();
  a.tile_off = op.tile_off.as<int64_t>();
  a.tile_dofs = op.tile_dofs.as<uint32_t>();
  a.u = u;
  a.lam = lam;
  a.perm = op.perm.as<int32_t>();
  a.g = g;
  a.nel = s.nc;
  a.ntiles = op.plan.ntiles;
  a.nch = op.nch64;
  a.nlc = op.plan.nlc;
  a.te = op.plan.te;
  a.cpl = 0;
  a.lds_slots = int(op.plan.max_tile_dofs);
  launch_grad(s.dim, s.k, s.kind, a, st);
  HIPCHK(hipGetLastError());
}

void op_export_d(Op& op, double* out, hipStream_t st) {
  const Space& s = *op.space;
  DOGIP_CHECK(out != nullptr, DOGIP_E_NULL, "null output");
  DOGIP_CHECK(!op.global_w && op.nq == 0, DOGIP_E_STATE, "this operator holds no per-cell D");
  launch_export_d(op.d64.as<double>(), op.perm.as<int32_t>(), out, s.nc, op.nch64, s.wt, s.nsym, st);
  HIPCHK(hipGetLastError());
}

dogip_op_info op_info(const Op& op) {
  const Space& s = *op.space;
  dogip_op_info i{};
  i.tile_cells = op.plan.te;
  i.variant = op.variant;
  i.has_fp32 = op.has32;
  i.ntiles = op.plan.ntiles;
  i.tile_dofs_total = int64_t(op.plan.tile_dofs.size());
  i.nshared = int64_t(op.plan.shared.size());
  i.max_tile_dofs = op.plan.max_tile_dofs;
  i.bytes_d64 = int64_t(op.d64.bytes + op.dg64.bytes + op.qs64.bytes + op.qk64.bytes);
  i.bytes_d32 = int64_t(op.d32.bytes + op.dg32.bytes + op.qs32.bytes + op.qk32.bytes);
  i.bytes_index = int64_t(op.lidx.bytes + op.tile_off.bytes + op.tile_dofs.bytes + op.shared.bytes +
                          op.stage_off.bytes + op.sh_pair.bytes + op.sh_more_off.bytes + op.sh_more.bytes + op.stage.bytes +
                          op.gw_rec.bytes + op.gw_off.bytes + op.gw_inc_ptr.bytes + op.gw_inc.bytes);
  i.ndofs_w = op.global_w ? op.gplan.nw : 0;
  i.nq = op.nq;
  i.stage_entries = op_stage_entries(op);
  // values read per apply: D per cell and W node, D per global W dof, or (quadrature
  // points) one factor per cell and point plus the cell's R^-1 R^-T
  const double nd = op.nq > 0     ? (double(op.nq) + (s.kind == DOGIP_SE ? s.nsym : 0)) * s.nc
                    : op.global_w ? double(op.gplan.nw)
                                  : double(s.wt) * s.nsym * s.nc;
  const double conn = 4.0 * s.vt * s.nc, vec = 2.0 * 8.0 * s.ndofs;
  i.alg_bytes_f64 = 8.0 * nd + conn + vec;
  i.alg_bytes_f32 = 4.0 * nd + conn + vec;
  // multiplications per cell as counted in eq. comp_eff, two flops each
  const double mults = 2.0 * double(s.nnz_bhat - s.nnz_pm1) + double(s.kind == DOGIP_SE ? s.dim * s.dim : 1) * s.wt;
  i.alg_flops = 2.0 * mults * double(s.nc);
  if (op.nq > 0)  // dense tables: interpolation and projection at every point, plus the point product
    i.alg_flops = 2.0 * double(op.nq) * (2.0 * s.nb * s.vt + (s.kind == DOGIP_SE ? s.dim * s.dim : 1)) * s.nc;
  return i;
}

void op_timer_enable(Op& op, bool on) { op.timer->on = on; }

void op_timer_read(Op& op, double* tile_ms, double* finish_ms, int64_t* count) {
  double st = 0.0, sf = 0.0;
  for (size_t i = 0; i < op.timer->used; ++i) {
    const auto& e = op.timer->ev[i];
    HIPCHK(hipEventSynchronize(e[2]));
    float t0 = 0.f, t1 = 0.f;
    HIPCHK(hipEventElapsedTime(&t0, e[0], e[1]));
    HIPCHK(hipEventElapsedTime(&t1, e[1], e[2]));
    st += t0;
    sf += t1;
  }
  if (tile_ms) *tile_ms = st;
  if (finish_ms) *finish_ms = sf;
  if (count) *count = int64_t(op.timer->used);
  op.timer->clear();
}

}  // namespace dogip
