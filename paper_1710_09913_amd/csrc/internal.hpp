// Internal data structures of libdogip (host side).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dogip.h"

namespace dogip {

// Error carrying a status code; converted to the return value at the C boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DOGIP_CHECK(cond, code, msg)                 \
  do {                                               \
    if (!(cond)) throw ::dogip::Error((code), (msg)); \
  } while (0)

void hip_check(hipError_t e, const char* what);
#define HIPCHK(x) ::dogip::hip_check((x), #x)

// Device buffer owned by RAII.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  void alloc(size_t n);
  void free();
  ~DevBuf() { free(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Edges and (3D) faces of a mesh, numbered in the lexicographic order of their sorted
// vertex tuples: per cell and local entity the entity id, and the cells sharing each.
struct MeshEntities {
  std::vector<int32_t> cell_edge, edge_cells;  // [nc][(d+1)d/2], [ne]
  std::vector<int32_t> cell_face, face_cells;  // [nc][4] (face opposite local vertex j), [nf]
  int64_t ne = 0, nf = 0;
};

struct Mesh {
  int dim = 0;
  int64_t nv = 0, nc = 0;
  std::vector<double> xyz;     // [nv][dim]
  std::vector<int32_t> cells;  // [nc][dim+1]
  // n for the unit-cube mesh of n^dim cubes split into Kuhn simplices (make_unit_mesh),
  // whose halving is nested in it; 0 for other meshes
  int unit_n = 0;
  // built at the first space on this mesh and shared by the others (the orders of a
  // p-multigrid hierarchy, the double-grid lattice)
  mutable std::mutex ent_mu;
  mutable std::shared_ptr<const MeshEntities> ent;
  // cells in the Morton order of their centroids (the tile order of every operator on
  // this mesh), built once
  mutable std::shared_ptr<const std::vector<int32_t>> cell_order;
};
// the mesh's cell order, built once
std::shared_ptr<const std::vector<int32_t>> mesh_cell_order(const Mesh& m);
// the mesh's entities, built once
std::shared_ptr<const MeshEntities> mesh_entities(const Mesh& m);

struct Space {
  std::shared_ptr<const Mesh> mesh;
  int dim = 0, k = 0, kind = 0, bc = 0;
  int vt = 0, wt = 0, nsym = 0, nb = 0;
  int64_t nc = 0, ndofs = 0;
  std::vector<int32_t> cell_dofs;  // [nc][vt]
  std::vector<double> dof_xyz;     // [ndofs][dim]
  std::vector<int32_t> boundary;   // ascending
  std::vector<uint8_t> is_bnd;     // [ndofs]
  std::vector<double> bhat;        // [nb][wt][vt]
  std::vector<double> what;        // [wt]
  int64_t nnz_bhat = 0, nnz_pm1 = 0;
};

// Flags carried in the high bits of a tile dof entry.
constexpr uint32_t TD_BND = 0x80000000u;     // Dirichlet dof: gathered as 0, written y = u
constexpr uint32_t TD_SHARED = 0x40000000u;  // non-Dirichlet dof touched by several tiles: partial sum staged
constexpr uint32_t TD_OWNER = 0x20000000u;   // the tile of lowest index touching this dof
constexpr uint32_t TD_MASK = 0x1fffffffu;    // dof index (< 2^29)

// Cell tiling: cells reordered along a Morton curve of their centroids and cut
// into tiles of TE cells; each tile lists the distinct dofs it touches.
struct TilePlan {
  int te = 0;
  // lanes of the FP64 and FP32 apply workgroups: a tile of te cells runs on `lanes` lanes
  // in te / lanes passes; 0 lets each launch choose (tile_lanes)
  int lanes64 = 0, lanes32 = 0;
  int64_t ntiles = 0, nel_pad = 0;
  std::vector<int32_t> perm;        // internal cell -> mesh cell
  std::vector<int64_t> tile_off;    // [ntiles+1]
  std::vector<uint32_t> tile_dofs;  // dof | flags
  std::vector<uint16_t> lidx;       // AoSoA [nel_pad/64][nlc][64][8]: slot of each local node
  std::vector<int32_t> shared;      // non-boundary dofs touched by several tiles, ascending
  std::vector<int64_t> stage_off;   // [ntiles+1] staging offsets of each tile's shared entries
  std::vector<uint32_t> sh_rowptr;  // [nshared+1] staging slots of shared dof i: sh_slots[rowptr[i]..]
  std::vector<uint32_t> sh_slots;   // grouped by shared dof, ascending tile order
  // the same lists for the finish kernel (pair_lists): the first two slots of each shared
  // dof side by side, the others apart
  std::vector<uint32_t> sh_pair, sh_more_off, sh_more;
  int nlc = 0;                      // 16-byte chunks of local indices per cell
  int64_t max_tile_dofs = 0;
};

// D layout: AoSoA, cell e, flat value f = i*nsym + c at
//   ((e/64) * nch + f/vec) * 64 * vec + (e%64) * vec + f%vec,  vec = 16 / sizeof(value).
inline int64_t d_chunks(int wt, int nsym, int vec) { return (int64_t(wt) * nsym + vec - 1) / vec; }

// Global projection form (Theorem 1): one D value per global W dof (C_{N,2k}).  Each
// W dof is owned by one cell, the first in tile order holding it.  The W nodes inside
// one sub-simplex of a cell share their cells, hence their owner, so what a cell owns
// is a mask over its sub-simplex slots (ref::node_entity).  D is stored per wave of 64
// cells: for each slot s in order, for each node j of the slot (lattice order), the
// values of the lanes owning s, in lane order.  A lane finds node j of slot s at
// base_s + j * count_s + rank_s, with count_s and rank_s from a wave ballot of its
// ownership bit and base_s the running sum of (nodes of slot) * count over the slots
// before s.  Every owned value is read once per apply, by coalesced loads.
constexpr int gw_slots(int d) { return d == 2 ? 7 : 15; }
struct GlobalPlan {
  int64_t nw = 0;                  // global W dofs
  std::vector<uint32_t> mask;      // [nel_pad] owned slots per cell (internal order)
  std::vector<int64_t> woff;       // [nel_pad/64 + 1] wave ranges of D
  std::vector<int64_t> inc_ptr;    // [nw+1] cells holding each W dof (by position)
  std::vector<int64_t> inc;        // internal cell * W_T + local node, ascending
};
GlobalPlan make_global_plan(const Space& s, const TilePlan& p);

struct PcgWork;
struct OpTimer;
struct Pmg;

struct Op {
  std::shared_ptr<const Space> space;
  TilePlan plan;  // host copy (perm needed for outputs)
  int variant = 0;
  bool has32 = false;
  int64_t nch64 = 0, nch32 = 0;
  DevBuf d64, d32, lidx, tile_off, tile_dofs, shared, perm, cells, xyz, what, bhat64, bhat32, invdiag;
  DevBuf invdiag32;  // FP32 copy of the inverse diagonal (operators with DOGIP_OP_FP32)
  DevBuf stage_off, sh_pair, sh_more_off, sh_more, stage, bnd;  // second pass: shared dofs, Dirichlet rows
  bool global_w = false;                               // global projection form
  GlobalPlan gplan;
  int nq = 0;                                          // quadrature-point operator: points per cell
  DevBuf qtab64, qtab32, qs64, qs32, qk64, qk32, qw;
  DevBuf gw_rec, gw_off, gw_inc_ptr, gw_inc, dg64, dg32;
  std::unique_ptr<PcgWork> pcg;
  std::unique_ptr<OpTimer> timer;
  // the coefficient the D was built from (for the coarser operators of the p-multigrid
  // preconditioner); coef_kind_copy < 0 when D did not come from a coefficient form
  int coef_kind_copy = -1;
  DevBuf coef_copy;
  // or the inclusion coefficient D was built from by sub-cell quadrature (inc_depth >= 0)
  std::vector<double> inc_balls;
  double inc_in = 0.0, inc_out = 0.0;
  int inc_depth = -1, inc_ng = 0;
  std::unique_ptr<Pmg> pmg;  // p-multigrid hierarchy, built at the first multigrid solve
  ~Op();
};

// f(i) for i in [0, n) on up to 16 host threads (contiguous ranges); f must not throw
template <class F>
inline void parallel_for(int64_t n, F&& f) {
  const int64_t nt = std::min<int64_t>(std::max<unsigned>(1u, std::thread::hardware_concurrency()), 16);
  if (nt <= 1 || n < 2 * nt) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int64_t k = 0; k < nt; ++k)
    th.emplace_back([&f, k, chunk, n] {
      for (int64_t i = k * chunk; i < std::min(n, (k + 1) * chunk); ++i) f(i);
    });
  for (auto& x : th) x.join();
}

// f(t) for t in [0, ntasks), one host thread per task (ntasks small); f must not throw
template <class F>
inline void parallel_tasks(int64_t ntasks, F&& f) {
  if (ntasks <= 1) {
    if (ntasks == 1) f(0);
    return;
  }
  std::vector<std::thread> th;
  for (int64_t t = 0; t < ntasks; ++t) th.emplace_back([&f, t] { f(t); });
  for (auto& x : th) x.join();
}

// Global numbering of the order-q Lagrange nodes of a mesh (see setup.cpp).
struct LatticeDofs {
  int nl = 0;                      // nodes per cell
  int64_t ndofs = 0;
  std::vector<int32_t> cell_dofs;  // [nc][nl], local nodes in lattice order
  std::vector<double> xyz;         // [ndofs][dim] (when asked for)
  std::vector<uint8_t> is_bnd;     // [ndofs] on a boundary facet (when asked for)
};
LatticeDofs number_lattice(const Mesh& m, int q, bool xyz);

// Conventional quadrature-point apply: the collapsed (Duffy) Gauss-Legendre rule on the
// reference simplex with n points per direction (s outermost: x1 = s, x2 = t (1-s),
// x3 = v (1-s)(1-t)), exact for total degree <= 2n - d; and the V basis values (projection) or
// reference gradients (elliptic) at the points, [nq][nb][vt].
void collapsed_rule(int d, int n, std::vector<double>& pts, std::vector<double>& wts);
void basis_table(int d, int k, int kind, const std::vector<double>& pts, std::vector<double>& tab);
// Values of the order kf-1 basis at the order kf lattice nodes, [V_T(kf)][V_T(kf-1)]: the
// embedding of P_{kf-1} in P_kf on the reference cell (p-multigrid prolongation).
void coarse_basis_at_nodes(int d, int kf, std::vector<double>& tab);

// ---- host setup ----
std::shared_ptr<Mesh> make_mesh(int dim, int64_t nv, const double* xyz, int64_t nc, const int32_t* cells);
std::shared_ptr<Mesh> make_unit_mesh(int dim, int n);
std::shared_ptr<Space> make_space(std::shared_ptr<const Mesh> mesh, int k, int kind, int bc);
TilePlan make_tiles(const Space& s, int te);
void reference_tables(int dim, int k, int kind, std::vector<double>& bhat, std::vector<double>& what,
                      int64_t& nnz, int64_t& nnz_pm1);

// ---- operator ----
std::unique_ptr<Op> make_op(std::shared_ptr<const Space> s, int coef_kind, const double* coef, unsigned flags,
                            int tile_waves, int variant, hipStream_t st);
void op_set_coef(Op& op, int coef_kind, const double* coef, hipStream_t st);
// energy (optional): [ntiles] tile partials of u . A u, followed by op_finish_energy_count(op)
// partials of the Dirichlet rows
void op_apply(Op& op, const double* u, double* y, int prec, hipStream_t st, double* energy_partials = nullptr);
// partial sums an apply stages for shared dofs (the staging buffer's length in doubles)
int64_t op_stage_entries(const Op& op);
// the apply with a caller's staging buffer of at least op_stage_entries(op) doubles
// (device memory; the operator's own is left alone); allocates nothing
void op_apply_staged(Op& op, const double* u, double* y, int prec, double* stage, hipStream_t st);
// the apply with the library's per-device static staging buffer (noalloc.hip)
void op_apply_noalloc(Op& op, const double* u, double* y, int prec, hipStream_t st);
void op_diag(Op& op, double* diag, hipStream_t st);
void op_grad(Op& op, const double* u, const double* lam, double* g, hipStream_t st);
void op_set_tile_lanes(Op& op, int lanes64, int lanes32);
void op_export_d(Op& op, double* out, hipStream_t st);
dogip_op_info op_info(const Op& op);
int op_pcg(Op& op, const double* b, double* x, const dogip_solve_opts& o, dogip_solve_stats& stats, hipStream_t st);
void op_timer_enable(Op& op, bool on);
void op_timer_read(Op& op, double* tile_ms, double* finish_ms, int64_t* count);

// ---- kernel launchers (defined in the .hip files) ----
struct ApplyLaunch {
  const void* D;
  const uint16_t* lidx;
  const int64_t* tile_off;
  const uint32_t* tile_dofs;
  const void* bhat;      // looped variant: [nb][wt][vt] in the compute precision
  const double* u;
  double* y;
  const float* u32;      // FP32 vectors (mixed CG): used instead of u and y when set
  float* y32;
  double* energy;        // optional per-tile partial of u^T A u (nullptr: not computed)
  const int64_t* stage_off;  // [ntiles+1] staging offsets of the tiles' shared entries
  double* stage;             // staging buffer of shared partial sums
  int64_t nel;
  int64_t ntiles;
  int64_t nch;           // D chunks per cell
  int nlc;               // local-index chunks per cell
  int te;                // cells per tile
  int cpl;               // cells per lane (passes): the workgroup has te / cpl lanes; 0: chosen at launch
  int lds_slots;         // LDS slots per tile (>= max tile dofs)
  int tile_base;         // first tile of this launch (batch uses 0)
  const uint32_t* gw_mask;  // global projection form: owned slots per cell (else null)
  const int64_t* gw_woff;   // [waves+1] wave ranges of D (D then holds one value per W dof)
  // quadrature-point operator: basis table [nq][nb][vt], per-point factors
  // w_q |det R_T| a(x_q) AoSoA [(e/64)][nq][64], per-cell R^-1 R^-T packed AoSoA [(e/64)][s][64]
  const void* qtab;
  const void* qs;
  const void* qk;
  int nq;
};

// Dynamic LDS a tile kernel's workgroup may take (gfx950: 160 KB per compute unit and per
// workgroup, less a little for the kernels' static arrays).
constexpr int64_t LDS_TILE_MAX = 160 * 1024 - 1024;
// Lanes of a tile kernel's workgroup for tiles of te cells and `lds` bytes of dynamic LDS:
// `requested` when positive (checked: a multiple of 64 dividing te, within the kernel's
// launch bound), else the count that keeps the most waves resident per compute unit, ties
// going to fewer lanes (more, smaller workgroups); cached per (kernel, te, lds).  Passes
// take a tile's cells in ascending order whatever the lanes, so results do not depend on it.
int tile_lanes(const void* kernel, int te, size_t lds, int requested);
bool launch_apply(int dim, int k, int kind, int prec, int variant, const ApplyLaunch& a, hipStream_t st);
// FP32 apply of 3D P3 elliptic operators with the B^ products on the matrix cores
// (kern_apply_mfma.hip); D32 in the layout of d32_pos with nch32 < 0
bool launch_apply_mfma(bool energy, const ApplyLaunch& a, hipStream_t st);
int64_t mfma_d32_per_wave();
int64_t mfma_lds_tables();  // bytes of LDS the matrix-core kernel adds to a tile's arrays
bool has_mfma(int dim, int k, int kind);
bool launch_apply_global(int dim, int k, int prec, int variant, const ApplyLaunch& a, hipStream_t st);
bool has_unrolled(int dim, int k, int kind);
bool has_factored(int dim, int k, int kind);
// host copies of the factored elliptic B^ tables (DOGIP_VARIANT_FACTORED); false if none
bool factored_tables(int dim, int k, double* b1, double* b2);

struct DiagLaunch {
  const double* D;
  const uint16_t* lidx;
  const int64_t* tile_off;
  const uint32_t* tile_dofs;
  const double* bhat;
  double* out;
  int64_t nel, ntiles, nch;
  int nlc, te, cpl, lds_slots;  // cells per tile, cells per lane (0: chosen at launch)
  const uint32_t* gw_mask;  // global projection form (D one value per W dof), else null
  const int64_t* gw_woff;
  double* stage;             // the apply's staging buffer: tile partials of shared dofs
  const int64_t* stage_off;
};
void launch_diag(int dim, int k, int kind, const DiagLaunch& a, hipStream_t st);
void launch_diag_global(int dim, int k, const DiagLaunch& a, hipStream_t st);

// Quadrature-point operator: per-point factors and per-cell geometry from the samples.
struct QpSetupLaunch {
  const double* xyz;
  const int32_t* cells;  // internal order
  const int32_t* perm;
  const double* coef;    // [ncells][nq] samples a(x_q), mesh order
  const double* w;       // [nq] reference weights
  double* qs64;
  float* qs32;           // may be null
  double* qk64;          // elliptic only
  float* qk32;
  int64_t nel;
  int nq, dim, kind;
};
void launch_qp_setup(const QpSetupLaunch& a, hipStream_t st);
bool launch_apply_qp(int dim, int k, int kind, int prec, const ApplyLaunch& a, hipStream_t st);
void launch_diag_qp(int dim, int k, int kind, const ApplyLaunch& a, double* out, hipStream_t st);
std::unique_ptr<Op> make_op_qp(std::shared_ptr<const Space> s, int n, const double* coef, unsigned flags,
                               int tile_waves, hipStream_t st);

struct GradLaunch {
  const double* D;
  const uint16_t* lidx;
  const int64_t* tile_off;
  const uint32_t* tile_dofs;
  const double* bhat;
  const double* u;
  const double* lam;
  const int32_t* perm;
  double* g;
  int64_t nel, ntiles, nch;
  int nlc, te, cpl, lds_slots;  // cells per tile, cells per lane (0: chosen at launch)
};
void launch_grad(int dim, int k, int kind, const GradLaunch& a, hipStream_t st);

struct BuildDLaunch {
  const double* xyz;
  const int32_t* cells;  // internal order [nel][dim+1]
  const int32_t* perm;   // internal -> mesh cell
  const double* what;    // [wt]
  const double* coef;
  double* d64;
  float* d32;            // may be null
  int64_t nel, nel_pad, nch64, nch32;  // nch32 < 0: the matrix-core layout of D32 (d32_pos)
  int dim, kind, coef_kind, wt, nsym;
};
void launch_build_d(const BuildDLaunch& a, hipStream_t st);

// D for an inclusion coefficient by sub-cell quadrature (kern_subcell.hip).
struct SubLaunch {
  const double* xyz;
  const int32_t* cells;  // internal order
  const double* balls;   // [nballs][dim+1]: center, radius
  const double* gpts;    // [ng][dim] reference rule of the leaves
  const double* gwts;    // [ng]
  const double* what;    // [wt]
  double* d64;
  float* d32;            // may be null
  double* npts;          // optional [nel]: points evaluated per cell
  double a_in, a_out;
  int64_t nel, nch64, nch32;
  int nballs, ng, depth, kind;
};
void launch_build_d_sub(int dim, int q, const SubLaunch& a, hipStream_t st);
void op_set_inclusions(Op& op, int nballs, const double* balls, double a_in, double a_out, int depth, int ng,
                       double* mean_points, hipStream_t st);
// Global projection form: D at position j (tile layout) = sum over inc[inc_ptr[j] ..
// inc_ptr[j+1]) (internal cell * wt + node) of the cell's integral of m phi^W_node.
void launch_build_dg(const BuildDLaunch& a, const int64_t* inc_ptr, const int64_t* inc, int64_t nw, double* dg64,
                     float* dg32, hipStream_t st);
void launch_export_d(const double* d64, const int32_t* perm, double* out, int64_t nel, int64_t nch64, int wt,
                     int nsym, hipStream_t st);
void launch_zero_indexed(double* y, const int32_t* idx, int64_t n, hipStream_t st);
// Second pass of an apply: y[shared[i]] = the sum of shared dof i's staged partials in
// ascending tile order (fixed order) and y[b] = u[b] on Dirichlet dofs; with benergy, the
// sums of u_b^2 per block of the Dirichlet range (finish_energy_count of them).
// The partials' slots come as pair lists: pair[2i], pair[2i+1] are the first two slots
// (every shared dof has at least two); bit 31 of pair[2i+1] set means more follow, at
// more[more_off[i] .. more_off[i+1]).  One dependent load fewer than a CSR walk.
void pair_lists(const std::vector<uint32_t>& rowptr, const std::vector<uint32_t>& slots, std::vector<uint32_t>& pair,
                std::vector<uint32_t>& more_off, std::vector<uint32_t>& more);
// Each thread of the finish handles FINISH_PER_THREAD entries, FINISH_THREADS apart, so a
// block covers FINISH_ENTRIES consecutive entries and a thread's loads are independent.
constexpr int FINISH_THREADS = 256, FINISH_PER_THREAD = 4, FINISH_ENTRIES = FINISH_THREADS * FINISH_PER_THREAD;
inline int64_t finish_blocks(int64_t nshared, int64_t nbnd) {
  return std::max<int64_t>(1, (nshared + nbnd + FINISH_ENTRIES - 1) / FINISH_ENTRIES);
}
inline int64_t finish_first_energy_block(int64_t nshared, int64_t nbnd) {
  return std::min(nshared / FINISH_ENTRIES, finish_blocks(nshared, nbnd) - 1);
}
inline int64_t finish_energy_count(int64_t nshared, int64_t nbnd) {
  return finish_blocks(nshared, nbnd) - finish_first_energy_block(nshared, nbnd);
}
inline int64_t op_finish_energy_count(const Op& op) {
  return finish_energy_count(int64_t(op.plan.shared.size()), int64_t(op.space->boundary.size()));
}
void launch_apply_finish(const double* stage, const uint32_t* pair, const uint32_t* more_off, const uint32_t* more,
                         const int32_t* shared, int64_t nshared, const int32_t* bnd, int64_t nbnd, const double* u,
                         double* y, double* benergy, hipStream_t st);
void launch_invert(const double* d, double* inv, int64_t n, hipStream_t st);
void launch_to_f32(const double* x, float* y, int64_t n, hipStream_t st);
// FP32 apply on FP32 vectors with the energy partials (the mixed CG iteration):
// y32 = A32 u32, energy as op_apply.
void op_apply_v32(Op& op, const float* u, float* y, hipStream_t st, double* energy_partials);
bool op_has_v32(const Op& op);
void launch_apply_finish32(const double* stage, const uint32_t* pair, const uint32_t* more_off, const uint32_t* more,
                           const int32_t* shared, int64_t nshared, const int32_t* bnd, int64_t nbnd, const float* u,
                           float* y, double* benergy, hipStream_t st);

}  // namespace dogip
