// Batched operators: many independent problems applied and solved together.
#pragma once

#include <memory>
#include <vector>

#include "internal.hpp"
#include "solve.hpp"

namespace dogip {

// Device descriptor of one problem of a batch.
struct BatchDesc {
  const void* D64;
  const void* D32;
  const uint16_t* lidx;
  const int64_t* tile_off;
  const uint32_t* tile_dofs;
  const int64_t* stage_off;
  int64_t nel, ntiles, nch64, nch32;
  int64_t voff;        // offset of the problem's dofs in the concatenated vectors
  int64_t stage_base;  // offset of its staging entries in the batch staging buffer
  int64_t tile_base;   // offset of its tiles in the batch tile numbering
  int nlc, te, lds_slots, k;
};

struct BatchLaunch {
  const BatchDesc* desc;
  const uint64_t* items;  // (problem << 32) | tile, largest work first
  uint32_t* counter;      // work-queue head, reset before every launch
  int64_t nitems;
  const double* u;
  double* y;
  const float* u32;       // FP32 vectors (mixed CG): used instead of u and y when set
  float* y32;
  double* stage;
  double* energy;         // [total tiles] tile energies (ENERGY launches)
  const int* active;      // optional: skip problems with active[p] == 0
  const int* mask;        // optional: skip problems with mask[p] != mask_val
  int mask_val;
  int prec;
};

// Per-problem CG state on the device.
struct BatchPcgState {
  PcgScalars* sc;
  double* rr_true;
  int* iters;
  int* need;    // residual replacement requested
  int* stalls;
  int* active;
  int* state;     // 0 running, 1 converged, 2 failed (breakdown or non-finite)
  int* use64;     // mixed mode: the problem switched to the FP64 apply
  int* last_rep;  // iteration count at the last replacement
  double* rr_min; // smallest true residual norm^2 so far
};

struct BatchVecArgs {
  const int64_t* voff;
  const double* invd;
  double* r;
  double* p;
  bool v32;             // mixed CG: r, p (and A p) stored in FP32
  bool stream;          // vectors used once per iteration read and written non-temporally (stream_vectors)
  const float* invd32;
  float* r32;
  float* p32;
  double* part;  // [np][gx][3]
  BatchPcgState s;
  const int* act;  // problems the per-iteration kernels work on
  int nact;
  int gx, np;
  double tol;
};

struct BatchWork;

struct Batch {
  std::vector<std::shared_ptr<Op>> ops;
  std::vector<int64_t> offsets;  // dof offsets of the concatenated vectors [nops+1]
  int dim = 2, kind = 0;
  int64_t ntiles_total = 0, nitems = 0, nshared = 0, nbnd = 0;
  size_t lds64 = 0, lds32 = 0;
  unsigned grid64 = 0, grid32 = 0;
  DevBuf desc, items, counter, voff, stage, tile_base, shared, rowptr, slots, bnd, bnd_off, invd, sh_off;
  DevBuf pair, more_off, more;  // the shared-dof lists as pair lists (apply's finish kernel)
  DevBuf invd32;  // FP32 copy of invd (all operators with DOGIP_OP_FP32)
  std::vector<uint64_t> items_host;  // work items, largest first
  std::unique_ptr<BatchWork> w;
  ~Batch();
};

std::unique_ptr<Batch> make_batch(const std::vector<std::shared_ptr<Op>>& ops, hipStream_t st);
void batch_apply(Batch& b, const double* u, double* y, int prec, hipStream_t st);
int batch_pcg(Batch& b, const double* rhs, double* x, const dogip_solve_opts& o, dogip_solve_stats* stats,
              hipStream_t st);

// kernel launchers (kern_batch.hip)
void launch_batch_apply(int dim, int kind, const BatchLaunch& bl, unsigned grid, size_t lds, bool energy,
                        hipStream_t st);
int batch_blocks_per_cu(int dim, int kind, int prec, size_t lds);
void bk_init(const BatchVecArgs& v, const double* b, double* x, hipStream_t st);
void bk_fin_pq(const BatchVecArgs& v, const double* energy, const int64_t* tile_base, const int32_t* bnd,
               const int64_t* bnd_off, hipStream_t st);
void bk_xr(const BatchVecArgs& v, double* x, const void* q, hipStream_t st);
void bk_fin_rz(const BatchVecArgs& v, double delta, int mixed, hipStream_t st);
void bk_p(const BatchVecArgs& v, hipStream_t st);
void bk_replace(const BatchVecArgs& v, const double* b, const double* y, int mixed, hipStream_t st);
void bk_resid(const BatchVecArgs& v, const double* b, const double* y, double* out, hipStream_t st);
// u, y: double, or float when f32
void bk_finish(const BatchVecArgs& v, const int* act, int nact, const double* stage, const uint32_t* rowptr,
               const uint32_t* slots, const int32_t* shared, const int64_t* sh_off, const int32_t* bnd,
               const int64_t* bnd_off, const void* u, void* y, bool f32, hipStream_t st);

}  // namespace dogip
