// Batched operators: one persistent launch applies many independent problems, and
// segmented vector kernels run one CG per problem with per-problem scalars.
#include "batch.hpp"
#include "kern_apply.hpp"
#include "solve.hpp"

namespace dogip {
namespace dev {

// Persistent apply: every workgroup takes (problem, tile) items from a queue
// (largest work first) until the queue is exhausted; problems whose flag in
// `active` (or `mask`) is zero are skipped.
template <int D, int KIND, typename T, bool ENERGY, bool V32 = false>
__global__ __launch_bounds__(256) void k_batch_apply(BatchLaunch bl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t cur;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(bl.counter, 1u);
    __syncthreads();
    const uint32_t it = cur;
    __syncthreads();
    if (it >= bl.nitems) break;
    const uint64_t item = bl.items[it];
    const int p = int(item >> 32);
    const int64_t t = int64_t(item & 0xffffffffu);
    if ((bl.active && !bl.active[p]) || (bl.mask && bl.mask[p] != bl.mask_val)) continue;
    const BatchDesc& d = bl.desc[p];
    ApplyLaunch a{};
    a.D = bl.prec == DOGIP_F64 ? d.D64 : d.D32;
    a.lidx = d.lidx;
    a.tile_off = d.tile_off;
    a.tile_dofs = d.tile_dofs;
    if constexpr (V32) {
      a.u32 = bl.u32 + d.voff;
      a.y32 = bl.y32 + d.voff;
    } else {
      a.u = bl.u + d.voff;
      a.y = bl.y + d.voff;
    }
    a.stage_off = d.stage_off;
    a.stage = bl.stage + d.stage_base;
    a.nel = d.nel;
    a.ntiles = d.ntiles;
    a.nch = bl.prec == DOGIP_F64 ? d.nch64 : d.nch32;
    a.nlc = d.nlc;
    a.te = d.te;
    a.cpl = 1;
    a.lds_slots = d.lds_slots;
    double* eo = ENERGY ? bl.energy + d.tile_base + t : nullptr;
    constexpr int V = DOGIP_VARIANT_UNROLLED;
    constexpr int PF = sizeof(T) == 8 ? DOGIP_PF64 : DOGIP_PF32;
    switch (d.k) {
      case 1: tile_body<D, 1, KIND, T, V, ENERGY, PF, 0, V32, false>(a, t, smem, eo); break;
      case 2: tile_body<D, 2, KIND, T, V, ENERGY, PF, 0, V32, false>(a, t, smem, eo); break;
      case 3: tile_body<D, 3, KIND, T, V, ENERGY, PF, 0, V32, false>(a, t, smem, eo); break;
      default: tile_body<D, 4, KIND, T, V, ENERGY, PF, 0, V32, false>(a, t, smem, eo); break;
    }
    __syncthreads();
  }
}

__global__ void k_reset_counter(uint32_t* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0u;
}

__device__ __forceinline__ int p_of(const int* act) { return act ? act[blockIdx.y] : int(blockIdx.y); }

__device__ __forceinline__ double bwave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block partials of up to 3 sums: part[(p * gridDim.x + blockIdx.x) * 3 + c].
__device__ __forceinline__ void bpartials(const double* v, int nc, double* part, int p) {
  __shared__ double red[3][4];
  const int w = threadIdx.x >> 6;
  for (int c = 0; c < nc; ++c) {
    const double s = bwave_sum(v[c]);
    if ((threadIdx.x & 63) == 0) red[c][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < nc; ++c) part[(int64_t(p) * gridDim.x + blockIdx.x) * 3 + c] = red[c][0] + red[c][1] + red[c][2] + red[c][3];
}

// Sum of n values with one 256-thread block (fixed order); result in thread 0.
__device__ __forceinline__ double bsum(const double* x, int64_t n, int64_t stride) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i * stride];
  s = bwave_sum(s);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

// blockIdx.y indexes the list act of problems (all problems when act is null)
#define PROBLEM_RANGE(p, lo, hi)               \
  const int p = act ? act[blockIdx.y] : int(blockIdx.y); \
  const int64_t lo = voff[p], hi = voff[p + 1]; \
  for (int64_t i = lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < hi; i += int64_t(gridDim.x) * blockDim.x)

// r = b, z = invd r, p = z; partials (r.z, r.r, b.b).  V: storage type of r, p and
// invd (FP32 in the mixed CG; the arithmetic and sums stay FP64, each value rounded once).
template <typename V>
__global__ __launch_bounds__(256) void k_b_init(const int* __restrict__ act, const int64_t* __restrict__ voff, const double* __restrict__ b,
                                                const V* __restrict__ invd, V* __restrict__ r,
                                                V* __restrict__ pv, double* __restrict__ x,
                                                double* __restrict__ part) {
  double v[3] = {0.0, 0.0, 0.0};
  PROBLEM_RANGE(p, lo, hi) {
    const double bi = b[i];
    const V ri = V(bi);
    const double zi = double(invd[i]) * double(ri);
    r[i] = ri;
    pv[i] = V(zi);
    x[i] = 0.0;
    v[0] += double(ri) * zi;
    v[1] += double(ri) * double(ri);
    v[2] += bi * bi;
  }
  bpartials(v, 3, part, p_of(act));
}

__global__ __launch_bounds__(256) void k_b_fin_init(const double* __restrict__ part, int gx, BatchPcgState s,
                                                    double tol) {
  const int p = blockIdx.x;
  const double rz = bsum(part + int64_t(p) * gx * 3 + 0, gx, 3);
  const double rr = bsum(part + int64_t(p) * gx * 3 + 1, gx, 3);
  const double bb = bsum(part + int64_t(p) * gx * 3 + 2, gx, 3);
  if (threadIdx.x == 0) {
    PcgScalars& c = s.sc[p];
    c.rho = rz;
    c.rr = rr;
    c.bb = bb;
    c.flags = (isfinite(rz) && isfinite(rr) && isfinite(bb)) ? 0 : PCG_NONFINITE;
    s.rr_true[p] = rr;
    s.rr_min[p] = rr;
    s.iters[p] = 0;
    s.need[p] = 0;
    s.stalls[p] = 0;
    s.use64[p] = 0;
    s.last_rep[p] = 0;
    s.active[p] = (c.flags == 0 && rr > tol * tol * bb) ? 1 : 0;
    s.state[p] = c.flags ? 2 : (s.active[p] ? 0 : 1);
  }
}

// pq = sum of the problem's tile energies + p_b^2 over its Dirichlet dofs; alpha = rho / pq
template <typename V>
__global__ __launch_bounds__(256) void k_b_fin_pq(const int* __restrict__ act, const double* __restrict__ energy,
                                                  const int64_t* __restrict__ tile_base, const int32_t* __restrict__ bnd,
                                                  const int64_t* __restrict__ bnd_off, const V* __restrict__ pv,
                                                  BatchPcgState s) {
  const int p = act[blockIdx.x];
  if (!s.active[p]) return;
  const double e = bsum(energy + tile_base[p], tile_base[p + 1] - tile_base[p], 1);
  __shared__ double red[4];
  double q = 0.0;
  for (int64_t i = bnd_off[p] + threadIdx.x; i < bnd_off[p + 1]; i += blockDim.x) {
    const double v = double(pv[bnd[i]]);
    q += v * v;
  }
  q = bwave_sum(q);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double pq = e + red[0] + red[1] + red[2] + red[3];
    PcgScalars& c = s.sc[p];
    c.pq = pq;
    if (!isfinite(pq))
      c.flags |= PCG_NONFINITE;
    else if (!(pq > 0.0))
      c.flags |= PCG_BREAKDOWN;
    c.alpha = c.flags ? 0.0 : c.rho / pq;
    if (c.flags) {
      s.active[p] = 0;
      s.state[p] = 2;
    }
  }
}

// a vector element that an iteration reads once: non-temporal for FP64 vectors when S
// (the host's stream_vectors over the whole batch)
template <bool S, typename V>
__device__ __forceinline__ V streamed(const V* a) {
  if constexpr (S && sizeof(V) == 8)
    return __builtin_nontemporal_load(a);
  else
    return *a;
}

template <typename V, bool S>
__global__ __launch_bounds__(256) void k_b_xr(const int* __restrict__ act, const int64_t* __restrict__ voff,
                                              double* __restrict__ x, V* __restrict__ r,
                                              const V* __restrict__ pv, const V* __restrict__ q,
                                              const V* __restrict__ invd, BatchPcgState s,
                                              double* __restrict__ part) {
  if (!s.active[p_of(act)]) return;
  const double alpha = s.sc[p_of(act)].alpha;
  double v[2] = {0.0, 0.0};
  PROBLEM_RANGE(p, lo, hi) {
    // with S the iterate, read and written once per iteration, is non-temporal, so that the
    // memory-side cache keeps the index arrays and directions of the next apply; with FP64
    // vectors A p and the inverse diagonal too (batched FP64 PCG 0.8% faster; with FP32
    // vectors, which the cache holds more easily, they stay cached)
    if constexpr (S)
      __builtin_nontemporal_store(fma(alpha, double(pv[i]), __builtin_nontemporal_load(x + i)), x + i);
    else
      x[i] = fma(alpha, double(pv[i]), x[i]);
    const V ri = V(fma(-alpha, double(streamed<S>(q + i)), double(r[i])));
    r[i] = ri;
    v[0] += double(ri) * (double(streamed<S>(invd + i)) * double(ri));
    v[1] += double(ri) * double(ri);
  }
  bpartials(v, 2, part, p_of(act));
}

__global__ __launch_bounds__(256) void k_b_fin_rz(const int* __restrict__ act, const double* __restrict__ part, int gx,
                                                  BatchPcgState s, double tol, double delta, int mixed) {
  const int p = act[blockIdx.x];
  if (!s.active[p]) return;
  const double rz = bsum(part + int64_t(p) * gx * 3 + 0, gx, 3);
  const double rr = bsum(part + int64_t(p) * gx * 3 + 1, gx, 3);
  if (threadIdx.x == 0) {
    PcgScalars& c = s.sc[p];
    if (!isfinite(rz) || !isfinite(rr)) c.flags |= PCG_NONFINITE;
    c.beta = (c.rho != 0.0 && c.flags == 0) ? rz / c.rho : 0.0;
    c.rho = rz;
    c.rr = rr;
    s.iters[p] += 1;
    const double thr = tol * tol * c.bb;
    if (c.flags) {
      s.active[p] = 0;
      s.state[p] = 2;
    } else if (rr <= thr) {
      s.need[p] = 2;  // apparent convergence: verify on the FP64 residual (and restart the direction)
    } else if (mixed && !s.use64[p] && s.need[p] == 0 &&
               (rr <= delta * delta * s.rr_true[p] || s.iters[p] - s.last_rep[p] >= 512)) {
      s.need[p] = 1;  // FP32 directions: replace the residual (keep the direction) after a reduction
                      // by delta, and at least every 512 iterations
    }
  }
}

template <typename V, bool S>
__global__ __launch_bounds__(256) void k_b_p(const int* __restrict__ act, const int64_t* __restrict__ voff,
                                             V* __restrict__ pv, const V* __restrict__ r,
                                             const V* __restrict__ invd, BatchPcgState s) {
  if (!s.active[p_of(act)]) return;
  const double beta = s.sc[p_of(act)].beta;
  PROBLEM_RANGE(p, lo, hi) pv[i] = V(fma(beta, double(pv[i]), double(streamed<S>(invd + i)) * double(r[i])));
}

// residual replacement for problems with need[p]: r = b - A64 x (the true r.r from the
// unrounded FP64 residual)
template <typename V>
__global__ __launch_bounds__(256) void k_b_replace(const int* __restrict__ act, const int64_t* __restrict__ voff,
                                                   const double* __restrict__ b, const double* __restrict__ y,
                                                   const V* __restrict__ invd, V* __restrict__ r,
                                                   V* __restrict__ pv, BatchPcgState s,
                                                   double* __restrict__ part) {
  if (!s.active[p_of(act)] || !s.need[p_of(act)]) return;
  const bool restart = s.need[p_of(act)] >= 2;
  double v[2] = {0.0, 0.0};
  PROBLEM_RANGE(p, lo, hi) {
    const double rd = b[i] - y[i];
    const V ri = V(rd);
    const double zi = double(invd[i]) * double(ri);
    r[i] = ri;
    if (restart) pv[i] = V(zi);
    v[0] += double(ri) * zi;
    v[1] += rd * rd;
  }
  bpartials(v, 2, part, p_of(act));
}

__global__ __launch_bounds__(256) void k_b_fin_replace(const int* __restrict__ act, const double* __restrict__ part,
                                                       int gx, BatchPcgState s, double tol, int mixed) {
  const int p = act[blockIdx.x];
  if (!s.active[p] || !s.need[p]) return;
  const double rz = bsum(part + int64_t(p) * gx * 3 + 0, gx, 3);
  const double rr = bsum(part + int64_t(p) * gx * 3 + 1, gx, 3);
  if (threadIdx.x == 0) {
    PcgScalars& c = s.sc[p];
    if (s.need[p] == 3) {
      // the direction restart that follows a replacement with a gap (see below): the
      // same residual again, no bookkeeping
      c.rho = rz;
      s.need[p] = 0;
      return;
    }
    if (!isfinite(rz) || !isfinite(rr)) c.flags |= PCG_NONFINITE;
    const bool gap = rr > GAP_RR * fmax(c.rr, 1e-300);
    if (mixed && !s.use64[p]) {
      // FP32 operator: a stall is a true residual well above the recursive one (the
      // FP32 error dominates); a true residual far above its minimum is divergence
      const bool diverged = rr > DIVERGE_RR * s.rr_min[p];
      s.stalls[p] = diverged ? 3 : (gap ? s.stalls[p] + 1 : 0);
    } else {
      s.stalls[p] = rr > 0.25 * s.rr_true[p] ? s.stalls[p] + 1 : 0;
    }
    s.rr_min[p] = fmin(s.rr_min[p], rr);
    c.rho = rz;
    c.rr = rr;
    s.rr_true[p] = rr;
    // a recursive residual far below the true one no longer describes the iterate (it lost
    // its accuracy, or the Krylov space ran out and the last steps ran on rounding noise):
    // the kept direction belongs to it, so a second pass restarts the direction from the
    // true residual (need 3)
    s.need[p] = (gap && s.need[p] == 1 && !c.flags && rr > tol * tol * c.bb) ? 3 : 0;
    s.last_rep[p] = s.iters[p];
    if (c.flags) {
      s.active[p] = 0;
      s.state[p] = 2;
    } else if (rr <= tol * tol * c.bb) {
      s.active[p] = 0;
      s.state[p] = 1;
    } else if (mixed && !s.use64[p]) {
      if (s.stalls[p] >= 3) {
        s.use64[p] = 1;  // the FP32 operator stopped reducing the true residual: continue in FP64
        s.stalls[p] = 0;
      }
    } else if (s.stalls[p] >= 2) {
      s.active[p] = 0;  // below the attainable accuracy: stop, reported as not converged
    }
  }
}

// per-problem ||b - y||^2 (final check)
__global__ __launch_bounds__(256) void k_b_resid(const int* __restrict__ act, const int64_t* __restrict__ voff,
                                                 const double* __restrict__ b, const double* __restrict__ y,
                                                 double* __restrict__ part) {
  double v[1] = {0.0};
  PROBLEM_RANGE(p, lo, hi) {
    const double d = b[i] - y[i];
    v[0] += d * d;
  }
  bpartials(v, 1, part, p_of(act));
}

// Second pass of a batched apply restricted to the problems in act: shared-dof sums
// and Dirichlet rows of each listed problem.
template <typename V>
__global__ __launch_bounds__(256) void k_b_finish(const int* __restrict__ act, const double* __restrict__ stage,
                                                  const uint32_t* __restrict__ rowptr, const uint32_t* __restrict__ slots,
                                                  const int32_t* __restrict__ shared, const int64_t* __restrict__ sh_off,
                                                  const int32_t* __restrict__ bnd, const int64_t* __restrict__ bnd_off,
                                                  const V* __restrict__ u, V* __restrict__ y) {
  const int p = act[blockIdx.y];
  const int64_t s0 = sh_off[p], s1 = sh_off[p + 1], b0 = bnd_off[p], b1 = bnd_off[p + 1];
  const int64_t n = (s1 - s0) + (b1 - b0);
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) {
    if (k < s1 - s0) {
      const int64_t i = s0 + k;
      double acc = 0.0;
      for (uint32_t j = rowptr[i]; j < rowptr[i + 1]; ++j) acc += stage[slots[j]];
      y[shared[i]] = V(acc);
    } else {
      const int32_t d = bnd[b0 + k - (s1 - s0)];
      y[d] = u[d];
    }
  }
}

__global__ __launch_bounds__(256) void k_b_fin_resid(const double* __restrict__ part, int gx, double* out) {
  const double t = bsum(part + int64_t(blockIdx.x) * gx * 3, gx, 3);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

template <int D, int KIND>
void batch_apply_t(const BatchLaunch& bl, unsigned grid, size_t lds, bool energy, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, bl.counter);
  if (bl.u32) {  // FP32 vectors: the CG iteration (energy partials always taken)
    if (bl.prec == DOGIP_F64)
      hipLaunchKernelGGL((k_batch_apply<D, KIND, double, true, true>), dim3(grid), dim3(256), lds, st, bl);
    else
      hipLaunchKernelGGL((k_batch_apply<D, KIND, float, true, true>), dim3(grid), dim3(256), lds, st, bl);
    return;
  }
  if (bl.prec == DOGIP_F64) {
    if (energy)
      hipLaunchKernelGGL((k_batch_apply<D, KIND, double, true>), dim3(grid), dim3(256), lds, st, bl);
    else
      hipLaunchKernelGGL((k_batch_apply<D, KIND, double, false>), dim3(grid), dim3(256), lds, st, bl);
  } else {
    if (energy)
      hipLaunchKernelGGL((k_batch_apply<D, KIND, float, true>), dim3(grid), dim3(256), lds, st, bl);
    else
      hipLaunchKernelGGL((k_batch_apply<D, KIND, float, false>), dim3(grid), dim3(256), lds, st, bl);
  }
}

template <int D, int KIND>
int batch_occupancy(int prec, size_t lds) {
  int n = 0;
  if (prec == DOGIP_F64)
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_batch_apply<D, KIND, double, true>), 256, lds));
  else
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (k_batch_apply<D, KIND, float, true>), 256, lds));
  return n;
}

}  // namespace dev

void launch_batch_apply(int dim, int kind, const BatchLaunch& bl, unsigned grid, size_t lds, bool energy,
                        hipStream_t st) {
  DOGIP_CHECK(dim == 2, DOGIP_E_RANGE, "batched launches are built for 2D problems");
  if (kind == KIND_SE)
    dev::batch_apply_t<2, KIND_SE>(bl, grid, lds, energy, st);
  else
    dev::batch_apply_t<2, KIND_WP>(bl, grid, lds, energy, st);
}

int batch_blocks_per_cu(int dim, int kind, int prec, size_t lds) {
  DOGIP_CHECK(dim == 2, DOGIP_E_RANGE, "batched launches are built for 2D problems");
  return kind == KIND_SE ? dev::batch_occupancy<2, KIND_SE>(prec, lds) : dev::batch_occupancy<2, KIND_WP>(prec, lds);
}

void bk_init(const BatchVecArgs& v, const double* b, double* x, hipStream_t st) {
  if (v.v32)
    hipLaunchKernelGGL(dev::k_b_init<float>, dim3(v.gx, v.np), dim3(256), 0, st, nullptr, v.voff, b, v.invd32, v.r32,
                       v.p32, x, v.part);
  else
    hipLaunchKernelGGL(dev::k_b_init<double>, dim3(v.gx, v.np), dim3(256), 0, st, nullptr, v.voff, b, v.invd, v.r,
                       v.p, x, v.part);
  hipLaunchKernelGGL(dev::k_b_fin_init, dim3(v.np), dim3(256), 0, st, v.part, v.gx, v.s, v.tol);
}
void bk_fin_pq(const BatchVecArgs& v, const double* energy, const int64_t* tile_base, const int32_t* bnd,
               const int64_t* bnd_off, hipStream_t st) {
  if (v.v32)
    hipLaunchKernelGGL(dev::k_b_fin_pq<float>, dim3(v.nact), dim3(256), 0, st, v.act, energy, tile_base, bnd, bnd_off,
                       v.p32, v.s);
  else
    hipLaunchKernelGGL(dev::k_b_fin_pq<double>, dim3(v.nact), dim3(256), 0, st, v.act, energy, tile_base, bnd, bnd_off,
                       v.p, v.s);
}
void bk_xr(const BatchVecArgs& v, double* x, const void* q, hipStream_t st) {
  const dim3 g(v.gx, v.nact);
  const auto* q32 = static_cast<const float*>(q);
  const auto* q64 = static_cast<const double*>(q);
  if (v.v32 && v.stream)
    hipLaunchKernelGGL((dev::k_b_xr<float, true>), g, dim3(256), 0, st, v.act, v.voff, x, v.r32, v.p32, q32, v.invd32,
                       v.s, v.part);
  else if (v.v32)
    hipLaunchKernelGGL((dev::k_b_xr<float, false>), g, dim3(256), 0, st, v.act, v.voff, x, v.r32, v.p32, q32, v.invd32,
                       v.s, v.part);
  else if (v.stream)
    hipLaunchKernelGGL((dev::k_b_xr<double, true>), g, dim3(256), 0, st, v.act, v.voff, x, v.r, v.p, q64, v.invd, v.s,
                       v.part);
  else
    hipLaunchKernelGGL((dev::k_b_xr<double, false>), g, dim3(256), 0, st, v.act, v.voff, x, v.r, v.p, q64, v.invd,
                       v.s, v.part);
}
void bk_fin_rz(const BatchVecArgs& v, double delta, int mixed, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_b_fin_rz, dim3(v.nact), dim3(256), 0, st, v.act, v.part, v.gx, v.s, v.tol, delta, mixed);
}
void bk_p(const BatchVecArgs& v, hipStream_t st) {
  const dim3 g(v.gx, v.nact);
  if (v.v32)  // FP32 vectors: every load cached (streamed<S> is a plain load for them)
    hipLaunchKernelGGL((dev::k_b_p<float, false>), g, dim3(256), 0, st, v.act, v.voff, v.p32, v.r32, v.invd32, v.s);
  else if (v.stream)
    hipLaunchKernelGGL((dev::k_b_p<double, true>), g, dim3(256), 0, st, v.act, v.voff, v.p, v.r, v.invd, v.s);
  else
    hipLaunchKernelGGL((dev::k_b_p<double, false>), g, dim3(256), 0, st, v.act, v.voff, v.p, v.r, v.invd, v.s);
}
void bk_replace(const BatchVecArgs& v, const double* b, const double* y, int mixed, hipStream_t st) {
  if (v.v32)
    hipLaunchKernelGGL(dev::k_b_replace<float>, dim3(v.gx, v.nact), dim3(256), 0, st, v.act, v.voff, b, y, v.invd32,
                       v.r32, v.p32, v.s, v.part);
  else
    hipLaunchKernelGGL(dev::k_b_replace<double>, dim3(v.gx, v.nact), dim3(256), 0, st, v.act, v.voff, b, y, v.invd,
                       v.r, v.p, v.s, v.part);
  hipLaunchKernelGGL(dev::k_b_fin_replace, dim3(v.nact), dim3(256), 0, st, v.act, v.part, v.gx, v.s, v.tol, mixed);
}
void bk_resid(const BatchVecArgs& v, const double* b, const double* y, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_b_resid, dim3(v.gx, v.np), dim3(256), 0, st, nullptr, v.voff, b, y, v.part);
  hipLaunchKernelGGL(dev::k_b_fin_resid, dim3(v.np), dim3(256), 0, st, v.part, v.gx, out);
}

void bk_finish(const BatchVecArgs& v, const int* act, int nact, const double* stage, const uint32_t* rowptr,
               const uint32_t* slots, const int32_t* shared, const int64_t* sh_off, const int32_t* bnd,
               const int64_t* bnd_off, const void* u, void* y, bool f32, hipStream_t st) {
  if (nact <= 0) return;
  if (f32)
    hipLaunchKernelGGL(dev::k_b_finish<float>, dim3(v.gx, nact), dim3(256), 0, st, act, stage, rowptr, slots, shared,
                       sh_off, bnd, bnd_off, static_cast<const float*>(u), static_cast<float*>(y));
  else
    hipLaunchKernelGGL(dev::k_b_finish<double>, dim3(v.gx, nact), dim3(256), 0, st, act, stage, rowptr, slots, shared,
                       sh_off, bnd, bnd_off, static_cast<const double*>(u), static_cast<double*>(y));
}

}  // namespace dogip
