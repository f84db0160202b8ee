// Tile kernel of the DoGIP apply (Algorithm 1 with the transpose of eq. ep_dogip_mul):
// one workgroup per tile of te cells, one lane per cell in each of te / lanes passes.
//
//   1. gather: the tile's distinct dofs u[dof] -> LDS (0 for Dirichlet dofs)
//   2. per cell: local slots -> u_T from LDS; y_T = B^^T D_T B^ u_T streaming D_T
//      (AoSoA, 16-byte chunks, non-temporal); y_T added into LDS (ds_add)
//   3. flush: dofs only this tile touches are stored to y, the tile's partial sums
//      for dofs shared with other tiles go to a staging buffer that a second pass
//      adds up in a fixed order; Dirichlet dofs are left to the second pass.
// With ENERGY, the tile also writes sum_T u_T^T A_T u_T, which with u_B^2 once per
// Dirichlet dof (second pass) is u . (A u), the p^T A p of CG.  It is taken at the
// flush as sum over the tile's slots of u_slot * y_slot (both in LDS): the same sum
// regrouped by dof, with no extra registers in the element loop.
#pragma once

#include "kern_common.hpp"

namespace dogip {
namespace dev {

#ifndef DOGIP_PF64
#define DOGIP_PF64 2
#endif
#ifndef DOGIP_PF32
#define DOGIP_PF32 3
#endif
#ifndef DOGIP_WPE
#define DOGIP_WPE 1
#endif

constexpr int GB = 8;  // tile dof entries handled per thread in one batch

// Gather of one batch: entries j = j0 + g * blockDim.x; u -> LDS (0 for Dirichlet
// dofs), accumulation slots zeroed.  The GB loads of a thread are in flight together.
template <typename T, typename VU, typename A>
__device__ __forceinline__ void gather_batch(const uint32_t* __restrict__ td, int64_t nd, int64_t j0,
                                             const VU* __restrict__ u, T* us, A* ys, uint32_t (&e)[GB]) {
  VU v[GB];
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    const int64_t j = j0 + int64_t(g) * blockDim.x;
    e[g] = j < nd ? td[j] : TD_BND;
  }
#pragma unroll
  for (int g = 0; g < GB; ++g) v[g] = (e[g] & TD_BND) ? VU(0) : u[e[g] & TD_MASK];
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    const int64_t j = j0 + int64_t(g) * blockDim.x;
    if (j < nd) {
      us[j] = T(v[g]);
      ys[j] = A(0);
    }
  }
}

// Tile entries j0 + g * blockDim.x of one batch (TD_BND past the end).
__device__ __forceinline__ void load_entries(const uint32_t* __restrict__ td, int64_t nd, int64_t j0,
                                             uint32_t (&e)[GB]) {
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    const int64_t j = j0 + int64_t(g) * blockDim.x;
    e[g] = j < nd ? td[j] : TD_BND;
  }
}

// Flush of one batch: shared entries -> staging (second pass sums them), exclusive
// entries -> y; Dirichlet entries are written by the second pass.
template <bool ENERGY, typename T, typename VY, typename A>
__device__ __forceinline__ void flush_batch(const uint32_t (&e)[GB], int64_t nd, int64_t j0, const A* ys,
                                            const T* us, double* __restrict__ stage, VY* __restrict__ y,
                                            double& en) {
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    const int64_t j = j0 + int64_t(g) * blockDim.x;
    if (j >= nd || (e[g] & TD_BND)) continue;
    if constexpr (ENERGY) en = fma(double(us[j]), double(ys[j]), en);
    if (e[g] & TD_SHARED)
      stage[j] = double(ys[j]);
    else
      y[e[g] & TD_MASK] = VY(ys[j]);
  }
}

// Work of one tile (one workgroup).  T is the element arithmetic precision (D is
// stored in T); the per-tile accumulation in LDS is always FP64 (ds_add_f64; FP32
// accumulation, which would halve the LDS arrays, measured 10-45% slower).  The
// flush reads the tile's entries again rather than holding them in registers through
// the element passes (which took the FP32 kernel from 128 to 133 VGPRs).  energy_out: where the
// tile's sum_T u_T^T A_T u_T goes (ENERGY only).  MODE 1: global projection form, D
// holds one value per W dof in the per-wave layout of GlobalPlan; MODE 2: the
// conventional quadrature-point apply (ElemQ).
// V32: FP32 input and output vectors (a.u32, a.y32).  MP: tiles in passes (a.cpl); without it
// one pass (cpl 1), which lets the compiler keep fewer values live (2D P5 FP64: 165 VGPRs,
// 3 waves per SIMD, against 243 with the pass loop).
template <int D, int K, int KIND, typename T, int VARIANT, bool ENERGY, int PF, int MODE = 0, bool V32 = false,
          bool MP = true>
__device__ __forceinline__ void tile_body(const ApplyLaunch& a, int64_t t, unsigned char* smem, double* energy_out) {
  using E = Elem<D, K, KIND, T, T, VARIANT, false, PF>;
  constexpr int VT = dim_p(D, K);
  double* ys = reinterpret_cast<double*>(smem);
  T* us = reinterpret_cast<T*>(ys + a.lds_slots);
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  const uint32_t* td = a.tile_dofs + o0;
  uint32_t ent[GB];
  const auto* uin = [&] {
    if constexpr (V32)
      return a.u32;
    else
      return a.u;
  }();
  auto* yout = [&] {
    if constexpr (V32)
      return a.y32;
    else
      return a.y;
  }();
  // the tile's cells are taken in cpl passes of `lanes` cells, one per lane; pass c holds
  // tile cells [c * lanes, (c + 1) * lanes), i.e. global waves t * te / 64 + c * lanes / 64 + wave
  const int cpl = MP ? a.cpl : 1, lanes = a.te / cpl, me = int(threadIdx.x >> 6), nw = (lanes + 63) >> 6;
  auto cell_of = [&](int c) -> int64_t {
    return int(threadIdx.x) < lanes ? t * a.te + int64_t(c) * lanes + threadIdx.x : a.nel;
  };
  auto wave_of = [&](int c) -> int64_t {
    return t * (a.te >> 6) + c * (lanes >> 6) + __builtin_amdgcn_readfirstlane(me);
  };
  // the first D chunks of each cell are requested before the gather (and those of the next
  // pass before this pass's LDS accumulation), so their latency overlaps it (element-wise
  // form, compile-time B^).  FP64 D: 2% faster with one pass per tile.  FP32 D: 1.7% slower
  // with one pass (a wave per SIMD lost to the registers), 2.4% faster at 3D P3, whose
  // 1536-cell tiles run 12 waves per compute unit, within the 168 VGPRs of 3 waves per SIMD.
  constexpr bool PRE = MODE == 0 && (VARIANT == DOGIP_VARIANT_UNROLLED || VARIANT == DOGIP_VARIANT_FACTORED) &&
                       (sizeof(T) == 8 || (D == 3 && K == 3 && VARIANT == DOGIP_VARIANT_UNROLLED));
  // the flush's first entries are requested before the last accumulation in one-pass tiles;
  // in passes that cost more than it saved (3D 64^3 P2 FP64 Jacobi-PCG 0.056 -> 0.068 s,
  // factored 3D P3: 256 VGPRs and scratch)
  constexpr bool EARLY_ENTRIES = !MP;
  typename E::V pre[E::NPRE];
  auto preload = [&](int c) {
    if constexpr (PRE) {
      if (cell_of(c) < a.nel)
        E::preload(reinterpret_cast<const typename E::V*>(a.D) + (wave_of(c) * a.nch) * 64 + (threadIdx.x & 63), pre);
    }
  };
  __shared__ int turn;  // the wave whose cells are added next (pass c, wave w: turn c * nw + w)
  if (threadIdx.x == 0) turn = 0;
  preload(0);
  for (int64_t j0 = threadIdx.x; j0 < nd; j0 += int64_t(GB) * blockDim.x) gather_batch<T>(td, nd, j0, uin, us, ys, ent);
  __syncthreads();
  for (int c = 0;; ++c) {
    const int64_t e = cell_of(c);
    double yacc[VT];
    int sl[VT];
    if (e < a.nel) {
      const int lane = threadIdx.x & 63;
      const int64_t w = wave_of(c);
      int li[VT];
      load_lidx<VT>(a.lidx, w, a.nlc, lane, li);
      T ue[VT], ye[VT];
      sfor<VT>([&](auto L) { ue[L] = us[li[L]]; });
      if constexpr (MODE == 1) {
        ElemG<D, K, T, VARIANT>::run(static_cast<const T*>(a.D) + a.gw_woff[e >> 6], a.gw_mask[e], ue, ye);
      } else if constexpr (MODE == 2) {
        ElemQ<D, K, KIND, T>::run(a, w, lane, ue, ye);
      } else {
        const typename E::V* dp = reinterpret_cast<const typename E::V*>(a.D) + (w * a.nch) * 64 + lane;
        E::template run<PRE>(dp, ue, ye, pre);
      }
      sfor<VT>([&](auto L) { yacc[L] = double(ye[L]); sl[L] = li[L]; });
    }
    // LDS accumulation one wave after the other (passes in order), so the sums are bitwise
    // reproducible: in passes by wave turns (a wave that has added goes on with its next
    // pass), in one-pass tiles by a barrier per wave (cheaper for a few waves: the batched
    // 2D apply took 18% longer with turns)
    auto accumulate = [&] {
      if constexpr (MP) {
        if (me < nw) {
          wait_turn(&turn, c * nw + me);
          if (e < a.nel) sfor<VT>([&](auto L) { atomicAdd(&ys[sl[L]], yacc[L]); });
          pass_turn(&turn);
        }
      } else {
        for (int wv = 0; wv < nw; ++wv) {
          if (me == wv && e < a.nel) sfor<VT>([&](auto L) { atomicAdd(&ys[sl[L]], yacc[L]); });
          __syncthreads();
        }
      }
    };
    if (c + 1 < cpl) {
      preload(c + 1);
      accumulate();
      continue;
    }
    // last pass: the flush's first entries are requested before the accumulation, so their
    // latency overlaps it (they are live only from here, not through the element passes)
    if constexpr (EARLY_ENTRIES) load_entries(td, nd, threadIdx.x, ent);
    accumulate();
    break;
  }
  if constexpr (MP) __syncthreads();  // every wave's sums are in before the flush reads them
  double* stage = a.stage + a.stage_off[t];
  double en = 0.0;
  for (int64_t j0 = threadIdx.x; j0 < nd; j0 += int64_t(GB) * blockDim.x) {
    if (!EARLY_ENTRIES || j0 != threadIdx.x) load_entries(td, nd, j0, ent);
    flush_batch<ENERGY>(ent, nd, j0, ys, us, stage, yout, en);
  }
  if constexpr (ENERGY) {
    __shared__ double red[8];
    const double s = block_sum(en, red);
    if (threadIdx.x == 0) *energy_out = s;
  }
}

// One workgroup per tile; workgroup -> tile mapping keeps each XCD on a contiguous range.
template <int D, int K, int KIND, typename T, int VARIANT, bool ENERGY, int PF, bool V32, bool MP>
__global__ __launch_bounds__(sizeof(T) == 8 ? 512 : 768, DOGIP_WPE) void k_apply(ApplyLaunch a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = a.tile_base + xcd_tile(blockIdx.x, gridDim.x);
  tile_body<D, K, KIND, T, VARIANT, ENERGY, PF, 0, V32, MP>(a, t, smem, ENERGY ? a.energy + t : nullptr);
}

// One pass (the kernel without the pass loop) when the tile fits the workgroup: the lanes
// asked for equal the tile, or none were asked for and the tile is within the launch bound.
// The factored kernels always take the pass loop (2D P5 FP64: 0.133 ms with it, 0.175 ms
// without, where the straight-line body takes 254 VGPRs).
template <int D, int K, int KIND, typename T, int VARIANT, bool ENERGY, int PF, bool V32>
void launch_k_apply(const ApplyLaunch& a, size_t lds, hipStream_t st) {
  const int bound = sizeof(T) == 8 ? 512 : 768;
  if constexpr (VARIANT != DOGIP_VARIANT_FACTORED) {
    if (a.cpl == 1 || (a.cpl <= 0 && a.te <= bound)) {
      ApplyLaunch b = a;
      b.cpl = 1;
      launch_tiles((k_apply<D, K, KIND, T, VARIANT, ENERGY, PF, V32, false>), b, lds, st);
      return;
    }
  }
  launch_tiles((k_apply<D, K, KIND, T, VARIANT, ENERGY, PF, V32, true>), a, lds, st);
}

template <int D, int K, typename T, int VARIANT, bool ENERGY>
__global__ __launch_bounds__(512, DOGIP_WPE) void k_apply_g(ApplyLaunch a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = a.tile_base + xcd_tile(blockIdx.x, gridDim.x);
  tile_body<D, K, KIND_WP, T, VARIANT, ENERGY, 0, 1>(a, t, smem, ENERGY ? a.energy + t : nullptr);
}

template <int D, int K, typename T, int VARIANT>
void launch_apply_g_p(bool energy, const ApplyLaunch& a, hipStream_t st) {
  const size_t lds = size_t(a.lds_slots) * (sizeof(double) + sizeof(T));
  if (energy)
    launch_tiles((k_apply_g<D, K, T, VARIANT, true>), a, lds, st);
  else
    launch_tiles((k_apply_g<D, K, T, VARIANT, false>), a, lds, st);
}

template <int D, int K, int VARIANT>
bool launch_apply_g_t(int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  if (prec == DOGIP_F64)
    launch_apply_g_p<D, K, double, VARIANT>(energy, a, st);
  else
    launch_apply_g_p<D, K, float, VARIANT>(energy, a, st);
  return true;
}

template <int D, int K, int KIND, int VARIANT>
bool launch_apply_t(int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  constexpr bool UNR = VARIANT == DOGIP_VARIANT_UNROLLED || VARIANT == DOGIP_VARIANT_FACTORED;
  constexpr int P64 = UNR ? DOGIP_PF64 : 0;
  constexpr int P32 = UNR ? DOGIP_PF32 : 0;
  if (prec == DOGIP_F64) {
    const size_t lds = size_t(a.lds_slots) * (sizeof(double) + sizeof(double));
    if (energy)
      launch_k_apply<D, K, KIND, double, VARIANT, true, P64, false>(a, lds, st);
    else
      launch_k_apply<D, K, KIND, double, VARIANT, false, P64, false>(a, lds, st);
  } else {
    const size_t lds = size_t(a.lds_slots) * (sizeof(double) + sizeof(float));
    if (a.u32) {
      if (!energy) return false;  // FP32 vectors: the CG iteration only
      launch_k_apply<D, K, KIND, float, VARIANT, true, P32, true>(a, lds, st);
    } else if (energy) {
      launch_k_apply<D, K, KIND, float, VARIANT, true, P32, false>(a, lds, st);
    } else {
      launch_k_apply<D, K, KIND, float, VARIANT, false, P32, false>(a, lds, st);
    }
  }
  return true;
}

}  // namespace dev
}  // namespace dogip

// Case list helper for the instantiation files.
#define DOGIP_APPLY_CASE(D, K, KIND, VAR) \
  case (KIND) * 16 + (K):                 \
    return dev::launch_apply_t<D, K, KIND, VAR>(prec, energy, a, st);
