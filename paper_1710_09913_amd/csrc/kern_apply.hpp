// Tile kernel of the DoGIP apply (Algorithm 1 with the transpose of eq. ep_dogip_mul):
// one workgroup per tile of TE cells, one lane per cell.
//
//   1. gather: the tile's distinct dofs u[dof] -> LDS (0 for Dirichlet dofs)
//   2. per cell: local slots -> u_T from LDS; y_T = B^^T D_T B^ u_T streaming D_T
//      (AoSoA, 16-byte chunks, non-temporal); y_T added into LDS (ds_add)
//   3. flush: dofs only this tile touches are stored, dofs shared with other
//      tiles are added with a device atomic (the caller zeroed them), Dirichlet
//      dofs get y = u.
// With ENERGY, the tile also writes sum_T u_T^T A_T u_T (+ u_B^2 once per
// Dirichlet dof) = u . (A u), which CG needs as p^T A p.
#pragma once

#include "kern_common.hpp"

namespace dogip {
namespace dev {

template <int D, int K, int KIND, typename T, int VARIANT, bool ENERGY>
__global__ __launch_bounds__(512) void k_apply(ApplyLaunch a) {
  using E = Elem<D, K, KIND, T, T, VARIANT, ENERGY>;
  constexpr int VT = E::VT;
  extern __shared__ __align__(16) unsigned char smem[];
  T* us = reinterpret_cast<T*>(smem);
  T* ys = us + a.lds_slots;
  const int64_t t = a.tile_base + xcd_tile(blockIdx.x, gridDim.x);
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) {
    const uint32_t td = a.tile_dofs[o0 + j];
    us[j] = (td & TD_BND) ? T(0) : T(a.u[td & TD_MASK]);
    ys[j] = T(0);
  }
  __syncthreads();
  const int64_t e = t * a.te + threadIdx.x;
  T en = T(0);
  if (e < a.nel) {
    const int lane = threadIdx.x & 63;
    const int64_t w = t * (a.te >> 6) + __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    int li[VT];
    load_lidx<VT>(a.lidx, w, a.nlc, lane, li);
    T ue[VT], ye[VT];
    sfor<VT>([&](auto L) { ue[L] = us[li[L]]; });
    const typename E::V* dp = reinterpret_cast<const typename E::V*>(a.D) + (w * a.nch) * 64 + lane;
    en = E::run(dp, ue, ye);
    sfor<VT>([&](auto L) { atomicAdd(&ys[li[L]], ye[L]); });
  }
  __syncthreads();
  double eb = 0.0;
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) {
    const uint32_t td = a.tile_dofs[o0 + j];
    const uint32_t dof = td & TD_MASK;
    if (td & TD_BND) {
      const double ub = a.u[dof];
      a.y[dof] = ub;
      if (ENERGY && (td & TD_OWNER)) eb += ub * ub;
    } else if (td & TD_SHARED) {
      unsafeAtomicAdd(&a.y[dof], double(ys[j]));
    } else {
      a.y[dof] = double(ys[j]);
    }
  }
  if constexpr (ENERGY) {
    __shared__ double red[8];
    const double s = block_sum(double(en) + eb, red);
    if (threadIdx.x == 0) a.energy[t] = s;
  }
}

template <int D, int K, int KIND, int VARIANT>
bool launch_apply_t(int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  const dim3 grid(unsigned(a.ntiles)), block(unsigned(a.te));
  if (prec == DOGIP_F64) {
    const size_t lds = size_t(2) * a.lds_slots * sizeof(double);
    if (energy)
      hipLaunchKernelGGL((k_apply<D, K, KIND, double, VARIANT, true>), grid, block, lds, st, a);
    else
      hipLaunchKernelGGL((k_apply<D, K, KIND, double, VARIANT, false>), grid, block, lds, st, a);
  } else {
    const size_t lds = size_t(2) * a.lds_slots * sizeof(float);
    if (energy)
      hipLaunchKernelGGL((k_apply<D, K, KIND, float, VARIANT, true>), grid, block, lds, st, a);
    else
      hipLaunchKernelGGL((k_apply<D, K, KIND, float, VARIANT, false>), grid, block, lds, st, a);
  }
  return true;
}

}  // namespace dev
}  // namespace dogip

// Case list helper for the instantiation files.
#define DOGIP_APPLY_CASE(D, K, KIND, VAR) \
  case (KIND) * 16 + (K):                 \
    return dev::launch_apply_t<D, K, KIND, VAR>(prec, energy, a, st);
