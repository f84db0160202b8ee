// FP32 apply of the 3D P3 elliptic operator with the two B^ products of Algorithm 1
// (g = B^ u_T and y_T = B^^T h, eq. ep_dogip_mul) on the matrix cores.
//
// Every entry of B^ for 3D P3 (reference gradients of the cubic basis at the nodes of
// P_4) has at most 8 significant bits, so B^ is exact in bfloat16.  The vector operand
// (u_T, then h = D_T g) is split into three bfloat16 terms, x = hi + mid + lo, exactly:
// hi keeps the leading 8 bits of the FP32 value, mid the next 8 of the remainder and lo
// the rest, each by truncation (the remainders are exact FP32 differences).  Each
// product of a B^ entry with a term is then exact in FP32, and v_mfma_f32_16x16x32_bf16
// sums them in FP32: the products carry the rounding of FP32 accumulation only, as in
// the FP32 vector kernel.
//
// One wave works on its 64 cells as four blocks of 16 (the MFMA column index n), lane
// l = 16 q + n.  Layouts (lane q of column n):
//   * first product, G [144 x 16] = B1 [144 x 32] . U [32 x 16]: row 4 i + r is the
//     component r < 3 of W node i (row 4 i + 3 and nodes >= 35 are zero); column slot
//     8 q + t of U holds local dof L(q, t) = 4 q + t (t < 4) or 16 + 4 q + t - 4 (t >= 4,
//     only q = 0 has such dofs: 16..19).  The accumulator of M-block m gives lane q the
//     3 components of node 4 m + q, so h = D_T,i g_i is formed in the lane.
//   * second product, Y [32 x 16] = B2 [32 x 160] . H [160 x 16]: K-block j takes the
//     accumulators of M-blocks 2j and 2j+1 as they sit in the lanes (slot 8 q + t is
//     node 8 j + q, component t for t < 4, and node 8 j + 4 + q, component t - 4, for
//     t >= 4), with B2's columns permuted to match; its M-blocks give lane q local
//     dofs 4 q .. 4 q + 3 and 16 + 4 q .. 16 + 4 q + 3, the same L(q, t) as U.
// B1 and B2, 19 operand registers per lane, are tables copied to LDS per workgroup.
// D (FP32) is stored for this layout: per wave, block (cell block b, M-block m), the 64
// lanes' 6 packed components as 4 + 2 floats ([4][64] then [2][64] floats).
#include "kern_apply.hpp"

#include <bit>

namespace dogip {
namespace dev {

using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));
using u32x4 = uint32_t __attribute__((ext_vector_type(4)));
using f32x4 = float __attribute__((ext_vector_type(4)));
using f32x2 = float __attribute__((ext_vector_type(2)));

constexpr int MF_VT = 20, MF_WT = 35, MF_MB1 = 9, MF_KB2 = 5, MF_TABS = MF_MB1 + 2 * MF_KB2;

// local dof of K slot t of lane quarter q (first product), -1 for a zero slot
constexpr int mf_dof(int q, int t) {
  const int v = t < 4 ? 4 * q + t : 16 + 4 * q + (t - 4);
  return v < MF_VT ? v : -1;
}

constexpr uint16_t bf16_bits(double b) {
  const uint32_t u = std::bit_cast<uint32_t>(float(b));
  return uint16_t(u >> 16);
}
constexpr bool bf16_exact(double b) { return (std::bit_cast<uint32_t>(float(b)) & 0xffffu) == 0 && double(float(b)) == b; }

// The operand tables: [MF_TABS][64 lanes][8] bfloat16.  Tables 0..8: B1's M-blocks;
// 9 + 5 mo + j: B2's M-block mo, K-block j.
struct MfTables {
  uint16_t v[MF_TABS][64][8];
  bool exact;
  constexpr MfTables() : v{}, exact(true) {
    constexpr auto& B = CT<3, 3, KIND_SE>::t.v;  // [r][i][l]
    for (int mb = 0; mb < MF_MB1; ++mb)
      for (int l = 0; l < 64; ++l)
        for (int t = 0; t < 8; ++t) {
          const int row = 16 * mb + (l & 15), i = row / 4, r = row % 4, v = mf_dof(l >> 4, t);
          const double b = (r < 3 && i < MF_WT && v >= 0) ? B[r][i][v] : 0.0;
          exact = exact && bf16_exact(b);
          this->v[mb][l][t] = bf16_bits(b);
        }
    for (int mo = 0; mo < 2; ++mo)
      for (int j = 0; j < MF_KB2; ++j)
        for (int l = 0; l < 64; ++l)
          for (int t = 0; t < 8; ++t) {
            const int v = 16 * mo + (l & 15), q = l >> 4;
            const int i = t < 4 ? 8 * j + q : 8 * j + 4 + q, r = t & 3;
            const double b = (r < 3 && i < MF_WT && v < MF_VT) ? B[r][i][v] : 0.0;
            exact = exact && bf16_exact(b);
            this->v[MF_MB1 + MF_KB2 * mo + j][l][t] = bf16_bits(b);
          }
  }
};
constexpr MfTables mf_tables_host{};
static_assert(mf_tables_host.exact, "B^ of 3D P3 must be exact in bfloat16");
__constant__ MfTables mf_tables = mf_tables_host;

// x = hi + mid + lo exactly; the three bfloat16 vectors of 8 FP32 values
__device__ __forceinline__ void split3(const float (&x)[8], bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  u32x4 h, m, o;
  sfor<4>([&](auto P) {
    constexpr int p = P;
    uint32_t hb[2], mb[2], lb[2];
    sfor<2>([&](auto S) {
      const float v = x[2 * p + S];
      hb[S] = __float_as_uint(v) & 0xffff0000u;
      const float r1 = v - __uint_as_float(hb[S]);
      mb[S] = __float_as_uint(r1) & 0xffff0000u;
      const float r2 = r1 - __uint_as_float(mb[S]);
      lb[S] = __float_as_uint(r2) & 0xffff0000u;
    });
    h[p] = (hb[0] >> 16) | hb[1];
    m[p] = (mb[0] >> 16) | mb[1];
    o[p] = (lb[0] >> 16) | lb[1];
  });
  hi = __builtin_bit_cast(bf16x8, h);
  mid = __builtin_bit_cast(bf16x8, m);
  lo = __builtin_bit_cast(bf16x8, o);
}

__device__ __forceinline__ f32x4 mma3(const bf16x8& a, const bf16x8& hi, const bf16x8& mid, const bf16x8& lo,
                                      f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, mid, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, c, 0, 0, 0);
}

// FP32 floats of D per wave in the MFMA layout
constexpr int MF_DWAVE = 4 * MF_MB1 * 384;

template <bool ENERGY, bool V32>
__global__ __launch_bounds__(512, DOGIP_WPE) void k_apply_mfma(ApplyLaunch a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = a.tile_base + xcd_tile(blockIdx.x, gridDim.x);
  u32x4* tab = reinterpret_cast<u32x4*>(smem);  // [MF_TABS][64]
  double* ys = reinterpret_cast<double*>(smem + MF_TABS * 64 * 16);
  float* us = reinterpret_cast<float*>(ys + a.lds_slots);
  {
    const u32x4* src = reinterpret_cast<const u32x4*>(&mf_tables.v[0][0][0]);
    for (int i = threadIdx.x; i < MF_TABS * 64; i += blockDim.x) tab[i] = src[i];
  }
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  const uint32_t* td = a.tile_dofs + o0;
  const bool one = nd <= int64_t(GB) * blockDim.x;
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
  if (one) {
    gather_batch<float>(td, nd, threadIdx.x, uin, us, ys, ent);
  } else {
    for (int64_t j0 = threadIdx.x; j0 < nd; j0 += int64_t(GB) * blockDim.x) gather_batch<float>(td, nd, j0, uin, us, ys, ent);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, q = lane >> 4, n = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int64_t w = t * (a.te >> 6) + wv;
  const int64_t cell0 = w * 64;
  const bool wave_live = int(threadIdx.x) < a.te && cell0 < a.nel;
  // The wave's 4 x 9 steps (cell block nb, first-product M-block mb) run as one unrolled
  // sequence; the D values of step s + 2 are requested at step s (a ring of three), so
  // the loads stay ahead of the matrix-core work without holding a block's D at once.
  float yv[4][8];
  const u32x4* lp = reinterpret_cast<const u32x4*>(a.lidx) + (w * a.nlc) * 64;
  if (wave_live) {
    const float* dw = static_cast<const float*>(a.D) + w * MF_DWAVE;
    constexpr int NS = 4 * MF_MB1;
    f32x4 r4[3];
    f32x2 r2[3];
    auto request = [&](auto S) {
      constexpr int st = S, nb = st / MF_MB1, mb = st % MF_MB1;
      if (4 * mb + q < MF_WT) {
        const float* p = dw + (nb * MF_MB1 + mb) * 384;
        r4[st % 3] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + lane);
        r2[st % 3] = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p + 256) + lane);
      }
    };
    request(std::integral_constant<int, 0>{});
    request(std::integral_constant<int, 1>{});
    bf16x8 uh, um, ul;
    f32x4 y0, y1;
    float hv[8];
    sfor<NS>([&](auto S) {
      constexpr int st = S, nb = st / MF_MB1, mb = st % MF_MB1;
      if constexpr (mb == 0) {
        // a compiler barrier: the operand tables are read from LDS again for each block
        // instead of being held in registers across the blocks (76 registers)
        asm volatile("" ::: "memory");
        // the block's u_T: local slots of L(q, 0..7) from the cell's local-index chunks
        // (chunk q/2, half q%2; for q = 0 also the first half of chunk 2)
        const int cl = 16 * nb + n;
        const bool live = cell0 + cl < a.nel;
        const u32x4 c0 = lp[(q >> 1) * 64 + cl];
        uint32_t pw[4];
        pw[0] = (q & 1) ? c0[2] : c0[0];
        pw[1] = (q & 1) ? c0[3] : c0[1];
        if (q == 0) {
          const u32x4 c2 = lp[2 * 64 + cl];
          pw[2] = c2[0];
          pw[3] = c2[1];
        } else {
          pw[2] = pw[3] = 0xffffffffu;
        }
        float uu[8];
        sfor<8>([&](auto T) {
          const uint32_t sv = (pw[T / 2] >> (16 * (T % 2))) & 0xffffu;
          uu[T] = (live && sv != 0xffffu) ? us[sv] : 0.0f;
        });
        split3(uu, uh, um, ul);
        y0 = f32x4{0.f, 0.f, 0.f, 0.f};
        y1 = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      if constexpr (st + 2 < NS) request(std::integral_constant<int, st + 2>{});
      const f32x4 g = mma3(__builtin_bit_cast(bf16x8, tab[mb * 64 + lane]), uh, um, ul, f32x4{0.f, 0.f, 0.f, 0.f});
      float h0 = 0.f, h1 = 0.f, h2 = 0.f;
      if (4 * mb + q < MF_WT) {
        const f32x4 d4 = r4[st % 3];
        const f32x2 d2 = r2[st % 3];
        // packed symmetric (00, 01, 02, 11, 12, 22)
        h0 = __builtin_fmaf(d4[2], g[2], __builtin_fmaf(d4[1], g[1], d4[0] * g[0]));
        h1 = __builtin_fmaf(d2[0], g[2], __builtin_fmaf(d4[3], g[1], d4[1] * g[0]));
        h2 = __builtin_fmaf(d2[1], g[2], __builtin_fmaf(d2[0], g[1], d4[2] * g[0]));
      }
      constexpr int hf = mb & 1;
      hv[4 * hf + 0] = h0;
      hv[4 * hf + 1] = h1;
      hv[4 * hf + 2] = h2;
      hv[4 * hf + 3] = 0.f;
      if constexpr (hf == 1 || mb == MF_MB1 - 1) {
        // K-block j of the second product: the accumulators of M-blocks 2j and 2j+1
        constexpr int j = mb / 2;
        if constexpr (hf == 0) sfor<4>([&](auto C) { hv[4 + C] = 0.f; });
        bf16x8 hh, hm, hl;
        split3(hv, hh, hm, hl);
        y0 = mma3(__builtin_bit_cast(bf16x8, tab[(MF_MB1 + j) * 64 + lane]), hh, hm, hl, y0);
        y1 = mma3(__builtin_bit_cast(bf16x8, tab[(MF_MB1 + MF_KB2 + j) * 64 + lane]), hh, hm, hl, y1);
      }
      if constexpr (mb == MF_MB1 - 1) {
        sfor<4>([&](auto C) {
          yv[nb][C] = y0[int(C)];
          yv[nb][4 + C] = y1[int(C)];
        });
      }
    });
  }
  // LDS accumulation one wave after the other (bitwise reproducible sums)
  const int nw = (a.te + 63) >> 6;
  for (int r = 0; r < nw; ++r) {
    if (wv == r && wave_live)
      sfor<4>([&](auto NB) {
        // the block's slots again (the chunks were read in the element phase)
        const int cl = 16 * NB + n;
        if (cell0 + cl < a.nel) {
          const u32x4 c0 = lp[(q >> 1) * 64 + cl];
          uint32_t pw[4];
          pw[0] = (q & 1) ? c0[2] : c0[0];
          pw[1] = (q & 1) ? c0[3] : c0[1];
          if (q == 0) {
            const u32x4 c2 = lp[2 * 64 + cl];
            pw[2] = c2[0];
            pw[3] = c2[1];
          } else {
            pw[2] = pw[3] = 0xffffffffu;
          }
          sfor<8>([&](auto T) {
            const uint32_t sv = (pw[T / 2] >> (16 * (T % 2))) & 0xffffu;
            if (sv != 0xffffu) atomicAdd(&ys[sv], double(yv[NB][T]));
          });
        }
      });
    __syncthreads();
  }
  double* stage = a.stage + a.stage_off[t];
  double en = 0.0;
  if (one) {
    flush_batch<ENERGY>(ent, nd, threadIdx.x, ys, us, stage, yout, en);
  } else {
    for (int64_t j0 = threadIdx.x; j0 < nd; j0 += int64_t(GB) * blockDim.x) {
#pragma unroll
      for (int g = 0; g < GB; ++g) {
        const int64_t j = j0 + int64_t(g) * blockDim.x;
        ent[g] = j < nd ? td[j] : TD_BND;
      }
      flush_batch<ENERGY>(ent, nd, j0, ys, us, stage, yout, en);
    }
  }
  if constexpr (ENERGY) {
    __shared__ double red[8];
    const double sum = block_sum(en, red);
    if (threadIdx.x == 0) a.energy[t] = sum;
  }
}

}  // namespace dev

// D floats per wave of the MFMA layout (allocation and construction)
int64_t mfma_d32_per_wave() { return dev::MF_DWAVE; }
int64_t mfma_lds_tables() { return int64_t(dev::MF_TABS) * 64 * 16; }

bool launch_apply_mfma(bool energy, const ApplyLaunch& a, hipStream_t st) {
  const dim3 grid(unsigned(a.ntiles)), block(unsigned(a.te));
  const size_t lds = size_t(dev::MF_TABS) * 64 * 16 + size_t(a.lds_slots) * (sizeof(double) + sizeof(float));
  if (a.u32) {
    if (!energy) return false;  // FP32 vectors: the CG iteration only
    hipLaunchKernelGGL((dev::k_apply_mfma<true, true>), grid, block, lds, st, a);
  } else if (energy) {
    hipLaunchKernelGGL((dev::k_apply_mfma<true, false>), grid, block, lds, st, a);
  } else {
    hipLaunchKernelGGL((dev::k_apply_mfma<false, false>), grid, block, lds, st, a);
  }
  return true;
}

}  // namespace dogip
