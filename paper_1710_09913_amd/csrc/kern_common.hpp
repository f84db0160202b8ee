// Device helpers shared by the libdogip kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "internal.hpp"
#include "reftab.hpp"

namespace dogip {
namespace dev {

template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// Compile-time loop: f(integral_constant<int, i>) for i = 0..N-1.
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}
template <int A, class F, int... Is>
__device__ __forceinline__ void sfor_from_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, A + Is>{}), ...);
}
// Compile-time loop over A..B-1.
template <int A, int B, class F>
__device__ __forceinline__ void sfor_range(F&& f) {
  if constexpr (B > A) sfor_from_impl<A>(f, std::make_integer_sequence<int, B - A>{});
}

// Workgroups are dispatched round-robin over the 8 XCDs; map them so that each
// XCD (own L2) works on one contiguous range of tiles, which are neighbours in
// the Morton order and share dofs.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t nblk) {
  const int64_t x = bid & 7, pos = bid >> 3, q = nblk >> 3, r = nblk & 7;
  return x * q + (x < r ? x : r) + pos;
}

template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));

// Streaming load of one 16-byte chunk (D is read once per apply).
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// h = D g for one W node: scalar (projection) or packed symmetric d x d (elliptic).
template <int NB, int S, typename T>
__device__ __forceinline__ void dmul(const T (&dv)[S], const T (&g)[NB], T (&h)[NB]) {
  if constexpr (S == 1) {
    h[0] = dv[0] * g[0];
  } else if constexpr (NB == 2) {
    h[0] = fma_t(dv[1], g[1], dv[0] * g[0]);
    h[1] = fma_t(dv[2], g[1], dv[1] * g[0]);
  } else {
    h[0] = fma_t(dv[2], g[2], fma_t(dv[1], g[1], dv[0] * g[0]));
    h[1] = fma_t(dv[4], g[2], fma_t(dv[3], g[1], dv[1] * g[0]));
    h[2] = fma_t(dv[5], g[2], fma_t(dv[4], g[1], dv[2] * g[0]));
  }
}

// Position of value f (= node * s + component) of cell lane of wave w in the FP32 copy of
// D: AoSoA 16-byte chunks by 64 cells ([w][nch32][64][4]), or with nch32 < 0 the layout of
// the matrix-core apply of 3D P3 (per wave, per block of 16 cells and group of 4 nodes,
// the 64 lanes' 6 components as [4][64] then [2][64] floats; lane = 16 (node % 4) + cell % 16).
__device__ __forceinline__ int64_t d32_pos(int64_t w, int lane, int f, int64_t nch32) {
  if (nch32 >= 0) return (w * nch32 + (f >> 2)) * 256 + lane * 4 + (f & 3);
  const int i = f / 6, c = f - 6 * i, l = 16 * (i & 3) + (lane & 15);
  const int64_t base = ((w * 4 + (lane >> 4)) * 9 + (i >> 2)) * 384;
  return c < 4 ? base + l * 4 + c : base + 256 + l * 2 + (c - 4);
}

// Compile-time reference table (exact rationals rounded once to double).
template <int D, int K, int KIND>
struct CT {
  static constexpr ref::BTable<D, K, KIND> t{};
};

template <int D, int K>
struct CF {
  static constexpr ref::FTable<D, K> t{};
};

// The same table in device constant memory, in the compute precision, for the
// looped element body (wave-uniform index -> scalar loads).
template <int D, int K, int KIND, typename T>
struct CArr {
  using TB = ref::BTable<D, K, KIND>;
  T v[TB::NB * TB::WT * TB::VT];
  constexpr CArr() : v{} {
    for (int r = 0; r < TB::NB; ++r)
      for (int i = 0; i < TB::WT; ++i)
        for (int l = 0; l < TB::VT; ++l) v[(r * TB::WT + i) * TB::VT + l] = T(CT<D, K, KIND>::t.v[r][i][l]);
  }
};
template <int D, int K, int KIND, typename T>
__constant__ CArr<D, K, KIND, T> ctab{};

// Element body.  ue: local dof values; ye: local result (overwritten); dp: this
// lane's first D chunk (chunk j of the cell at dp[j * 64]).  Returns the cell
// energy u_T^T A_T u_T when ENERGY is set.  In the unrolled body the D chunks of
// W node i + PF are requested while node i is computed (prefetch distance PF).
template <int D, int K, int KIND, typename T, typename TD, int VARIANT, bool ENERGY, int PF = 0>
struct Elem {
  using TB = ref::BTable<D, K, KIND>;
  static constexpr int VT = TB::VT, WT = TB::WT, NB = TB::NB;
  static constexpr int S = KIND == KIND_SE ? n_sym(D) : 1;
  static constexpr int VEC = 16 / int(sizeof(TD));
  static constexpr int NCH = (WT * S + VEC - 1) / VEC;
  using V = vec_t<TD, VEC>;

  // node step at which chunk j is requested, and the first chunk requested at step i
  static constexpr int issue_step(int j) { return (j * VEC) / S - PF < 0 ? 0 : (j * VEC) / S - PF; }
  static constexpr int first_chunk(int i) {
    int j = 0;
    while (j < NCH && issue_step(j) < i) ++j;
    return j;
  }

  // the chunks requested before the first node is computed (unrolled body): a caller may
  // request them early (preload) and hand them to run
  static constexpr int NPRE = WT > 1 ? first_chunk(1) : NCH;
  __device__ __forceinline__ static void preload(const V* __restrict__ dp, V (&pre)[NPRE]) {
    sfor<NPRE>([&](auto J) { pre[J] = ld_stream(dp + J * 64); });
  }

  template <bool PRE = false>
  __device__ __forceinline__ static T run(const V* __restrict__ dp, const T (&ue)[VT], T (&ye)[VT],
                                          const V* pre = nullptr) {
    T en = T(0);
    sfor<VT>([&](auto L) { ye[L] = T(-0.0); });
    if constexpr (VARIANT == DOGIP_VARIANT_FACTORED) {
      // B^ = (I (x) B2) B1: G = B1 u_T (the gradient at the P_{k-1} nodes), per W node
      // g = B2_i G, h = D_i g, H += B2_i^T h, and y_T = B1^T H at the end
      using FT = ref::FTable<D, K>;
      constexpr int NJ = FT::NJ;
      T G[NB][NJ], H[NB][NJ];
      sfor<NB>([&](auto R) {
        sfor<NJ>([&](auto J) {
          T acc = T(-0.0);
          sfor<VT>([&](auto L) {
            constexpr double b = CF<D, K>::t.b1[R][J][L];
            if constexpr (b == 1.0)
              acc = acc + ue[L];
            else if constexpr (b == -1.0)
              acc = acc - ue[L];
            else if constexpr (b != 0.0)
              acc = fma_t(T(b), ue[L], acc);
          });
          G[R][J] = acc;
          H[R][J] = T(-0.0);
        });
      });
      V ch[NCH];
      sfor<WT>([&](auto I) {
        if constexpr (PRE && I == 0)
          sfor<NPRE>([&](auto J) { ch[J] = pre[J]; });
        else
          sfor_range<first_chunk(I), (I + 1 < WT ? first_chunk(I + 1) : NCH)>(
              [&](auto J) { ch[J] = ld_stream(dp + J * 64); });
        T g[NB];
        sfor<NB>([&](auto R) {
          T acc = T(-0.0);
          sfor<NJ>([&](auto J) {
            constexpr double b = CF<D, K>::t.b2[I][J];
            if constexpr (b == 1.0)
              acc = acc + G[R][J];
            else if constexpr (b != 0.0)
              acc = fma_t(T(b), G[R][J], acc);
          });
          g[R] = acc;
        });
        T dv[S];
        sfor<S>([&](auto C) {
          constexpr int f = I * S + C;
          dv[C] = T(ch[f / VEC][f % VEC]);
        });
        T h[NB];
        dmul<NB, S>(dv, g, h);
        if constexpr (ENERGY) sfor<NB>([&](auto R) { en = fma_t(g[R], h[R], en); });
        sfor<NB>([&](auto R) {
          sfor<NJ>([&](auto J) {
            constexpr double b = CF<D, K>::t.b2[I][J];
            if constexpr (b == 1.0)
              H[R][J] = H[R][J] + h[R];
            else if constexpr (b != 0.0)
              H[R][J] = fma_t(T(b), h[R], H[R][J]);
          });
        });
      });
      sfor<VT>([&](auto L) {
        T acc = T(-0.0);
        sfor<NB>([&](auto R) {
          sfor<NJ>([&](auto J) {
            constexpr double b = CF<D, K>::t.b1[R][J][L];
            if constexpr (b == 1.0)
              acc = acc + H[R][J];
            else if constexpr (b == -1.0)
              acc = acc - H[R][J];
            else if constexpr (b != 0.0)
              acc = fma_t(T(b), H[R][J], acc);
          });
        });
        ye[L] = acc;
      });
    } else if constexpr (VARIANT == DOGIP_VARIANT_UNROLLED) {
      V ch[NCH];
      sfor<WT>([&](auto I) {
        if constexpr (PRE && I == 0)
          sfor<NPRE>([&](auto J) { ch[J] = pre[J]; });
        else
          sfor_range<first_chunk(I), (I + 1 < WT ? first_chunk(I + 1) : NCH)>(
              [&](auto J) { ch[J] = ld_stream(dp + J * 64); });
        T g[NB];
        sfor<NB>([&](auto R) {
          T acc = T(-0.0);
          sfor<VT>([&](auto L) {
            constexpr double b = CT<D, K, KIND>::t.v[R][I][L];
            if constexpr (b == 1.0)
              acc = acc + ue[L];
            else if constexpr (b == -1.0)
              acc = acc - ue[L];
            else if constexpr (b != 0.0)
              acc = fma_t(T(b), ue[L], acc);
          });
          g[R] = acc;
        });
        T dv[S];
        sfor<S>([&](auto C) {
          constexpr int f = I * S + C;
          dv[C] = T(ch[f / VEC][f % VEC]);
        });
        T h[NB];
        dmul<NB, S>(dv, g, h);
        if constexpr (ENERGY) sfor<NB>([&](auto R) { en = fma_t(g[R], h[R], en); });
        sfor<NB>([&](auto R) {
          sfor<VT>([&](auto L) {
            constexpr double b = CT<D, K, KIND>::t.v[R][I][L];
            if constexpr (b == 1.0)
              ye[L] = ye[L] + h[R];
            else if constexpr (b == -1.0)
              ye[L] = ye[L] - h[R];
            else if constexpr (b != 0.0)
              ye[L] = fma_t(T(b), h[R], ye[L]);
          });
        });
      });
    } else {
      const T* bt = ctab<D, K, KIND, T>.v;
      const TD* dsc = reinterpret_cast<const TD*>(dp);
      for (int i = 0; i < WT; ++i) {
        T g[NB];
        sfor<NB>([&](auto R) {
          const T* br = bt + (R * WT + i) * VT;
          T acc = T(-0.0);
          sfor<VT>([&](auto L) { acc = fma_t(br[L], ue[L], acc); });
          g[R] = acc;
        });
        T dv[S];
        sfor<S>([&](auto C) {
          const int f = i * S + C;
          dv[C] = T(__builtin_nontemporal_load(dsc + (f / VEC) * 64 * VEC + (f % VEC)));
        });
        T h[NB];
        dmul<NB, S>(dv, g, h);
        if constexpr (ENERGY) sfor<NB>([&](auto R) { en = fma_t(g[R], h[R], en); });
        sfor<NB>([&](auto R) {
          const T* br = bt + (R * WT + i) * VT;
          sfor<VT>([&](auto L) { ye[L] = fma_t(br[L], h[R], ye[L]); });
        });
      }
    }
    return en;
  }
};

// W nodes of the projection form grouped by sub-simplex slot (global variant, looped
// body): nodes of slot s are node[first[s] .. first[s+1]) in lattice order.
template <int D, int K>
struct CSlots {
  static constexpr int WT = dim_p(D, 2 * K), NS = gw_slots(D);
  int first[NS + 1];
  uint8_t node[WT];
  constexpr CSlots() : first{}, node{} {
    int c = 0;
    for (int e = 0; e < NS; ++e) {
      first[e] = c;
      for (int i = 0; i < WT; ++i)
        if (ref::node_entity(D, 2 * K, i) == e) node[c++] = uint8_t(i);
    }
    first[NS] = c;
  }
};
template <int D, int K>
__constant__ CSlots<D, K> cslots{};

// Where this lane's values of each owned slot sit in the wave's D range (see
// GlobalPlan): count, rank and base per slot from a ballot of the ownership bits.
template <int D, int K>
struct WaveSlots {
  static constexpr int NS = gw_slots(D);
  int cnt[NS], rank[NS], base[NS];
  __device__ __forceinline__ explicit WaveSlots(uint32_t mask) {
    int acc = 0;
    const uint32_t lane = __lane_id();
    sfor<NS>([&](auto E) {
      constexpr int ne = ref::entity_nodes(D, 2 * K, E);
      if constexpr (ne > 0) {
        const uint64_t b = __ballot((mask >> E) & 1u);
        cnt[E] = __popcll(b);
        rank[E] = __popcll(b & ((uint64_t(1) << lane) - 1));
        base[E] = acc;
        acc += ne * cnt[E];
      } else {
        cnt[E] = rank[E] = base[E] = 0;
      }
    });
  }
};

// Element body of the global projection form (Theorem 1).  The cell applies D only at
// the W nodes of the sub-simplex slots it owns (mask); the other nodes are applied by
// the cells that own them.  dw: the wave's D range.  Nodes are visited slot by slot.
template <int D, int K, typename T, int VARIANT>
struct ElemG {
  using TB = ref::BTable<D, K, KIND_WP>;
  static constexpr int VT = TB::VT, WT = TB::WT, NS = gw_slots(D);

  __device__ __forceinline__ static void run(const T* __restrict__ dw, uint32_t mask, const T (&ue)[VT],
                                             T (&ye)[VT]) {
    const WaveSlots<D, K> ws(mask);
    sfor<VT>([&](auto L) { ye[L] = T(-0.0); });
    if constexpr (VARIANT == DOGIP_VARIANT_UNROLLED) {
      sfor<WT>([&](auto I) {
        constexpr int e = ref::node_entity(D, 2 * K, I), j = ref::entity_rank(D, 2 * K, I);
        const bool own = (mask >> e) & 1u;
        T acc = T(-0.0);
        sfor<VT>([&](auto L) {
          constexpr double b = CT<D, K, KIND_WP>::t.v[0][I][L];
          if constexpr (b == 1.0)
            acc = acc + ue[L];
          else if constexpr (b == -1.0)
            acc = acc - ue[L];
          else if constexpr (b != 0.0)
            acc = fma_t(T(b), ue[L], acc);
        });
        T dv = T(0);
        if (own) dv = __builtin_nontemporal_load(dw + ws.base[e] + j * ws.cnt[e] + ws.rank[e]);
        const T h = dv * acc;
        sfor<VT>([&](auto L) {
          constexpr double b = CT<D, K, KIND_WP>::t.v[0][I][L];
          if constexpr (b == 1.0)
            ye[L] = ye[L] + h;
          else if constexpr (b == -1.0)
            ye[L] = ye[L] - h;
          else if constexpr (b != 0.0)
            ye[L] = fma_t(T(b), h, ye[L]);
        });
      });
    } else {
      const T* bt = ctab<D, K, KIND_WP, T>.v;
      sfor<NS>([&](auto E) {
        constexpr int ne = ref::entity_nodes(D, 2 * K, E);
        if constexpr (ne > 0) {
          const bool own = (mask >> E) & 1u;
          const T* dp = dw + ws.base[E] + ws.rank[E];
          for (int j = 0; j < ne; ++j) {
            const int i = cslots<D, K>.node[cslots<D, K>.first[E] + j];
            const T* br = bt + i * VT;
            T acc = T(-0.0);
            sfor<VT>([&](auto L) { acc = fma_t(br[L], ue[L], acc); });
            T dv = T(0);
            if (own) dv = __builtin_nontemporal_load(dp + j * ws.cnt[E]);
            const T h = dv * acc;
            sfor<VT>([&](auto L) { ye[L] = fma_t(br[L], h, ye[L]); });
          }
        }
      });
    }
  }
};

// Element body of the conventional quadrature-point apply: for each point q,
// g = G_q u_T (values, or reference gradients), h = s_q g (projection) or s_q K_T g
// (elliptic, K_T = R^-1 R^-T), y_T += G_q^T h; s_q = w_q |det R_T| a(x_q).  The table
// index is wave-uniform.
template <int D, int K, int KIND, typename T>
struct ElemQ {
  static constexpr int VT = dim_p(D, K), NB = KIND == KIND_SE ? D : 1, S = KIND == KIND_SE ? n_sym(D) : 1;

  __device__ __forceinline__ static void run(const ApplyLaunch& a, int64_t w, int lane, const T (&ue)[VT],
                                             T (&ye)[VT]) {
    const T* qs = static_cast<const T*>(a.qs) + (w * a.nq) * 64 + lane;
    const T* G = static_cast<const T*>(a.qtab);
    T kc[S];
    if constexpr (KIND == KIND_SE) {
      const T* qk = static_cast<const T*>(a.qk) + (w * S) * 64 + lane;
      sfor<S>([&](auto C) { kc[C] = qk[C * 64]; });
    }
    sfor<VT>([&](auto L) { ye[L] = T(-0.0); });
    for (int q = 0; q < a.nq; ++q) {
      const T sq = __builtin_nontemporal_load(qs + q * 64);
      const T* gq = G + q * NB * VT;
      T g[NB];
      sfor<NB>([&](auto R) {
        T acc = T(-0.0);
        sfor<VT>([&](auto L) { acc = fma_t(gq[R * VT + L], ue[L], acc); });
        g[R] = acc;
      });
      T h[NB];
      if constexpr (KIND == KIND_SE) {
        dmul<NB, S>(kc, g, h);
        sfor<NB>([&](auto R) { h[R] = sq * h[R]; });
      } else {
        h[0] = sq * g[0];
      }
      sfor<NB>([&](auto R) { sfor<VT>([&](auto L) { ye[L] = fma_t(gq[R * VT + L], h[R], ye[L]); }); });
    }
  }
};

// Local indices of one cell: nlc 16-byte chunks of 8 uint16 slots, AoSoA by 64 cells.
template <int VT>
__device__ __forceinline__ void load_lidx(const uint16_t* __restrict__ lidx, int64_t w, int nlc, int lane,
                                          int (&li)[VT]) {
  const vec_t<uint32_t, 4>* p = reinterpret_cast<const vec_t<uint32_t, 4>*>(lidx) + (w * nlc) * 64 + lane;
  sfor<(VT + 7) / 8>([&](auto C) {
    const vec_t<uint32_t, 4> c = p[C * 64];
    sfor<8>([&](auto J) {
      constexpr int l = C * 8 + J;
      if constexpr (l < VT) li[l] = int((c[J / 2] >> (16 * (J % 2))) & 0xffffu);
    });
  });
}

// Sum over the workgroup (any size that is a multiple of 64), result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

}  // namespace dev

// Launch with `lds` bytes of dynamic LDS; above 64 KB the kernel's limit is raised first
// (a gfx950 workgroup may hold up to 160 KB).
template <typename Kern, typename... Args>
void launch_lds(Kern k, dim3 grid, dim3 block, size_t lds, hipStream_t st, Args... args) {
  if (lds > 65536)
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  hipLaunchKernelGGL(k, grid, block, lds, st, args...);
}

// Launch a tile kernel (one workgroup per tile) whose launch record L carries te and cpl
// (cells per lane; 0: the lanes of tile_lanes); extra arguments follow the record.
template <typename Kern, typename L, typename... Args>
void launch_tiles(Kern k, const L& a0, size_t lds, hipStream_t st, Args... args) {
  L a = a0;
  a.cpl = a.te / tile_lanes(reinterpret_cast<const void*>(k), a.te, lds, a.cpl > 0 ? a.te / a.cpl : 0);
  launch_lds(k, dim3(unsigned(a.ntiles)), dim3(unsigned(a.te / a.cpl)), lds, st, a, args...);
}

namespace dev {

// Ordered accumulation without workgroup barriers: the waves of a tile add their cells'
// sums into LDS in a fixed order of turns 0, 1, 2, ... counted in LDS.  A wave polls (with
// s_sleep) until the counter reaches its turn, adds, and passes the turn on with a release,
// so every slot receives its terms in the same order as with a barrier after each wave, and
// waves that are not adding go on with their next pass.  The wait is bounded (about 0.1 s
// of polling, then the wave goes on unordered), so a broken turn sequence cannot hang.
__device__ __forceinline__ void wait_turn(const int* turn, int my) {
  for (int it = 0; __hip_atomic_load(turn, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != my; ++it) {
    if (it > (1 << 22)) break;
    __builtin_amdgcn_s_sleep(1);
  }
}
__device__ __forceinline__ void pass_turn(int* turn) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(turn, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Cell of tile t that lane threadIdx.x takes in pass c: a tile of a.te cells runs on
// a.te / a.cpl lanes in a.cpl passes, pass c holding tile cells [c * lanes, (c + 1) * lanes).
// Lanes beyond a smaller tile (batched launches) get a.nel (no cell).
template <typename L>
__device__ __forceinline__ int64_t tile_cell(const L& a, int64_t t, int c) {
  const int lanes = a.te / a.cpl;
  return int(threadIdx.x) < lanes ? t * a.te + int64_t(c) * lanes + threadIdx.x : a.nel;
}

// Add one pass's per-cell contributions ye into the tile's LDS sums, one wave after the
// other (passes in order), so that the sums are bitwise reproducible.
template <int VT, typename L>
__device__ __forceinline__ void diag_accumulate(const L& a, int64_t e, const int (&li)[VT], const double (&ye)[VT],
                                                double* ys) {
  const int nw = (a.te / a.cpl + 63) >> 6, me = int(threadIdx.x >> 6);
  for (int wv = 0; wv < nw; ++wv) {
    if (me == wv && e < a.nel) sfor<VT>([&](auto J) { atomicAdd(&ys[li[J]], ye[J]); });
    __syncthreads();
  }
}

// Store a tile's sums: exclusive dofs to out, Dirichlet rows 1, shared dofs to the
// staging buffer for the second pass, which adds them in a fixed order.  The diagonal is
// the same bit for bit from run to run.
template <typename L>
__device__ __forceinline__ void diag_store(const L& a, int64_t t, const double* ys, double* __restrict__ out) {
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  double* stage = a.stage + a.stage_off[t];
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) {
    const uint32_t td = a.tile_dofs[o0 + j];
    const uint32_t dof = td & TD_MASK;
    if (td & TD_BND)
      out[dof] = 1.0;
    else if (td & TD_SHARED)
      stage[j] = ys[j];
    else
      out[dof] = ys[j];
  }
}

}  // namespace dev
}  // namespace dogip
