// Setup and auxiliary kernels: D construction (Theorems 2 and 4), D export,
// Jacobi diagonal, adjoint contraction, small vector kernels.
#include <algorithm>

#include "kern_common.hpp"

namespace dogip {
namespace dev {

// ---- D construction: one thread per cell (internal order) ----
// Projection: D_T,i = w^_i |T| m_T.  Elliptic: D_T,i = w^_i |T| R_T^-1 M_T R_T^-T
// (packed symmetric).  |T| = |det R_T| / d!, R_T columns X_r - X_0.
__global__ __launch_bounds__(256) void k_build_d(BuildDLaunch a) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= a.nel) return;
  const int dim = a.dim, d1 = dim + 1, ns = a.nsym, wt = a.wt;
  const int64_t uc = a.perm[e];
  auto store = [&](int f, double v) {
    a.d64[((e >> 6) * a.nch64 + (f >> 1)) * 128 + (e & 63) * 2 + (f & 1)] = v;
    if (a.d32) a.d32[d32_pos(e >> 6, int(e & 63), f, a.nch32)] = float(v);
  };
  if (a.coef_kind == DOGIP_COEF_RAW_D) {
    const int nd = wt * ns;
    for (int f = 0; f < nd; ++f) store(f, a.coef[uc * nd + f]);
    return;
  }
  double X[4][3] = {};
  for (int j = 0; j < d1; ++j) {
    const int64_t v = a.cells[e * d1 + j];
    for (int x = 0; x < dim; ++x) X[j][x] = a.xyz[v * dim + x];
  }
  double R[3][3] = {}, Ri[3][3] = {}, det;
  for (int x = 0; x < dim; ++x)
    for (int r = 0; r < dim; ++r) R[x][r] = X[r + 1][x] - X[0][x];
  if (dim == 2) {
    det = R[0][0] * R[1][1] - R[0][1] * R[1][0];
    Ri[0][0] = R[1][1] / det;
    Ri[0][1] = -R[0][1] / det;
    Ri[1][0] = -R[1][0] / det;
    Ri[1][1] = R[0][0] / det;
  } else {
    const double c00 = R[1][1] * R[2][2] - R[1][2] * R[2][1];
    const double c01 = R[1][2] * R[2][0] - R[1][0] * R[2][2];
    const double c02 = R[1][0] * R[2][1] - R[1][1] * R[2][0];
    det = R[0][0] * c00 + R[0][1] * c01 + R[0][2] * c02;
    Ri[0][0] = c00 / det;
    Ri[1][0] = c01 / det;
    Ri[2][0] = c02 / det;
    Ri[0][1] = (R[0][2] * R[2][1] - R[0][1] * R[2][2]) / det;
    Ri[1][1] = (R[0][0] * R[2][2] - R[0][2] * R[2][0]) / det;
    Ri[2][1] = (R[0][1] * R[2][0] - R[0][0] * R[2][1]) / det;
    Ri[0][2] = (R[0][1] * R[1][2] - R[0][2] * R[1][1]) / det;
    Ri[1][2] = (R[0][2] * R[1][0] - R[0][0] * R[1][2]) / det;
    Ri[2][2] = (R[0][0] * R[1][1] - R[0][1] * R[1][0]) / det;
  }
  const double vol = fabs(det) / (dim == 2 ? 2.0 : 6.0);
  double K[6] = {};
  if (a.kind == KIND_WP) {
    const double c = a.coef[uc];
    K[0] = a.coef_kind == DOGIP_COEF_LOGSCALAR ? exp(c) : c;
  } else {
    double M[3][3] = {};
    if (a.coef_kind == DOGIP_COEF_SYM) {
      int c = 0;
      for (int r = 0; r < dim; ++r)
        for (int s = r; s < dim; ++s) {
          M[r][s] = M[s][r] = a.coef[uc * ns + c];
          ++c;
        }
    } else {
      const double c = a.coef[uc];
      const double m = a.coef_kind == DOGIP_COEF_LOGSCALAR ? exp(c) : c;
      for (int r = 0; r < dim; ++r) M[r][r] = m;
    }
    int c = 0;
    for (int r = 0; r < dim; ++r)
      for (int s = r; s < dim; ++s) {
        double acc = 0.0;
        for (int p = 0; p < dim; ++p)
          for (int q = 0; q < dim; ++q) acc += Ri[r][p] * M[p][q] * Ri[s][q];
        K[c++] = acc;
      }
  }
  for (int i = 0; i < wt; ++i) {
    const double wv = a.what[i] * vol;
    for (int c = 0; c < ns; ++c) store(i * ns + c, wv * K[c]);
  }
}

__global__ __launch_bounds__(256) void k_export_d(const double* __restrict__ d64, const int32_t* __restrict__ perm,
                                                  double* __restrict__ out, int64_t nel, int64_t nch64, int nd) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nel * nd) return;
  const int64_t e = i / nd;
  const int f = int(i % nd);
  out[int64_t(perm[e]) * nd + f] = d64[((e >> 6) * nch64 + (f >> 1)) * 128 + (e & 63) * 2 + (f & 1)];
}

__global__ __launch_bounds__(256) void k_zero_indexed(double* __restrict__ y, const int32_t* __restrict__ idx,
                                                      int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[idx[i]] = 0.0;
}

// The finish entries of one thread (FINISH_PER_THREAD of them, FINISH_THREADS apart from
// i0): every index and partial sum is requested before any is used, so the loads of the
// entries are in flight together.  Shared dof i: its partial sums added in ascending tile
// order from zero (pair lists: the first two slots, then any others).  Dirichlet entry:
// y[b] = u[b] and u_b^2 into eb.
template <typename V>
__device__ __forceinline__ void finish_entries(int64_t i0, const double* __restrict__ stage,
                                               const uint32_t* __restrict__ pair, const uint32_t* __restrict__ more_off,
                                               const uint32_t* __restrict__ more, const int32_t* __restrict__ shared,
                                               int64_t nshared, const int32_t* __restrict__ bnd, int64_t nbnd,
                                               const V* __restrict__ u, V* __restrict__ y, double& eb) {
  constexpr int E = FINISH_PER_THREAD;
  vec_t<uint32_t, 2> pr[E];
  uint32_t m0[E], m1[E];
  int32_t dst[E];
  double p0[E], p1[E];
  // step 1: indices (the range of further slots is requested with the pair, so a dof with more
  // than two partials waits for one dependent load less)
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int64_t i = i0 + int64_t(c) * FINISH_THREADS;
    m0[c] = m1[c] = 0;
    if (i < nshared) {
      pr[c] = reinterpret_cast<const vec_t<uint32_t, 2>*>(pair)[i];
      dst[c] = shared[i];
      m0[c] = more_off[i];
      m1[c] = more_off[i + 1];
    } else if (i < nshared + nbnd) {
      dst[c] = bnd[i - nshared];
    }
  }
  // step 2: the first two partials (or u on Dirichlet rows) and the first further slot
  uint32_t s2[E];
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int64_t i = i0 + int64_t(c) * FINISH_THREADS;
    if (i < nshared) {
      p0[c] = stage[pr[c][0]];
      p1[c] = stage[pr[c][1] & 0x7fffffffu];
      if (m1[c] > m0[c]) s2[c] = more[m0[c]];
    } else if (i < nshared + nbnd) {
      p0[c] = double(u[dst[c]]);
    }
  }
#pragma unroll
  for (int c = 0; c < E; ++c) {
    const int64_t i = i0 + int64_t(c) * FINISH_THREADS;
    if (i < nshared) {
      double sum = 0.0;
      sum += p0[c];
      sum += p1[c];
      if (m1[c] > m0[c]) {
        sum += stage[s2[c]];
        for (uint32_t j = m0[c] + 1; j < m1[c]; ++j) sum += stage[more[j]];
      }
      y[dst[c]] = V(sum);
    } else if (i < nshared + nbnd) {
      y[dst[c]] = V(p0[c]);
      eb += p0[c] * p0[c];
    }
  }
}

// Second pass of the apply.  i < nshared: y[shared[i]] = sum of its staged partials,
// added in ascending tile order (deterministic).  nshared <= i < nshared + nbnd:
// Dirichlet identity row y[b] = u[b]; with benergy, every block from e0 on writes its
// share of sum u_b^2 (the identity rows' part of u . A u) to benergy[blockIdx.x - e0].
// FINISH_PER_THREAD entries per thread, FINISH_THREADS apart (independent loads in
// flight, coalesced per step): the grid covers nshared + nbnd.
__global__ __launch_bounds__(FINISH_THREADS) void k_apply_finish(const double* __restrict__ stage,
                                                      const uint32_t* __restrict__ pair,
                                                      const uint32_t* __restrict__ more_off,
                                                      const uint32_t* __restrict__ more,
                                                      const int32_t* __restrict__ shared, int64_t nshared,
                                                      const int32_t* __restrict__ bnd, int64_t nbnd,
                                                      const double* __restrict__ u, double* __restrict__ y,
                                                      double* __restrict__ benergy, int64_t e0) {
  double eb = 0.0;
  finish_entries(int64_t(blockIdx.x) * FINISH_ENTRIES + threadIdx.x, stage, pair, more_off, more, shared, nshared, bnd,
                 nbnd, u, y, eb);
  if (benergy && int64_t(blockIdx.x) >= e0) {  // block-uniform
    __shared__ double red[8];
    const double s = block_sum(eb, red);
    if (threadIdx.x == 0) benergy[blockIdx.x - e0] = s;
  }
}

// The second pass on FP32 vectors (mixed CG): partial sums added in FP64, stored in FP32.
__global__ __launch_bounds__(FINISH_THREADS) void k_apply_finish32(const double* __restrict__ stage,
                                                        const uint32_t* __restrict__ pair,
                                                        const uint32_t* __restrict__ more_off,
                                                        const uint32_t* __restrict__ more,
                                                        const int32_t* __restrict__ shared, int64_t nshared,
                                                        const int32_t* __restrict__ bnd, int64_t nbnd,
                                                        const float* __restrict__ u, float* __restrict__ y,
                                                        double* __restrict__ benergy, int64_t e0) {
  double eb = 0.0;
  finish_entries(int64_t(blockIdx.x) * FINISH_ENTRIES + threadIdx.x, stage, pair, more_off, more, shared, nshared, bnd,
                 nbnd, u, y, eb);
  if (benergy && int64_t(blockIdx.x) >= e0) {  // block-uniform
    __shared__ double red[8];
    const double s = block_sum(eb, red);
    if (threadIdx.x == 0) benergy[blockIdx.x - e0] = s;
  }
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = float(x[i]);
}

__global__ __launch_bounds__(256) void k_invert(const double* __restrict__ d, double* __restrict__ inv, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    inv[i] = 1.0 / d[i];
}

// ---- global projection form: D_j = sum over the cells holding W dof j of m_T |T| w^_i ----
// (raw D: the cells' values summed).  One thread per W dof in tile layout; the
// incidences are in ascending cell order, so the sums are reproducible.
__global__ __launch_bounds__(256) void k_build_dg(BuildDLaunch a, const int64_t* __restrict__ inc_ptr,
                                                  const int64_t* __restrict__ inc, int64_t nw, double* __restrict__ dg64,
                                                  float* __restrict__ dg32) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nw) return;
  const int dim = a.dim, d1 = dim + 1, wt = a.wt;
  double acc = 0.0;
  for (int64_t q = inc_ptr[j]; q < inc_ptr[j + 1]; ++q) {
    const int64_t e = inc[q] / wt;
    const int i = int(inc[q] - e * wt);
    const int64_t uc = a.perm[e];
    if (a.coef_kind == DOGIP_COEF_RAW_D) {
      acc += a.coef[uc * wt + i];
      continue;
    }
    double X[4][3] = {};
    for (int v = 0; v < d1; ++v) {
      const int64_t g = a.cells[e * d1 + v];
      for (int x = 0; x < dim; ++x) X[v][x] = a.xyz[g * dim + x];
    }
    double det;
    if (dim == 2) {
      det = (X[1][0] - X[0][0]) * (X[2][1] - X[0][1]) - (X[2][0] - X[0][0]) * (X[1][1] - X[0][1]);
    } else {
      double R[3][3];
      for (int x = 0; x < 3; ++x)
        for (int r = 0; r < 3; ++r) R[x][r] = X[r + 1][x] - X[0][x];
      det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
            R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
    }
    const double vol = fabs(det) / (dim == 2 ? 2.0 : 6.0);
    const double c = a.coef[uc];
    const double m = a.coef_kind == DOGIP_COEF_LOGSCALAR ? exp(c) : c;
    acc += a.what[i] * vol * m;
  }
  dg64[j] = acc;
  if (dg32) dg32[j] = float(acc);
}

// ---- Jacobi diagonal: diag_l = sum_T sum_i b_il^T D_T,i b_il, b_il = (B^[r][i][l])_r ----
template <int D, int K, int KIND>
__global__ __launch_bounds__(512) void k_diag(DiagLaunch a) {
  using TB = ref::BTable<D, K, KIND>;
  constexpr int VT = TB::VT, WT = TB::WT, NB = TB::NB, S = KIND == KIND_SE ? n_sym(D) : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* ys = reinterpret_cast<double*>(smem);
  const int64_t t = blockIdx.x;
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) ys[j] = 0.0;
  __syncthreads();
  for (int c = 0; c < a.cpl; ++c) {
  const int64_t e = tile_cell(a, t, c);
  int li[VT];
  double ye[VT];
  if (e < a.nel) {
    const int lane = threadIdx.x & 63;
    const int64_t w = e >> 6;
    load_lidx<VT>(a.lidx, w, a.nlc, lane, li);
    const double* dsc = a.D + (w * a.nch) * 128 + lane * 2;
    const double* bt = ctab<D, K, KIND, double>.v;
    sfor<VT>([&](auto L) { ye[L] = 0.0; });
    for (int i = 0; i < WT; ++i) {
      double dv[S];
      sfor<S>([&](auto C) {
        const int f = i * S + C;
        dv[C] = dsc[(f >> 1) * 128 + (f & 1)];
      });
      sfor<VT>([&](auto L) {
        double b[NB];
        sfor<NB>([&](auto R) { b[R] = bt[(R * WT + i) * VT + L]; });
        double h[NB];
        dmul<NB, S>(dv, b, h);
        double s = 0.0;
        sfor<NB>([&](auto R) { s = fma_t(b[R], h[R], s); });
        ye[L] += s;
      });
    }
  }
  diag_accumulate<VT>(a, e, li, ye, ys);
  }
  diag_store(a, t, ys, a.out);
}

// ---- Jacobi diagonal of the global projection form: diag_l = sum_j B_jl^2 D_j, each
// W dof j taken by the cell that owns it ----
template <int D, int K>
__global__ __launch_bounds__(512) void k_diag_g(DiagLaunch a) {
  using TB = ref::BTable<D, K, KIND_WP>;
  constexpr int VT = TB::VT;
  extern __shared__ __align__(16) unsigned char smem[];
  double* ys = reinterpret_cast<double*>(smem);
  const int64_t t = blockIdx.x;
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) ys[j] = 0.0;
  __syncthreads();
  for (int c = 0; c < a.cpl; ++c) {
  const int64_t e = tile_cell(a, t, c);
  int li[VT];
  double ye[VT];
  if (e < a.nel) {
    const int lane = threadIdx.x & 63;
    load_lidx<VT>(a.lidx, e >> 6, a.nlc, lane, li);
    const uint32_t mask = a.gw_mask[e];
    const WaveSlots<D, K> ws(mask);
    const double* dw = a.D + a.gw_woff[e >> 6];
    const double* bt = ctab<D, K, KIND_WP, double>.v;
    sfor<VT>([&](auto L) { ye[L] = 0.0; });
    sfor<gw_slots(D)>([&](auto E) {
      constexpr int ne = ref::entity_nodes(D, 2 * K, E);
      if constexpr (ne > 0) {
        if ((mask >> E) & 1u) {
          for (int j = 0; j < ne; ++j) {
            const int i = cslots<D, K>.node[cslots<D, K>.first[E] + j];
            const double dv = dw[ws.base[E] + j * ws.cnt[E] + ws.rank[E]];
            sfor<VT>([&](auto L) {
              const double b = bt[i * VT + L];
              ye[L] = fma(b * b, dv, ye[L]);
            });
          }
        }
      }
    });
  }
  diag_accumulate<VT>(a, e, li, ye, ys);
  }
  diag_store(a, t, ys, a.out);
}

// ---- adjoint contraction: g_T = -(B^ lam_T) . D_T (B^ u_T), boundary entries zero ----
template <int D, int K, int KIND>
__global__ __launch_bounds__(512) void k_grad(GradLaunch a) {
  using TB = ref::BTable<D, K, KIND>;
  constexpr int VT = TB::VT, WT = TB::WT, NB = TB::NB, S = KIND == KIND_SE ? n_sym(D) : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* us = reinterpret_cast<double*>(smem);
  double* ls = us + a.lds_slots;
  const int64_t t = blockIdx.x;
  const int64_t o0 = a.tile_off[t], nd = a.tile_off[t + 1] - o0;
  for (int64_t j = threadIdx.x; j < nd; j += blockDim.x) {
    const uint32_t td = a.tile_dofs[o0 + j];
    const bool b = td & TD_BND;
    us[j] = b ? 0.0 : a.u[td & TD_MASK];
    ls[j] = b ? 0.0 : a.lam[td & TD_MASK];
  }
  __syncthreads();
  for (int c = 0; c < a.cpl; ++c) {
  const int64_t e = tile_cell(a, t, c);
  if (e >= a.nel) break;
  const int lane = threadIdx.x & 63;
  const int64_t w = e >> 6;
  int li[VT];
  load_lidx<VT>(a.lidx, w, a.nlc, lane, li);
  double ue[VT], le[VT];
  sfor<VT>([&](auto L) {
    ue[L] = us[li[L]];
    le[L] = ls[li[L]];
  });
  const double* dsc = a.D + (w * a.nch) * 128 + lane * 2;
  const double* bt = ctab<D, K, KIND, double>.v;
  double en = 0.0;
  for (int i = 0; i < WT; ++i) {
    double gu[NB], gl[NB];
    sfor<NB>([&](auto R) {
      double su = 0.0, sl = 0.0;
      sfor<VT>([&](auto L) {
        const double b = bt[(R * WT + i) * VT + L];
        su = fma_t(b, ue[L], su);
        sl = fma_t(b, le[L], sl);
      });
      gu[R] = su;
      gl[R] = sl;
    });
    double dv[S];
    sfor<S>([&](auto C) {
      const int f = i * S + C;
      dv[C] = dsc[(f >> 1) * 128 + (f & 1)];
    });
    double h[NB];
    dmul<NB, S>(dv, gu, h);
    sfor<NB>([&](auto R) { en = fma_t(gl[R], h[R], en); });
  }
  a.g[a.perm[e]] = -en;
  }
}

template <int D, int K, int KIND>
void diag_t(const DiagLaunch& a, hipStream_t st) {
  launch_tiles((k_diag<D, K, KIND>), a, size_t(a.lds_slots) * sizeof(double), st);
}
template <int D, int K, int KIND>
void grad_t(const GradLaunch& a, hipStream_t st) {
  launch_tiles((k_grad<D, K, KIND>), a, size_t(2) * a.lds_slots * sizeof(double), st);
}

}  // namespace dev

static unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return unsigned(g);
}

void launch_build_d(const BuildDLaunch& a, hipStream_t st) {
  if (a.nel <= 0) return;
  hipLaunchKernelGGL(dev::k_build_d, dim3(unsigned((a.nel + 255) / 256)), dim3(256), 0, st, a);
}

void launch_build_dg(const BuildDLaunch& a, const int64_t* inc_ptr, const int64_t* inc, int64_t nw, double* dg64,
                     float* dg32, hipStream_t st) {
  if (nw <= 0) return;
  hipLaunchKernelGGL(dev::k_build_dg, dim3(unsigned((nw + 255) / 256)), dim3(256), 0, st, a, inc_ptr, inc, nw, dg64,
                     dg32);
}

void launch_diag_global(int dim, int k, const DiagLaunch& a, hipStream_t st) {
  const size_t lds = size_t(a.lds_slots) * sizeof(double);
  switch (dim * 16 + k) {
    case 32 + 1: launch_tiles((dev::k_diag_g<2, 1>), a, lds, st); break;
    case 32 + 2: launch_tiles((dev::k_diag_g<2, 2>), a, lds, st); break;
    case 32 + 3: launch_tiles((dev::k_diag_g<2, 3>), a, lds, st); break;
    case 32 + 4: launch_tiles((dev::k_diag_g<2, 4>), a, lds, st); break;
    case 32 + 5: launch_tiles((dev::k_diag_g<2, 5>), a, lds, st); break;
    case 32 + 6: launch_tiles((dev::k_diag_g<2, 6>), a, lds, st); break;
    case 32 + 7: launch_tiles((dev::k_diag_g<2, 7>), a, lds, st); break;
    case 32 + 8: launch_tiles((dev::k_diag_g<2, 8>), a, lds, st); break;
    case 48 + 1: launch_tiles((dev::k_diag_g<3, 1>), a, lds, st); break;
    case 48 + 2: launch_tiles((dev::k_diag_g<3, 2>), a, lds, st); break;
    case 48 + 3: launch_tiles((dev::k_diag_g<3, 3>), a, lds, st); break;
    case 48 + 4: launch_tiles((dev::k_diag_g<3, 4>), a, lds, st); break;
    default: throw Error(DOGIP_E_RANGE, "no kernel for this (dim, k)");
  }
}

void launch_export_d(const double* d64, const int32_t* perm, double* out, int64_t nel, int64_t nch64, int wt, int nsym,
                     hipStream_t st) {
  const int64_t n = nel * wt * nsym;
  hipLaunchKernelGGL(dev::k_export_d, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, d64, perm, out, nel, nch64,
                     wt * nsym);
}

void launch_zero_indexed(double* y, const int32_t* idx, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_zero_indexed, dim3(grid_for(n, 256)), dim3(256), 0, st, y, idx, n);
}

void launch_apply_finish(const double* stage, const uint32_t* pair, const uint32_t* more_off, const uint32_t* more,
                         const int32_t* shared, int64_t nshared, const int32_t* bnd, int64_t nbnd, const double* u,
                         double* y, double* benergy, hipStream_t st) {
  if (nshared + nbnd <= 0 && !benergy) return;
  const unsigned grid = unsigned(finish_blocks(nshared, nbnd));
  hipLaunchKernelGGL(dev::k_apply_finish, dim3(grid), dim3(FINISH_THREADS), 0, st, stage, pair, more_off, more, shared,
                     nshared, bnd, nbnd, u, y, benergy, finish_first_energy_block(nshared, nbnd));
}

void launch_apply_finish32(const double* stage, const uint32_t* pair, const uint32_t* more_off, const uint32_t* more,
                           const int32_t* shared, int64_t nshared, const int32_t* bnd, int64_t nbnd, const float* u,
                           float* y, double* benergy, hipStream_t st) {
  if (nshared + nbnd <= 0 && !benergy) return;
  const unsigned grid = unsigned(finish_blocks(nshared, nbnd));
  hipLaunchKernelGGL(dev::k_apply_finish32, dim3(grid), dim3(FINISH_THREADS), 0, st, stage, pair, more_off, more,
                     shared, nshared, bnd, nbnd, u, y, benergy, finish_first_energy_block(nshared, nbnd));
}

void launch_to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, st, x, y, n);
}

void launch_invert(const double* d, double* inv, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_invert, dim3(grid_for(n, 256)), dim3(256), 0, st, d, inv, n);
}

#define DOGIP_DG_CASES(F)                                                                                          \
  switch (dim * 1000 + kind * 16 + k) {                                                                            \
    case 2000 + 1: F<2, 1, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 2: F<2, 2, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 3: F<2, 3, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 4: F<2, 4, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 5: F<2, 5, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 6: F<2, 6, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 7: F<2, 7, KIND_WP>(a, st); break;                                                                 \
    case 2000 + 8: F<2, 8, KIND_WP>(a, st); break;                                                                 \
    case 2016 + 1: F<2, 1, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 2: F<2, 2, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 3: F<2, 3, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 4: F<2, 4, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 5: F<2, 5, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 6: F<2, 6, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 7: F<2, 7, KIND_SE>(a, st); break;                                                                 \
    case 2016 + 8: F<2, 8, KIND_SE>(a, st); break;                                                                 \
    case 3000 + 1: F<3, 1, KIND_WP>(a, st); break;                                                                 \
    case 3000 + 2: F<3, 2, KIND_WP>(a, st); break;                                                                 \
    case 3000 + 3: F<3, 3, KIND_WP>(a, st); break;                                                                 \
    case 3000 + 4: F<3, 4, KIND_WP>(a, st); break;                                                                 \
    case 3016 + 1: F<3, 1, KIND_SE>(a, st); break;                                                                 \
    case 3016 + 2: F<3, 2, KIND_SE>(a, st); break;                                                                 \
    case 3016 + 3: F<3, 3, KIND_SE>(a, st); break;                                                                 \
    case 3016 + 4: F<3, 4, KIND_SE>(a, st); break;                                                                 \
    default: throw Error(DOGIP_E_RANGE, "no kernel for this (dim, k, kind)");                                     \
  }

void launch_diag(int dim, int k, int kind, const DiagLaunch& a, hipStream_t st) { DOGIP_DG_CASES(dev::diag_t) }
void launch_grad(int dim, int k, int kind, const GradLaunch& a, hipStream_t st) { DOGIP_DG_CASES(dev::grad_t) }

}  // namespace dogip
