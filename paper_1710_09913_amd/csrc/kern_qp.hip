// Conventional quadrature-point apply (the matrix-free evaluation over integration
// points that Section 3.3 compares DoGIP with): per-point factors, apply and Jacobi
// diagonal kernels.
#include "kern_apply.hpp"

namespace dogip {
namespace dev {

// One thread per cell (internal order): s_q = w_q |det R_T| a(x_q) -> AoSoA
// [(e/64)][q][64]; elliptic: K_T = R^-1 R^-T packed upper triangle -> [(e/64)][c][64].
__global__ __launch_bounds__(256) void k_qp_setup(QpSetupLaunch a) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= a.nel) return;
  const int dim = a.dim, d1 = dim + 1;
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
  const double J = fabs(det);
  const int64_t uc = a.perm[e], w = e >> 6, lane = e & 63;
  for (int q = 0; q < a.nq; ++q) {
    const double s = a.w[q] * J * a.coef[uc * a.nq + q];
    const int64_t at = (w * a.nq + q) * 64 + lane;
    a.qs64[at] = s;
    if (a.qs32) a.qs32[at] = float(s);
  }
  if (a.kind == KIND_SE) {
    const int ns = dim * (dim + 1) / 2;
    int c = 0;
    for (int r = 0; r < dim; ++r)
      for (int t = r; t < dim; ++t) {
        double acc = 0.0;
        for (int p = 0; p < dim; ++p) acc += Ri[r][p] * Ri[t][p];
        const int64_t at = (w * ns + c) * 64 + lane;
        a.qk64[at] = acc;
        if (a.qk32) a.qk32[at] = float(acc);
        ++c;
      }
  }
}

template <int D, int K, int KIND, typename T, bool ENERGY>
__global__ __launch_bounds__(512, DOGIP_WPE) void k_apply_q(ApplyLaunch a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = a.tile_base + xcd_tile(blockIdx.x, gridDim.x);
  tile_body<D, K, KIND, T, DOGIP_VARIANT_LOOPED, ENERGY, 0, 2>(a, t, smem, ENERGY ? a.energy + t : nullptr);
}

template <int D, int K, int KIND>
bool launch_apply_q_t(int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  if (prec == DOGIP_F64) {
    const size_t lds = size_t(a.lds_slots) * (sizeof(double) + sizeof(double));
    if (energy)
      launch_tiles((k_apply_q<D, K, KIND, double, true>), a, lds, st);
    else
      launch_tiles((k_apply_q<D, K, KIND, double, false>), a, lds, st);
  } else {
    const size_t lds = size_t(a.lds_slots) * (sizeof(double) + sizeof(float));
    if (energy)
      launch_tiles((k_apply_q<D, K, KIND, float, true>), a, lds, st);
    else
      launch_tiles((k_apply_q<D, K, KIND, float, false>), a, lds, st);
  }
  return true;
}

// Jacobi diagonal: diag_l = sum_q s_q G_q,l^T K_T G_q,l (FP64 tables).
template <int D, int K, int KIND>
__global__ __launch_bounds__(512) void k_diag_q(ApplyLaunch a, double* __restrict__ out) {
  constexpr int VT = dim_p(D, K), NB = KIND == KIND_SE ? D : 1, S = KIND == KIND_SE ? n_sym(D) : 1;
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
    const double* qs = static_cast<const double*>(a.qs) + (w * a.nq) * 64 + lane;
    const double* G = static_cast<const double*>(a.qtab);
    double kc[S];
    if constexpr (KIND == KIND_SE) {
      const double* qk = static_cast<const double*>(a.qk) + (w * S) * 64 + lane;
      sfor<S>([&](auto C) { kc[C] = qk[C * 64]; });
    }
    sfor<VT>([&](auto L) { ye[L] = 0.0; });
    for (int q = 0; q < a.nq; ++q) {
      const double sq = qs[q * 64];
      const double* gq = G + q * NB * VT;
      sfor<VT>([&](auto L) {
        double b[NB], h[NB];
        sfor<NB>([&](auto R) { b[R] = gq[R * VT + L]; });
        if constexpr (KIND == KIND_SE)
          dmul<NB, S>(kc, b, h);
        else
          h[0] = b[0];
        double s = 0.0;
        sfor<NB>([&](auto R) { s = fma(b[R], h[R], s); });
        ye[L] = fma(sq, s, ye[L]);
      });
    }
  }
  diag_accumulate<VT>(a, e, li, ye, ys);
  }
  diag_store(a, t, ys, out);
}

template <int D, int K, int KIND>
void diag_q_t(const ApplyLaunch& a, double* out, hipStream_t st) {
  launch_tiles((k_diag_q<D, K, KIND>), a, size_t(a.lds_slots) * sizeof(double), st, out);
}

}  // namespace dev

void launch_qp_setup(const QpSetupLaunch& a, hipStream_t st) {
  if (a.nel <= 0) return;
  hipLaunchKernelGGL(dev::k_qp_setup, dim3(unsigned((a.nel + 255) / 256)), dim3(256), 0, st, a);
}

#define DOGIP_QP_CASES(F, ...)                                      \
  switch (dim * 1000 + kind * 16 + k) {                             \
    case 2000 + 1: F<2, 1, KIND_WP>(__VA_ARGS__); break;            \
    case 2000 + 2: F<2, 2, KIND_WP>(__VA_ARGS__); break;            \
    case 2000 + 3: F<2, 3, KIND_WP>(__VA_ARGS__); break;            \
    case 2000 + 4: F<2, 4, KIND_WP>(__VA_ARGS__); break;            \
    case 2000 + 5: F<2, 5, KIND_WP>(__VA_ARGS__); break;            \
    case 2016 + 1: F<2, 1, KIND_SE>(__VA_ARGS__); break;            \
    case 2016 + 2: F<2, 2, KIND_SE>(__VA_ARGS__); break;            \
    case 2016 + 3: F<2, 3, KIND_SE>(__VA_ARGS__); break;            \
    case 2016 + 4: F<2, 4, KIND_SE>(__VA_ARGS__); break;            \
    case 2016 + 5: F<2, 5, KIND_SE>(__VA_ARGS__); break;            \
    case 3000 + 1: F<3, 1, KIND_WP>(__VA_ARGS__); break;            \
    case 3000 + 2: F<3, 2, KIND_WP>(__VA_ARGS__); break;            \
    case 3000 + 3: F<3, 3, KIND_WP>(__VA_ARGS__); break;            \
    case 3016 + 1: F<3, 1, KIND_SE>(__VA_ARGS__); break;            \
    case 3016 + 2: F<3, 2, KIND_SE>(__VA_ARGS__); break;            \
    case 3016 + 3: F<3, 3, KIND_SE>(__VA_ARGS__); break;            \
    case 3016 + 4: F<3, 4, KIND_SE>(__VA_ARGS__); break;            \
    default: throw Error(DOGIP_E_RANGE, "no quadrature-point kernel for this (dim, k, kind)"); \
  }

bool launch_apply_qp(int dim, int k, int kind, int prec, const ApplyLaunch& a, hipStream_t st) {
  const bool energy = a.energy != nullptr;
  DOGIP_QP_CASES(dev::launch_apply_q_t, prec, energy, a, st)
  return true;
}

void launch_diag_qp(int dim, int k, int kind, const ApplyLaunch& a, double* out, hipStream_t st) {
  DOGIP_QP_CASES(dev::diag_q_t, a, out, st)
}

}  // namespace dogip
