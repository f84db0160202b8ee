// Vector kernels of the Jacobi-preconditioned CG (FP64 vectors and inner products).
// Reductions are deterministic: a fixed grid of RED_BLOCKS x 256 threads writes
// per-block partials, and a single 1024-thread block sums them in a fixed order.
#include <algorithm>
#include "kern_common.hpp"
#include "solve.hpp"

namespace dogip {
namespace dev {

// Accesses to vectors that a CG iteration (or smoother step) uses once: non-temporal when
// S (the host's stream_vectors: the iteration's vectors and the operator's index arrays
// exceed the memory-side cache), so that the cache keeps the index arrays and the
// direction that the next apply reads; cached otherwise.  At 3D 64^3 P3, Jacobi-PCG to
// 1e-8 with a non-temporal iterate: FP64 0.899 -> 0.856 s, mixed 0.507 -> 0.478 s; with
// A p and the inverse diagonal too (FP64 vectors) 0.856 -> 0.833 s; the multigrid's
// Chebyshev steps 1-2%.  Below the cache size the same accesses cost 2-4% (2D 512^2 P2-P4).
template <bool S>
__device__ __forceinline__ double load_once(const double* a) {
  if constexpr (S)
    return __builtin_nontemporal_load(a);
  else
    return *a;
}
template <bool S>
__device__ __forceinline__ void update_iterate(double* x, int64_t i, double a, double p) {
  if constexpr (S)
    __builtin_nontemporal_store(fma(a, p, __builtin_nontemporal_load(x + i)), x + i);
  else
    x[i] = fma(a, p, x[i]);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce up to 3 values over the block, thread 0 writes part[c * gridDim.x + blockIdx.x].
__device__ __forceinline__ void block_partials(double* v, int nc, double* part) {
  __shared__ double red[3][16];
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = 0; c < nc; ++c) {
    const double s = wave_sum(v[c]);
    if ((threadIdx.x & 63) == 0) red[c][w] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < nc; ++c) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += red[c][i];
      part[c * gridDim.x + blockIdx.x] = s;
    }
}

// Sum n values (strided per thread, then tree) with one block; result in thread 0.
__device__ __forceinline__ double block_total(const double* x, int64_t n) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
  s = wave_sum(s);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

// r = b - y (y may be null: r = b), p = invd r; partials (r.z, r.r, b.b)
__global__ __launch_bounds__(256) void k_pcg_init(const double* __restrict__ b, const double* __restrict__ y,
                                                  const double* __restrict__ invd, double* __restrict__ r,
                                                  double* __restrict__ p, int64_t n, double* __restrict__ part) {
  double v[3] = {0.0, 0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double bi = b[i];
    const double ri = y ? bi - y[i] : bi;
    const double zi = invd[i] * ri;
    r[i] = ri;
    p[i] = zi;
    v[0] += ri * zi;
    v[1] += ri * ri;
    v[2] += bi * bi;
  }
  block_partials(v, 3, part);
}

__global__ __launch_bounds__(1024) void k_fin_init(const double* __restrict__ part, int nparts, PcgScalars* s,
                                                   double* hist) {
  const double rz = block_total(part, nparts);
  const double rr = block_total(part + nparts, nparts);
  const double bb = block_total(part + 2 * nparts, nparts);
  if (threadIdx.x == 0) {
    s->rho = rz;
    s->rr = rr;
    s->bb = bb;
    s->flags = (isfinite(rz) && isfinite(rr) && isfinite(bb)) ? 0 : PCG_NONFINITE;
    hist[0] = rr;
  }
}

// pq = sum of the apply's tile energies; alpha = rho / pq
__global__ __launch_bounds__(1024) void k_fin_pq(const double* __restrict__ energy, int64_t ntiles, PcgScalars* s) {
  const double pq = block_total(energy, ntiles);
  if (threadIdx.x == 0) {
    s->pq = pq;
    if (!isfinite(pq))
      s->flags |= PCG_NONFINITE;
    else if (!(pq > 0.0))
      s->flags |= PCG_BREAKDOWN;
    s->alpha = (pq > 0.0 && s->flags == 0) ? s->rho / pq : 0.0;
  }
}

// x += alpha p, r -= alpha q, z = invd r; partials (r.z, r.r)
template <bool S>
__global__ __launch_bounds__(256) void k_pcg_xr(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                const double* __restrict__ invd, const PcgScalars* __restrict__ s,
                                                int64_t n, double* __restrict__ part) {
  const double alpha = s->alpha;
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    update_iterate<S>(x, i, alpha, p[i]);
    const double ri = fma(-alpha, load_once<S>(q + i), r[i]);
    r[i] = ri;
    v[0] += ri * (load_once<S>(invd + i) * ri);
    v[1] += ri * ri;
  }
  block_partials(v, 2, part);
}

__global__ __launch_bounds__(1024) void k_fin_rz(const double* __restrict__ part, int nparts, PcgScalars* s,
                                                 double* hist, int it) {
  const double rz = block_total(part, nparts);
  const double rr = block_total(part + nparts, nparts);
  if (threadIdx.x == 0) {
    if (!isfinite(rz) || !isfinite(rr)) s->flags |= PCG_NONFINITE;
    s->beta = (s->rho != 0.0 && s->flags == 0) ? rz / s->rho : 0.0;
    s->rho = rz;
    s->rr = rr;
    hist[it] = s->flags ? -1.0 : rr;
  }
}

// p = invd r + beta p
template <bool S>
__global__ __launch_bounds__(256) void k_pcg_p(double* __restrict__ p, const double* __restrict__ r,
                                               const double* __restrict__ invd, const PcgScalars* __restrict__ s,
                                               int64_t n) {
  const double beta = s->beta;
  GRID_STRIDE(i, n) p[i] = fma(beta, p[i], load_once<S>(invd + i) * r[i]);
}

// r = b - y; partial r.r
__global__ __launch_bounds__(256) void k_resid(const double* __restrict__ b, const double* __restrict__ y,
                                               double* __restrict__ r, int64_t n, double* __restrict__ part) {
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    const double ri = b[i] - y[i];
    r[i] = ri;
    v[0] += ri * ri;
  }
  block_partials(v, 1, part);
}

// residual replacement: r = b - y (y = A64 x); partials (r.z, r.r) with z = invd r;
// with p, also restart the search direction p = z
__global__ __launch_bounds__(256) void k_replace(const double* __restrict__ b, const double* __restrict__ y,
                                                 const double* __restrict__ invd, double* __restrict__ r,
                                                 double* __restrict__ p, int64_t n, double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double ri = b[i] - y[i];
    const double zi = invd[i] * ri;
    r[i] = ri;
    if (p) p[i] = zi;
    v[0] += ri * zi;
    v[1] += ri * ri;
  }
  block_partials(v, 2, part);
}

__global__ __launch_bounds__(1024) void k_fin_replace(const double* __restrict__ part, int nparts, PcgScalars* s) {
  const double rz = block_total(part, nparts);
  const double rr = block_total(part + nparts, nparts);
  if (threadIdx.x == 0) {
    if (!isfinite(rz) || !isfinite(rr)) s->flags |= PCG_NONFINITE;
    s->rho = rz;
    s->rr = rr;
  }
}

// partial a.b
__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                             double* __restrict__ part) {
  double v[1] = {0.0};
  GRID_STRIDE(i, n) v[0] += a[i] * b[i];
  block_partials(v, 1, part);
}

__global__ __launch_bounds__(1024) void k_fin_sum(const double* __restrict__ part, int nparts, double* out) {
  const double t = block_total(part, nparts);
  if (threadIdx.x == 0) *out = t;
}

__global__ __launch_bounds__(256) void k_axpy1(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  GRID_STRIDE(i, n) x[i] += d[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ x, double v, int64_t n) {
  GRID_STRIDE(i, n) x[i] = v;
}

// ---- p-multigrid pieces ----

// y = M x for a CSR matrix (rows ascending; the sums in column order, deterministic)
// y = A x (ACC: y += A x) for a CSR matrix, G lanes per row: the lanes of a group stride
// over the row's entries (coalesced reads of col and val), then a butterfly inside the
// group adds their partial sums in a fixed order
template <int G, bool ACC, typename TX>
__global__ __launch_bounds__(256) void k_csr(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                             const double* __restrict__ val, const TX* __restrict__ x,
                                             double* __restrict__ y, int64_t nrows) {
  const int lane = int(threadIdx.x) % G;
  const int64_t stride = int64_t(gridDim.x) * (256 / G);
  // the loop bound is the same for all lanes of a group, so the shuffles see the
  // whole group active
  for (int64_t row = (int64_t(blockIdx.x) * 256 + threadIdx.x) / G; row < nrows; row += stride) {
    double s = 0.0;
    const int64_t e = rowptr[row + 1];
    for (int64_t j = rowptr[row] + lane; j < e; j += G) s = fma(val[j], double(x[col[j]]), s);
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    if (lane == 0) y[row] = ACC ? y[row] + s : s;
  }
}

// x[idx[i]] = sum_j M[i][j] b[idx[j]] for a dense m x m matrix M (row-major), one block per
// row, the products summed in a fixed order
__global__ __launch_bounds__(256) void k_dense_solve(const double* __restrict__ M, const int32_t* __restrict__ idx,
                                                     int64_t m, const double* __restrict__ b, double* __restrict__ x) {
  __shared__ double red[4];
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += blockDim.x) s = fma(M[i * m + j], b[idx[j]], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) x[idx[i]] = (red[0] + red[1]) + (red[2] + red[3]);
}

// flexible CG scalars kept on the device: s[0] r.z, s[1] p.Ap, s[2] alpha, s[3] r.r,
// s[4] r.z (new z), s[5] r.z (previous z), s[6] beta, s[7] flag (1 breakdown, 2 non-finite)
__global__ void k_fcg_alpha(double* s) {
  const double rz = s[0], pq = s[1];
  const bool finite = isfinite(rz) && isfinite(pq);
  const bool ok = finite && pq > 0.0;
  s[2] = ok ? rz / pq : 0.0;
  if (!ok) s[7] = finite ? 1.0 : 2.0;
}
// flexible CG: beta = -(z_{k+1} . A p_k) / (p_k . A p_k) (s5, s1; s1 > 0 was checked by
// k_fcg_alpha), and r.z of the new iterate (s4) becomes the next numerator of alpha; a
// non-finite s4 or s5, or r.z <= 0 (the preconditioner is not positive there), is flagged
__global__ void k_fcg_beta(double* s) {
  const double rz = s[4], zq = s[5];
  const bool finite = isfinite(rz) && isfinite(zq);
  const bool ok = finite && rz > 0.0;
  s[6] = ok ? -zq / s[1] : 0.0;
  s[0] = rz;
  if (!ok) s[7] = finite ? 1.0 : 2.0;
}
// y += sign s[k] x (the fma of y = a x + y)
__global__ __launch_bounds__(256) void k_axpy_s(double* y, const double* __restrict__ x, const double* __restrict__ s,
                                                int k, double sign, int64_t n) {
  const double a = sign * s[k];
  GRID_STRIDE(i, n) y[i] = fma(a, x[i], y[i]);
}
// p = z + s[k] p (the fma of p = 1 z + beta p)
__global__ __launch_bounds__(256) void k_xpby_s(double* p, const double* __restrict__ z, const double* __restrict__ s,
                                                int k, int64_t n) {
  const double beta = s[k];
  GRID_STRIDE(i, n) p[i] = fma(1.0, z[i], beta * p[i]);
}

// x[idx[i]] = b[idx[i]]
__global__ __launch_bounds__(256) void k_copy_indexed(double* __restrict__ x, const double* __restrict__ b,
                                                      const int32_t* __restrict__ idx, int64_t n) {
  GRID_STRIDE(i, n) x[idx[i]] = b[idx[i]];
}

// d = s D^-1 r
__global__ __launch_bounds__(256) void k_cheb_init(const double* __restrict__ r, const double* __restrict__ invd,
                                                   double* __restrict__ d, double s, int64_t n) {
  GRID_STRIDE(i, n) d[i] = s * invd[i] * r[i];
}

// one Chebyshev step after t = A d: x += d, r -= t, d = c1 d + c2 D^-1 r
template <bool S>
__global__ __launch_bounds__(256) void k_cheb_step(double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ d, const double* __restrict__ t,
                                                   const double* __restrict__ invd, double c1, double c2, int64_t n) {
  GRID_STRIDE(i, n) {
    const double di = d[i];
    update_iterate<S>(x, i, 1.0, di);
    const double ri = r[i] - t[i];
    r[i] = ri;
    d[i] = fma(c1, di, c2 * invd[i] * ri);
  }
}

// y = a x + b y
__global__ __launch_bounds__(256) void k_axpby(double a, const double* x, double b, double* y,
                                               int64_t n) {
  GRID_STRIDE(i, n) y[i] = fma(a, x[i], b * y[i]);
}

// r = b - t
__global__ __launch_bounds__(256) void k_sub(const double* __restrict__ b, const double* __restrict__ t,
                                             double* __restrict__ r, int64_t n) {
  GRID_STRIDE(i, n) r[i] = b[i] - t[i];
}
// k_csr for a matrix whose values are a few exact constants: each entry is one 32-bit word,
// the column in the low 24 bits and the index of its value in a 256-entry table in the high
// 8 (4 bytes per entry instead of 12).  The table sits in LDS.  Two entries per lane are
// loaded before either is used; each lane still adds its entries in ascending order, so the
// result is bit for bit that of k_csr on the unpacked matrix.
template <int G, bool ACC, typename TX>
__global__ __launch_bounds__(256) void k_csr_pk(const int64_t* __restrict__ rowptr, const uint32_t* __restrict__ ent,
                                                const double* __restrict__ tab, const TX* __restrict__ x,
                                                double* __restrict__ y, int64_t nrows) {
  __shared__ double t[256];
  t[threadIdx.x] = tab[threadIdx.x];
  __syncthreads();
  const int lane = int(threadIdx.x) % G;
  const int64_t stride = int64_t(gridDim.x) * (256 / G);
  for (int64_t row = (int64_t(blockIdx.x) * 256 + threadIdx.x) / G; row < nrows; row += stride) {
    double s = 0.0;
    const int64_t e = rowptr[row + 1];
    int64_t j = rowptr[row] + lane;
    for (; j + G < e; j += 2 * G) {
      const uint32_t a = ent[j], b = ent[j + G];
      const double xa = double(x[a & 0xFFFFFFu]), xb = double(x[b & 0xFFFFFFu]);
      s = fma(t[a >> 24], xa, s);
      s = fma(t[b >> 24], xb, s);
    }
    if (j < e) {
      const uint32_t a = ent[j];
      s = fma(t[a >> 24], double(x[a & 0xFFFFFFu]), s);
    }
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    if (lane == 0) y[row] = ACC ? y[row] + s : s;
  }
}

// the same smoother steps with the residual and the search direction stored in FP32
// (the iterate x stays FP64; every operation is done in FP64 and rounded once on store)
__global__ __launch_bounds__(256) void k_sub_to32(const double* __restrict__ b, const double* __restrict__ t,
                                                  float* __restrict__ r, int64_t n) {
  GRID_STRIDE(i, n) r[i] = float(b[i] - t[i]);
}
__global__ __launch_bounds__(256) void k_cheb_init32(const float* __restrict__ r, const double* __restrict__ invd,
                                                     float* __restrict__ d, double s, int64_t n) {
  GRID_STRIDE(i, n) d[i] = float(s * invd[i] * double(r[i]));
}
template <bool S>
__global__ __launch_bounds__(256) void k_cheb_step32(double* __restrict__ x, float* __restrict__ r,
                                                     float* __restrict__ d, const float* __restrict__ t,
                                                     const double* __restrict__ invd, double c1, double c2,
                                                     int64_t n) {
  GRID_STRIDE(i, n) {
    const double di = double(d[i]);
    update_iterate<S>(x, i, 1.0, di);
    const double ri = double(r[i]) - double(t[i]);
    r[i] = float(ri);
    d[i] = float(fma(c1, di, c2 * invd[i] * ri));
  }
}

// deterministic start vector in [-1, 1): a multiplicative hash of the index
__global__ __launch_bounds__(256) void k_hash_fill(double* __restrict__ v, int64_t n) {
  GRID_STRIDE(i, n) {
    const uint32_t h = uint32_t(uint64_t(i) * 2654435761ull) ^ uint32_t(uint64_t(i) >> 16);
    v[i] = double(h) * (1.0 / 2147483648.0) - 1.0;
  }
}

// ---- the same iteration on FP32 vectors r, p, q (x stays FP64; arithmetic and inner
// products in FP64, each stored vector rounded once) ----

// r = b - y (y may be null), z = invd r; partials (r.z, r.r, b.b) of the stored values
__global__ __launch_bounds__(256) void k_pcg_init32(const double* __restrict__ b, const double* __restrict__ y,
                                                    const float* __restrict__ invd, float* __restrict__ r,
                                                    float* __restrict__ p, int64_t n, double* __restrict__ part) {
  double v[3] = {0.0, 0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double bi = b[i];
    const float ri = float(y ? bi - y[i] : bi);
    const double zi = double(invd[i]) * double(ri);
    r[i] = ri;
    p[i] = float(zi);
    v[0] += double(ri) * zi;
    v[1] += double(ri) * double(ri);
    v[2] += bi * bi;
  }
  block_partials(v, 3, part);
}

// x += alpha p, r -= alpha q, z = invd r; partials (r.z, r.r)
template <bool S>
__global__ __launch_bounds__(256) void k_pcg_xr32(double* __restrict__ x, float* __restrict__ r,
                                                  const float* __restrict__ p, const float* __restrict__ q,
                                                  const float* __restrict__ invd, const PcgScalars* __restrict__ s,
                                                  int64_t n, double* __restrict__ part) {
  const double alpha = s->alpha;
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    update_iterate<S>(x, i, alpha, double(p[i]));
    const float ri = float(fma(-alpha, double(q[i]), double(r[i])));
    r[i] = ri;
    v[0] += double(ri) * (double(invd[i]) * double(ri));
    v[1] += double(ri) * double(ri);
  }
  block_partials(v, 2, part);
}

// p = invd r + beta p
__global__ __launch_bounds__(256) void k_pcg_p32(float* __restrict__ p, const float* __restrict__ r,
                                                 const float* __restrict__ invd, const PcgScalars* __restrict__ s,
                                                 int64_t n) {
  const double beta = s->beta;
  GRID_STRIDE(i, n) p[i] = float(fma(beta, double(p[i]), double(invd[i]) * double(r[i])));
}

// residual replacement: r = b - y (y = A64 x): the true r.r from the unrounded FP64
// residual, r stored in FP32, r.z from the stored r; with p, restart p = z
__global__ __launch_bounds__(256) void k_replace32(const double* __restrict__ b, const double* __restrict__ y,
                                                   const float* __restrict__ invd, float* __restrict__ r,
                                                   float* __restrict__ p, int64_t n, double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double rd = b[i] - y[i];
    const float ri = float(rd);
    const double zi = double(invd[i]) * double(ri);
    r[i] = ri;
    if (p) p[i] = float(zi);
    v[0] += double(ri) * zi;
    v[1] += rd * rd;
  }
  block_partials(v, 2, part);
}

}  // namespace dev

static unsigned red_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > RED_BLOCKS) g = RED_BLOCKS;
  if (g < 1) g = 1;
  return unsigned(g);
}

// The reduction kernels always run with RED_BLOCKS blocks so the partial layout is fixed.
void vk_pcg_init(const double* b, const double* y, const double* invd, double* r, double* p, int64_t n, double* part,
                 PcgScalars* s, double* hist, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_pcg_init, dim3(RED_BLOCKS), dim3(256), 0, st, b, y, invd, r, p, n, part);
  hipLaunchKernelGGL(dev::k_fin_init, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, s, hist);
}
void vk_fin_pq(const double* energy, int64_t ntiles, PcgScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_fin_pq, dim3(1), dim3(1024), 0, st, energy, ntiles, s);
}
void vk_pcg_xr(double* x, double* r, const double* p, const double* q, const double* invd, const PcgScalars* s,
               int64_t n, double* part, bool stream, hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL(dev::k_pcg_xr<true>, dim3(RED_BLOCKS), dim3(256), 0, st, x, r, p, q, invd, s, n, part);
  else
    hipLaunchKernelGGL(dev::k_pcg_xr<false>, dim3(RED_BLOCKS), dim3(256), 0, st, x, r, p, q, invd, s, n, part);
}
void vk_fin_rz(const double* part, PcgScalars* s, double* hist, int it, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_fin_rz, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, s, hist, it);
}
void vk_pcg_p(double* p, const double* r, const double* invd, const PcgScalars* s, int64_t n, bool stream,
              hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL(dev::k_pcg_p<true>, dim3(red_grid(n) * 4), dim3(256), 0, st, p, r, invd, s, n);
  else
    hipLaunchKernelGGL(dev::k_pcg_p<false>, dim3(red_grid(n) * 4), dim3(256), 0, st, p, r, invd, s, n);
}
void vk_resid(const double* b, const double* y, double* r, int64_t n, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_resid, dim3(RED_BLOCKS), dim3(256), 0, st, b, y, r, n, part);
  hipLaunchKernelGGL(dev::k_fin_sum, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, out);
}
void vk_replace(const double* b, const double* y, const double* invd, double* r, double* p, int64_t n, double* part,
                PcgScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_replace, dim3(RED_BLOCKS), dim3(256), 0, st, b, y, invd, r, p, n, part);
  hipLaunchKernelGGL(dev::k_fin_replace, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, s);
}
void vk_dot(const double* a, const double* b, int64_t n, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_dot, dim3(RED_BLOCKS), dim3(256), 0, st, a, b, n, part);
  hipLaunchKernelGGL(dev::k_fin_sum, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, out);
}
void vk_axpy1(double* x, const double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_axpy1, dim3(red_grid(n) * 4), dim3(256), 0, st, x, d, n);
}
void vk_pcg_init32(const double* b, const double* y, const float* invd, float* r, float* p, int64_t n, double* part,
                   PcgScalars* s, double* hist, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_pcg_init32, dim3(RED_BLOCKS), dim3(256), 0, st, b, y, invd, r, p, n, part);
  hipLaunchKernelGGL(dev::k_fin_init, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, s, hist);
}

void vk_pcg_xr32(double* x, float* r, const float* p, const float* q, const float* invd, const PcgScalars* s,
                 int64_t n, double* part, bool stream, hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL(dev::k_pcg_xr32<true>, dim3(RED_BLOCKS), dim3(256), 0, st, x, r, p, q, invd, s, n, part);
  else
    hipLaunchKernelGGL(dev::k_pcg_xr32<false>, dim3(RED_BLOCKS), dim3(256), 0, st, x, r, p, q, invd, s, n, part);
}

void vk_pcg_p32(float* p, const float* r, const float* invd, const PcgScalars* s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_pcg_p32, dim3(red_grid(n) * 4), dim3(256), 0, st, p, r, invd, s, n);
}

void vk_replace32(const double* b, const double* y, const float* invd, float* r, float* p, int64_t n, double* part,
                  PcgScalars* s, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_replace32, dim3(RED_BLOCKS), dim3(256), 0, st, b, y, invd, r, p, n, part);
  hipLaunchKernelGGL(dev::k_fin_replace, dim3(1), dim3(1024), 0, st, part, RED_BLOCKS, s);
}

template <int G, typename TX>
static void csr_launch(const int64_t* rowptr, const int32_t* col, const double* val, const TX* x, double* y,
                       int64_t nrows, bool acc, hipStream_t st) {
  const int64_t g = std::min<int64_t>((nrows + 256 / G - 1) / (256 / G), 16384);
  if (acc)
    hipLaunchKernelGGL((dev::k_csr<G, true, TX>), dim3(unsigned(g)), dim3(256), 0, st, rowptr, col, val, x, y, nrows);
  else
    hipLaunchKernelGGL((dev::k_csr<G, false, TX>), dim3(unsigned(g)), dim3(256), 0, st, rowptr, col, val, x, y, nrows);
}

template <typename TX>
static void csr_any(const int64_t* rowptr, const int32_t* col, const double* val, const TX* x, double* y,
                    int64_t nrows, int64_t nnz, bool accumulate, hipStream_t st) {
  if (nrows <= 0) return;
  const double mean = double(nnz) / double(nrows);
  if (mean <= 3.0)
    csr_launch<2>(rowptr, col, val, x, y, nrows, accumulate, st);
  else if (mean <= 6.0)
    csr_launch<4>(rowptr, col, val, x, y, nrows, accumulate, st);
  else if (mean <= 24.0)
    csr_launch<8>(rowptr, col, val, x, y, nrows, accumulate, st);
  else
    csr_launch<16>(rowptr, col, val, x, y, nrows, accumulate, st);
}

template <int G, typename TX>
static void csr_pk_launch(const int64_t* rowptr, const uint32_t* ent, const double* tab, const TX* x, double* y,
                          int64_t nrows, bool acc, hipStream_t st) {
  const int64_t g = std::min<int64_t>((nrows + 256 / G - 1) / (256 / G), 16384);
  if (acc)
    hipLaunchKernelGGL((dev::k_csr_pk<G, true, TX>), dim3(unsigned(g)), dim3(256), 0, st, rowptr, ent, tab, x, y,
                       nrows);
  else
    hipLaunchKernelGGL((dev::k_csr_pk<G, false, TX>), dim3(unsigned(g)), dim3(256), 0, st, rowptr, ent, tab, x, y,
                       nrows);
}

template <typename TX>
static void csr_pk_any(const int64_t* rowptr, const uint32_t* ent, const double* tab, const TX* x, double* y,
                       int64_t nrows, int64_t nnz, bool accumulate, hipStream_t st) {
  if (nrows <= 0) return;
  const double mean = double(nnz) / double(nrows);
  if (mean <= 3.0)
    csr_pk_launch<2>(rowptr, ent, tab, x, y, nrows, accumulate, st);
  else if (mean <= 6.0)
    csr_pk_launch<4>(rowptr, ent, tab, x, y, nrows, accumulate, st);
  else if (mean <= 24.0)
    csr_pk_launch<8>(rowptr, ent, tab, x, y, nrows, accumulate, st);
  else
    csr_pk_launch<16>(rowptr, ent, tab, x, y, nrows, accumulate, st);
}

void vk_csr_pk(const int64_t* rowptr, const uint32_t* ent, const double* tab, const double* x, double* y,
               int64_t nrows, int64_t nnz, bool accumulate, hipStream_t st) {
  csr_pk_any(rowptr, ent, tab, x, y, nrows, nnz, accumulate, st);
}
void vk_csr_pk_x32(const int64_t* rowptr, const uint32_t* ent, const double* tab, const float* x, double* y,
                   int64_t nrows, int64_t nnz, hipStream_t st) {
  csr_pk_any(rowptr, ent, tab, x, y, nrows, nnz, false, st);
}

void vk_csr_x32(const int64_t* rowptr, const int32_t* col, const double* val, const float* x, double* y,
                int64_t nrows, int64_t nnz, hipStream_t st) {
  csr_any(rowptr, col, val, x, y, nrows, nnz, false, st);
}

void vk_csr(const int64_t* rowptr, const int32_t* col, const double* val, const double* x, double* y, int64_t nrows,
            int64_t nnz, bool accumulate, hipStream_t st) {
  csr_any(rowptr, col, val, x, y, nrows, nnz, accumulate, st);
}

void vk_cheb_init(const double* r, const double* invd, double* d, double s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_cheb_init, dim3(red_grid(n) * 4), dim3(256), 0, st, r, invd, d, s, n);
}
void vk_cheb_step(double* x, double* r, double* d, const double* t, const double* invd, double c1, double c2, int64_t n,
                  bool stream, hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL(dev::k_cheb_step<true>, dim3(red_grid(n) * 4), dim3(256), 0, st, x, r, d, t, invd, c1, c2, n);
  else
    hipLaunchKernelGGL(dev::k_cheb_step<false>, dim3(red_grid(n) * 4), dim3(256), 0, st, x, r, d, t, invd, c1, c2, n);
}
void vk_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_axpby, dim3(red_grid(n) * 4), dim3(256), 0, st, a, x, b, y, n);
}
void vk_sub(const double* b, const double* t, double* r, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_sub, dim3(red_grid(n) * 4), dim3(256), 0, st, b, t, r, n);
}
void vk_sub_to32(const double* b, const double* t, float* r, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_sub_to32, dim3(red_grid(n) * 4), dim3(256), 0, st, b, t, r, n);
}
void vk_cheb_init32(const float* r, const double* invd, float* d, double s, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_cheb_init32, dim3(red_grid(n) * 4), dim3(256), 0, st, r, invd, d, s, n);
}
void vk_cheb_step32(double* x, float* r, float* d, const float* t, const double* invd, double c1, double c2,
                    int64_t n, bool stream, hipStream_t st) {
  if (stream)
    hipLaunchKernelGGL(dev::k_cheb_step32<true>, dim3(red_grid(n) * 4), dim3(256), 0, st, x, r, d, t, invd, c1, c2, n);
  else
    hipLaunchKernelGGL(dev::k_cheb_step32<false>, dim3(red_grid(n) * 4), dim3(256), 0, st, x, r, d, t, invd, c1, c2,
                       n);
}
void vk_dense_solve(const double* M, const int32_t* idx, int64_t m, const double* b, double* x, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(dev::k_dense_solve, dim3(unsigned(m)), dim3(256), 0, st, M, idx, m, b, x);
}
void vk_fcg_alpha(double* s, hipStream_t st) { hipLaunchKernelGGL(dev::k_fcg_alpha, dim3(1), dim3(1), 0, st, s); }
void vk_fcg_beta(double* s, hipStream_t st) { hipLaunchKernelGGL(dev::k_fcg_beta, dim3(1), dim3(1), 0, st, s); }
void vk_axpy_s(double* y, const double* x, const double* s, int k, double sign, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_axpy_s, dim3(red_grid(n) * 4), dim3(256), 0, st, y, x, s, k, sign, n);
}
void vk_xpby_s(double* p, const double* z, const double* s, int k, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_xpby_s, dim3(red_grid(n) * 4), dim3(256), 0, st, p, z, s, k, n);
}
void vk_copy_indexed(double* x, const double* b, const int32_t* idx, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_copy_indexed, dim3(red_grid(n)), dim3(256), 0, st, x, b, idx, n);
}
void vk_hash_fill(double* v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_hash_fill, dim3(red_grid(n) * 4), dim3(256), 0, st, v, n);
}

void vk_fill(double* x, double v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_fill, dim3(red_grid(n) * 4), dim3(256), 0, st, x, v, n);
}

}  // namespace dogip
