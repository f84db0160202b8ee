// Device-side state of the CG solver and the vector kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "internal.hpp"

namespace dogip {

constexpr int RED_BLOCKS = 1024;  // fixed reduction grid (deterministic partial sums)
constexpr int PCG_BREAKDOWN = 1;
constexpr int PCG_NONFINITE = 2;

// Hand-over rules of the FP32-operator CG at a residual replacement (ratios of squared
// norms): the true residual above GAP_RR times the recursive one counts as a stall
// (three in a row hand over to FP64); above DIVERGE_RR times its minimum so far the
// iteration is taken as diverging and handed over at once.
constexpr double GAP_RR = 10.0;
constexpr double DIVERGE_RR = 1e4;

struct PcgScalars {
  double rho;    // r . z
  double rr;     // r . r
  double bb;     // b . b
  double pq;     // p . A p
  double alpha, beta;
  int flags;
  int pad;
};

// Device workspace of the CG solver, owned by the operator.
struct PcgWork {
  int64_t n = 0;
  int maxit = 0;
  DevBuf r, p, q, part, energy, scal, hist, rout, dx, yout, nrm;
  DevBuf r32, p32, q32;  // FP32 vectors of the mixed iteration (allocated on first use)
  double* hhist = nullptr;  // pinned mirror of hist
  ~PcgWork() {
    if (hhist) (void)hipHostFree(hhist);
  }
};

// Vector kernels whose iteration touches more bytes than the memory-side cache holds
// (256 MB on MI355X) read and write the vectors that an iteration uses once (the iterate;
// with FP64 vectors also A p and the inverse diagonal) non-temporally, so that the cache
// keeps the operator's index arrays and the direction for the next apply; smaller ones
// keep every vector cached.  bytes_per_dof: the vectors' bytes per dof; index_bytes: the
// operator's index arrays.
inline bool stream_vectors(int64_t n, int bytes_per_dof, int64_t index_bytes) {
  return double(n) * bytes_per_dof + double(index_bytes) > 256.0 * 1024 * 1024;
}

void vk_pcg_init(const double* b, const double* y, const double* invd, double* r, double* p, int64_t n, double* part,
                 PcgScalars* s, double* hist, hipStream_t st);
void vk_fin_pq(const double* energy, int64_t ntiles, PcgScalars* s, hipStream_t st);
void vk_pcg_xr(double* x, double* r, const double* p, const double* q, const double* invd, const PcgScalars* s,
               int64_t n, double* part, bool stream, hipStream_t st);
void vk_fin_rz(const double* part, PcgScalars* s, double* hist, int it, hipStream_t st);
void vk_pcg_p(double* p, const double* r, const double* invd, const PcgScalars* s, int64_t n, bool stream,
              hipStream_t st);
void vk_resid(const double* b, const double* y, double* r, int64_t n, double* part, double* out, hipStream_t st);
// r = b - y, and when p is given also p = invd r (restart); rho and rr refreshed
void vk_replace(const double* b, const double* y, const double* invd, double* r, double* p, int64_t n, double* part,
                PcgScalars* s, hipStream_t st);
void vk_dot(const double* a, const double* b, int64_t n, double* part, double* out, hipStream_t st);
// Plain Jacobi-PCG from x = 0 to the recursive relative residual tol (at most maxit
// iterations, no replacement): the inner solve of the multigrid coarsest level.
// Returns the iterations run.
int cg_inner(Op& op, const double* b, double* x, double tol, int maxit, int prec, hipStream_t st);
void vk_axpy1(double* x, const double* d, int64_t n, hipStream_t st);
void vk_fill(double* x, double v, int64_t n, hipStream_t st);
// p-multigrid: CSR product, Chebyshev smoothing steps, axpby, difference, start vector
// y = A x (accumulate: y += A x); a group of lanes per row, the group size from the
// mean row length nnz / nrows; deterministic (fixed reduction order)
void vk_csr(const int64_t* rowptr, const int32_t* col, const double* val, const double* x, double* y, int64_t nrows,
            int64_t nnz, bool accumulate, hipStream_t st);
// y = A x for an FP32 x (FP64 products and sums)
void vk_csr_x32(const int64_t* rowptr, const int32_t* col, const double* val, const float* x, double* y,
                int64_t nrows, int64_t nnz, hipStream_t st);
// the same for a packed matrix: ent[j] = column | (value index << 24), tab[256] the values
// (the column below 2^24); bit for bit equal to vk_csr on the unpacked matrix
void vk_csr_pk(const int64_t* rowptr, const uint32_t* ent, const double* tab, const double* x, double* y,
               int64_t nrows, int64_t nnz, bool accumulate, hipStream_t st);
void vk_csr_pk_x32(const int64_t* rowptr, const uint32_t* ent, const double* tab, const float* x, double* y,
                   int64_t nrows, int64_t nnz, hipStream_t st);
void vk_cheb_init(const double* r, const double* invd, double* d, double s, int64_t n, hipStream_t st);
void vk_cheb_step(double* x, double* r, double* d, const double* t, const double* invd, double c1, double c2, int64_t n,
                  bool stream, hipStream_t st);
void vk_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t st);
void vk_sub(const double* b, const double* t, double* r, int64_t n, hipStream_t st);
// FP32-storage forms of the smoother steps: r = float(b - t); d = float(s D^-1 r);
// x += d, r -= t, d = c1 d + c2 D^-1 r (FP64 arithmetic, FP32 r, d, t)
void vk_sub_to32(const double* b, const double* t, float* r, int64_t n, hipStream_t st);
void vk_cheb_init32(const float* r, const double* invd, float* d, double s, int64_t n, hipStream_t st);
void vk_cheb_step32(double* x, float* r, float* d, const float* t, const double* invd, double c1, double c2,
                    int64_t n, bool stream, hipStream_t st);
void vk_hash_fill(double* v, int64_t n, hipStream_t st);
// flexible CG on device scalars s[8] (r.z, p.Ap, alpha, r.r, new r.z, old r.z, beta, flag):
// alpha = r.z / p.Ap (flag 1 if p.Ap <= 0, 2 if not finite); beta = (new - old) / r.z,
// r.z = new; y += sign s[k] x; p = z + s[k] p
void vk_fcg_alpha(double* s, hipStream_t st);
void vk_fcg_beta(double* s, hipStream_t st);
void vk_axpy_s(double* y, const double* x, const double* s, int k, double sign, int64_t n, hipStream_t st);
void vk_xpby_s(double* p, const double* z, const double* s, int k, int64_t n, hipStream_t st);
// x[idx[i]] = b[idx[i]] for i < n
void vk_copy_indexed(double* x, const double* b, const int32_t* idx, int64_t n, hipStream_t st);
// x[idx[i]] = sum_j M[i][j] b[idx[j]], M dense m x m row-major (other entries of x untouched)
void vk_dense_solve(const double* M, const int32_t* idx, int64_t m, const double* b, double* x, hipStream_t st);
// The iteration on FP32 vectors (x FP64): the counterparts of vk_pcg_init, vk_pcg_xr,
// vk_pcg_p and vk_replace; the inner products stay FP64.
void vk_pcg_init32(const double* b, const double* y, const float* invd, float* r, float* p, int64_t n, double* part,
                   PcgScalars* s, double* hist, hipStream_t st);
void vk_pcg_xr32(double* x, float* r, const float* p, const float* q, const float* invd, const PcgScalars* s,
                 int64_t n, double* part, bool stream, hipStream_t st);
void vk_pcg_p32(float* p, const float* r, const float* invd, const PcgScalars* s, int64_t n, hipStream_t st);
void vk_replace32(const double* b, const double* y, const float* invd, float* r, float* p, int64_t n, double* part,
                  PcgScalars* s, hipStream_t st);

}  // namespace dogip
