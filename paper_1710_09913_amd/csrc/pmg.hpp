// p-multigrid preconditioner: the spaces P_k, P_{k-1}, ..., P_1 on one mesh, their DoGIP
// operators rebuilt from the fine operator's coefficient, and the transfers between them.
#pragma once

#include <memory>
#include <vector>

#include "internal.hpp"

namespace dogip {

struct PmgLevel {
  Op* op = nullptr;            // level 0: the fine operator itself
  std::unique_ptr<Op> own;     // coarser levels
  std::shared_ptr<Space> space;
  // prolongation to the next finer level (this level's vector -> the finer one), and
  // restriction (its transpose), both CSR with rows in ascending order
  DevBuf prow, pcol, pval, rrow, rcol, rval;
  // packed form when the values are at most 256 distinct constants and both sizes are
  // below 2^24 (then pcol/pval/rcol/rval stay empty): column | (value index << 24)
  bool packed = false;
  DevBuf ppk, rpk, ptab;
  int64_t n = 0, nfine = 0, nnz = 0;
  double lmax = 0.0;           // largest eigenvalue of D^-1 A (power iteration)
  double range = 0.0;          // the smoother damps [lmax / range, 1.1 lmax]
  // geometric level (P1 on the halved unit mesh): the cell of this level holding each
  // cell of the finer mesh
  bool hlevel = false;
  std::vector<int32_t> parent;
  // coarsest level when small: the inverse of A on its interior dofs (dense, row-major)
  DevBuf dinv, didx;
  int64_t nint = 0;
  DevBuf x, b;                 // the level's correction and right-hand side (not on level 0,
                               // which works on the outer CG's vectors)
  DevBuf r, d, t;              // V-cycle work vectors
};

struct Pmg {
  std::vector<std::unique_ptr<PmgLevel>> lv;  // lv[0] finest
  DevBuf r, z, p, q;           // outer flexible CG vectors (fine)
  DevBuf dots;                 // device scalars of the inner products
  DevBuf fcg;                  // the outer CG's scalars (vk_fcg_alpha)
  DevBuf e32;                  // tile partials the FP32-vector apply writes (unused)
  double coarse_tol = 0.1;     // relative residual of the coarsest level's inner solve
  bool stale = false;          // the fine D changed: the levels' D and lmax are redone
};

// Flexible CG on the fine operator preconditioned by one p-multigrid V-cycle per
// iteration (Chebyshev-Jacobi smoothing, coarsest level by Jacobi-PCG); prec_inner:
// the apply used inside the V-cycle.
int op_pcg_pmg(Op& op, const double* b, double* x, const dogip_solve_opts& o, dogip_solve_stats& stats, int prec_inner,
               hipStream_t st);

}  // namespace dogip
