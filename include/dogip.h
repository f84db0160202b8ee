/*
 * libdogip: element-wise DoGIP operator (double-grid quadrature with
 * interpolation-projection) on simplex meshes, for AMD Instinct MI355X (gfx950).
 *
 * The library discretises the two variational problems of the paper
 *   - weighted projection (Definition in Section 2.2, eq. bilf_gp):
 *       a(u, v) = int_Omega m u v,
 *   - scalar elliptic problem (Definition in Section 2.3, eq. bilf_se):
 *       a(u, v) = int_Omega M grad u . grad v,
 * on the continuous Lagrange space V = C_{N,k} (Section 2.1), and applies the
 * Galerkin matrix A (eq. linsys_gp / eq. linsys_se) in the factored form of
 * Theorems 2 and 4 without assembling it:
 *       A u = sum_T P_T^T  B^^T  D_T  B^  P_T u          (Algorithm 1)
 * with B^ the interpolation (projection: values, elliptic: reference gradients)
 * of the V basis at the nodes of the double-grid space W (C_{N,2k} for the
 * projection, D_{N,2k-2} for the elliptic problem), and D_T the (block-)
 * diagonal of coefficient integrals over the W basis.
 *
 * Conventions
 *   - Every function returns a status code; DOGIP_OK is 0.  No exception or
 *     abort crosses this interface.  dogip_last_error() gives a message for the
 *     last failing call of the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory of the current device (for instance torch tensors on cuda:0).  The
 *     caller owns every pointer it passes and keeps it valid for the duration of
 *     the call; asynchronous calls (marked async) read and write device memory
 *     in stream order, so the memory must stay valid until the stream reaches
 *     the call.
 *   - Streams are hipStream_t values passed as void*; NULL is the null stream.
 *   - Handles are opaque; destroy functions accept NULL.  A space keeps its
 *     mesh alive and an operator keeps its space alive, so handles may be
 *     destroyed in any order.
 *   - Dofs (Lagrange nodes of C_{N,k}) are numbered along the Morton (Z-order)
 *     curve of their coordinates in the mesh bounding box, ties in the order
 *     vertices, edge nodes, face nodes, cell nodes; dogip_space_dof_coords and
 *     dogip_space_cell_dofs expose the numbering.  Local nodes of a cell follow
 *     the lattice a/k, |a| <= k, in lexicographic order of (a_1, .., a_d) on the
 *     reference simplex conv{0, e_1, .., e_d}, vertex j of the cell mapped to
 *     the reference vertex j (0 -> origin).
 *   - Symmetric d x d tensors are packed as the upper triangle row by row:
 *     2D (00, 01, 11), 3D (00, 01, 02, 11, 12, 22).
 *   - Threads: calls on different operators (or batches) may run concurrently
 *     from different host threads, each on its own stream; every operator owns
 *     its work buffers.  Calls on one operator must not overlap.
 */
#ifndef DOGIP_H
#define DOGIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define DOGIP_OK 0
#define DOGIP_E_INVALID 1       /* malformed input: shape, index, degenerate cell */
#define DOGIP_E_RANGE 2         /* order, kind or parameter outside the supported range */
#define DOGIP_E_NULL 3          /* NULL handle or pointer where one is required */
#define DOGIP_E_HIP 4           /* HIP runtime failure */
#define DOGIP_E_NOMEM 5         /* host or device allocation failed */
#define DOGIP_E_NOT_CONVERGED 6 /* iteration limit reached; stats are filled */
#define DOGIP_E_BREAKDOWN 7     /* CG found p^T A p <= 0 (operator not SPD) */
#define DOGIP_E_NONFINITE 8     /* NaN or Inf in a residual or inner product */
#define DOGIP_E_STATE 9         /* operation needs data the handle does not hold */

/* ---- problem kinds (Sections 2.2 and 2.3) ---- */
#define DOGIP_WP 0 /* weighted projection, W = C_{N,2k}, D_T = diag(int_T m phi^W_i) */
#define DOGIP_SE 1 /* elliptic problem, W = D_{N,2k-2}, D_T = R_T^-1 (int_T M phi^W_i) R_T^-T */

/* ---- boundary conditions ---- */
#define DOGIP_BC_NONE 0       /* natural (Neumann) boundary */
#define DOGIP_BC_DIRICHLET0 1 /* zero Dirichlet on all of the boundary: identity rows and columns */

/* ---- coefficient forms for dogip_op_create / dogip_op_set_coef ---- */
#define DOGIP_COEF_SCALAR 0    /* [ncells]: m_T (projection) or a_T with M = a_T I (elliptic, Corollary) */
#define DOGIP_COEF_SYM 1       /* [ncells][d(d+1)/2]: symmetric M_T, packed (elliptic only) */
#define DOGIP_COEF_LOGSCALAR 2 /* [ncells]: theta_T, coefficient exp(theta_T) */
#define DOGIP_COEF_RAW_D 3     /* [ncells][W_T][s]: D itself, s = 1 (projection) or d(d+1)/2 (elliptic) */

/* ---- arithmetic precision of an apply ---- */
#define DOGIP_F64 0 /* FP64 D, FP64 element arithmetic */
#define DOGIP_F32 1 /* FP32 copy of D, FP32 element arithmetic and tile accumulation;
                       vectors stay FP64 */

/* ---- solve modes ---- */
#define DOGIP_SOLVE_F64 0 /* Jacobi-PCG with the FP64 apply */
/* Jacobi-PCG with the FP32 apply, refined in FP64 by residual replacement: the
 * recursive residual is replaced by b - A64 x (FP64 apply) each time it has
 * dropped by the factor inner_tol (default 0.1), at least every 512 iterations and
 * at apparent convergence (where the direction restarts; elsewhere it is kept).
 * x and the inner products are FP64; the residual, direction and A p are stored in
 * FP32 (element-wise operators; FP64 for the global and quadrature-point forms).
 * When the true residual stays well above the recursive one or diverges, the solve
 * finishes with FP64 CG. */
#define DOGIP_SOLVE_MIXED 1
/* FP64 iterative refinement that restarts an FP32-apply Jacobi-PCG for every
 * correction, each inner solve reducing its residual by inner_tol. */
#define DOGIP_SOLVE_MIXED_RESTART 2
/* Flexible CG preconditioned by a p-multigrid V-cycle (multigrid that fits the DoGIP
 * structure, which Section 4 leaves to future work): the orders k, k-1, ..., 1 on the
 * same mesh, each a DoGIP operator rebuilt from the operator's coefficient; the
 * prolongation embeds P_{j-1} in P_j (nodal values), the restriction is its transpose;
 * Chebyshev smoothing in D^-1 A (degree 3 on [lmax/8, 1.1 lmax], lmax by power
 * iteration) before and after the coarse correction.  Each order level's D is rebuilt
 * from the operator's coefficient, or by the same sub-cell quadrature for inclusions.
 * For the elliptic problem on a mesh from dogip_mesh_unit with n even, the hierarchy
 * continues below P_1 with P_1 on the nested unit meshes n/2, n/4, ... until the
 * coarsest has at most 400 interior dofs: a coarse cell's coefficient is the mean over
 * its 2^d children (of the logarithm for LOGSCALAR), or for inclusions the geometric
 * mean of the inclusion coefficient over a lattice of points of the coarse cell; P_1
 * interpolation between the meshes; Chebyshev degree 4 on [lmax/20, 1.1 lmax] there.  A
 * coarsest level with at most 1000 interior dofs is solved exactly (its dense inverse,
 * formed at set-up); a larger one by Jacobi-PCG to a relative residual of 0.1 (or
 * inner_tol, when in (0, 1)).  That inner solve varies the preconditioner, so the outer
 * CG is the flexible one: beta = -(z_{k+1} . A p_k) / (p_k . A p_k).  The hierarchy is
 * built at the first such solve; after a coefficient change the next one rebuilds only
 * the levels' D, diagonals, lmax and the coarse inverse.
 * Needs an element-wise operator whose D came from a SCALAR, SYM or LOGSCALAR
 * coefficient or from dogip_op_set_inclusions, else DOGIP_E_STATE.  iters counts outer
 * iterations; convergence is verified on the true FP64 residual; DOGIP_E_BREAKDOWN if
 * p.Ap or r.z (the preconditioned residual) is not positive. */
#define DOGIP_SOLVE_PMG 3
/* The same with the V-cycle's applies (smoothing, coarse solve) in FP32; the outer CG
 * and its residuals stay FP64.  Needs DOGIP_OP_FP32. */
#define DOGIP_SOLVE_PMG_MIXED 4
/* As DOGIP_SOLVE_MIXED (FP32 apply, FP64 residual replacement) with the residual,
 * direction and A p stored in FP64: only the apply (D, element arithmetic) is FP32;
 * x, r, every inner product and D's construction stay FP64.  Element-wise, global and
 * quadrature-point operators alike.  Needs DOGIP_OP_FP32. */
#define DOGIP_SOLVE_MIXED_V64 5

/* ---- dogip_op_create flags ---- */
#define DOGIP_OP_FP32 1u /* also build the FP32 copy of D (needed by DOGIP_F32 and MIXED) */
/* Global form of the weighted projection (Theorem 1): A = B^T A^DoGIP B with one D
 * value per dof of the continuous double-grid space C_{N,2k} (the element-wise
 * form of Theorem 2 stores one per cell and node).  Projection spaces only. */
#define DOGIP_OP_GLOBAL_W 2u

/* ---- element kernel variants ---- */
#define DOGIP_VARIANT_AUTO 0     /* tuned choice: unrolled where compiled, else looped */
#define DOGIP_VARIANT_UNROLLED 1 /* B^ as compile-time constants, zero entries skipped, +-1 free */
#define DOGIP_VARIANT_LOOPED 2   /* B^ read from device memory (wave-uniform loads), dense */
/* 3D P3 elliptic only: FP64 applies as UNROLLED; FP32 applies form the two B^ products
 * (eq. ep_dogip_mul) with bfloat16 matrix-core instructions.  B^ of 3D P3 is exact in
 * bfloat16 and the vector operand (u_T, then D_T B^ u_T) is split into three bfloat16
 * terms whose sum is the FP32 value exactly, so every product is exact and only the FP32
 * accumulation rounds, as in the vector kernel.  The FP32 copy of D is held in this
 * variant's own layout.  Not accepted by dogip_batch_create. */
#define DOGIP_VARIANT_MFMA 3
/* Elliptic problem, k >= 2 (2D k <= 5, 3D k <= 3): B^ applied in factored form
 * (Section 4's cheaper interpolation-projection operator): grad u_T in P_{k-1} is formed
 * at the P_{k-1} lattice nodes (B1), then interpolated to the W nodes (B2, exact since W
 * holds degree 2k-2 >= k-1), and the transpose likewise; B^ = (I_d x B2) B1 exactly, with
 * 534 instead of 1014 multiply-adds per product at 3D P3.  Same D, same layout. */
#define DOGIP_VARIANT_FACTORED 4

typedef struct dogip_mesh_s* dogip_mesh;
typedef struct dogip_space_s* dogip_space;
typedef struct dogip_op_s* dogip_op;
typedef struct dogip_batch_s* dogip_batch;
typedef void* dogip_stream; /* hipStream_t */

typedef struct {
  int32_t dim, k, kind, bc;
  int64_t ncells, ndofs, nboundary;
  int32_t vt;   /* V_T = dim P_k */
  int32_t wt;   /* W_T = dim P_q, q = 2k (projection) or 2k-2 (elliptic) */
  int32_t nsym; /* D values per W node: 1 or d(d+1)/2 */
  int32_t nb;   /* leading extent of B^: 1 (projection) or d (elliptic) */
  int64_t nnz_bhat, nnz_pm1_bhat; /* nonzero and +-1 entries of B^ (Section 3 counts) */
} dogip_space_info;

typedef struct {
  int32_t tile_cells;  /* cells per tile (one workgroup) */
  int32_t variant;     /* DOGIP_VARIANT_UNROLLED or _LOOPED actually used */
  int32_t has_fp32;
  int32_t nq;          /* quadrature-point operator: points per cell; 0 for DoGIP */
  int64_t ntiles, tile_dofs_total, nshared, max_tile_dofs;
  int64_t bytes_d64, bytes_d32, bytes_index; /* device bytes held */
  double alg_bytes_f64; /* algorithmic bytes of one apply: D + int32 connectivity + u + y */
  double alg_bytes_f32;
  double alg_flops;     /* 2 [2 (nnz B^ - nnz_pm1 B^) + d^2 W_T] ncells (Section 3 count, x2 for FMA) */
  int64_t ndofs_w;      /* DOGIP_OP_GLOBAL_W: dofs of C_{N,2k} (D values held); 0 otherwise */
  int64_t stage_entries; /* partial sums an apply stages for dofs shared by tiles (doubles) */
} dogip_op_info;

typedef struct {
  double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2 */
  int32_t maxit;       /* CG iteration cap (all inner iterations in mixed mode) */
  int32_t mode;        /* one of the DOGIP_SOLVE_* modes above */
  double inner_tol;    /* MIXED: replacement factor delta; MIXED_RESTART: reduction per inner solve;
                          PMG modes: the coarsest level's relative residual */
  int32_t max_outer;   /* mixed: refinement steps cap */
  int32_t check_every; /* CG iterations between host-side convergence checks (>= 1) */
  int32_t x0_given;    /* nonzero: x holds the initial guess; else x0 = 0 */
  int32_t pad0;
} dogip_solve_opts;

typedef struct {
  int32_t status;   /* same as the return code */
  int32_t iters;    /* CG iterations (inner iterations summed in mixed mode) */
  int32_t outer;    /* refinement steps (mixed), 1 for FP64 */
  int32_t pad0;
  double relres;      /* residual norm ratio tracked by the solver at exit */
  double relres_true; /* ||b - A x|| / ||b|| recomputed with the FP64 apply at exit */
  double seconds;     /* wall time of the call (host clock, after a final synchronize) */
} dogip_solve_stats;

/* Message for the last failing call on this thread ("" if none). */
const char* dogip_last_error(void);
/* Library interface version (increments on ABI changes). */
int dogip_version(void);
/* Number of visible HIP devices; 0 without a GPU (never fails). */
int dogip_device_count(void);
/* Diagnostic, host only: compares the compile-time B^ tables used by the
 * unrolled kernels with the run-time exact tables; *mismatches = entries that
 * differ (0 expected). */
int dogip_check_tables(int64_t* mismatches);

/* ---- mesh (Section 2.1: simplices with affine maps F_T(x^) = R_T x^ + S_T) ---- */

/* Copy a simplex mesh.  xyz: host [nv][dim] vertex coordinates.  cells: host
 * [nc][dim+1] vertex ids.  dim is 2 or 3.  Fails with DOGIP_E_INVALID on an
 * out-of-range vertex id, a vertex used by no cell, or a cell with
 * |det R_T| <= 1e-14 * (its longest edge)^dim. */
int dogip_mesh_create(int dim, int64_t nv, const double* xyz, int64_t nc, const int32_t* cells,
                      dogip_mesh* out);
/* The structured mesh family of Section 3: unit square with n x n squares of two
 * triangles (v00, v10, v11), (v00, v11, v01), or unit cube with n^3 cubes of six
 * Kuhn tetrahedra (v000 -> +e_p0 -> +e_p1 -> +e_p2 for each axis permutation p).
 * Vertex (i, j[, l]) has id i + (n+1)(j + (n+1) l). */
int dogip_mesh_unit(int dim, int n, dogip_mesh* out);
int dogip_mesh_info(dogip_mesh m, int* dim, int64_t* nv, int64_t* nc);
/* Copy coordinates ([nv][dim]) and cells ([nc][dim+1]) to host arrays (either may be NULL). */
int dogip_mesh_copy(dogip_mesh m, double* xyz, int32_t* cells);
void dogip_mesh_destroy(dogip_mesh m);

/* ---- space: V = C_{N,k} with the double-grid space of the chosen kind ---- */

/* k: 1..8 in 2D, 1..4 in 3D (the range of Tables 1-4).  kind: DOGIP_WP or
 * DOGIP_SE.  bc: DOGIP_BC_NONE or DOGIP_BC_DIRICHLET0.  Builds the dof map l_T,
 * the boundary dofs and B^, w^ on the host. */
int dogip_space_create(dogip_mesh m, int k, int kind, int bc, dogip_space* out);
int dogip_space_get_info(dogip_space s, dogip_space_info* info);
/* host [ndofs][dim] coordinates of the dofs. */
int dogip_space_dof_coords(dogip_space s, double* xyz);
/* host [ncells][vt] global dof of every local node. */
int dogip_space_cell_dofs(dogip_space s, int32_t* cell_dofs);
/* host [nboundary] boundary dofs (on facets owned by one cell), ascending. */
int dogip_space_boundary(dogip_space s, int32_t* bnd);
/* host copies of B^ ([nb][wt][vt], Theorems 2/4) and of w^ ([wt], w^_i =
 * int_T^ phi^W_i / |T^|); either pointer may be NULL. */
int dogip_space_bhat(dogip_space s, double* bhat, double* what);
/* host copies of the factors of the elliptic B^ that DOGIP_VARIANT_FACTORED applies:
 * b1 [dim][n1][vt], the gradient of the P_k basis at the n1 = dim P_{k-1} lattice nodes,
 * and b2 [wt][n1], the P_{k-1} basis at the W nodes (B^_r = b2 b1_r); either pointer may
 * be NULL.  DOGIP_E_RANGE where the variant does not exist (projection, k = 1, 3D k = 4). */
int dogip_space_bhat_factors(dogip_space s, double* b1, double* b2);
void dogip_space_destroy(dogip_space s);

/* ---- operator: D in device memory, tiles, Jacobi diagonal ---- */

/* Build the operator.  coef: device pointer in the form coef_kind (cells in mesh
 * order), read during the call only.  flags: DOGIP_OP_FP32, DOGIP_OP_GLOBAL_W or
 * both.  tile_waves: cells per tile / 64, 1..48 (1..8 for the matrix-core variant),
 * or 0 for the built-in default (24 for element-wise 3D operators with k >= 2, 8 for
 * the matrix-core variant and the global form there, else 4), stepped down while a
 * tile's LDS arrays (16 bytes per tile dof) exceed 159 KB (64 KB for the matrix-core
 * variant).  A tile's cells are taken by one workgroup in passes of as many cells as
 * it has lanes (see dogip_op_set_tile_lanes).  variant:
 * DOGIP_VARIANT_*.  D is built by the HIP kernels (Theorem 2: m_T |T| w^_i;
 * Theorem 4: w^_i |T| R_T^-1 M_T R_T^-T; or copied for RAW_D).  The call
 * synchronizes the stream before returning.  DOGIP_E_RANGE for a form that does
 * not fit the kind (SYM with the projection) and for DOGIP_OP_GLOBAL_W on an
 * elliptic space.  With DOGIP_OP_GLOBAL_W, D_j = int m phi^W_j is summed over the
 * cells holding W dof j (RAW_D: the cells' [ncells][wt] values are summed). */
int dogip_op_create(dogip_space s, int coef_kind, const double* coef, unsigned flags, int tile_waves,
                    int variant, dogip_stream stream, dogip_op* out);
/* Coefficient with jumps inside the cells, the case Sections 2 and 3.3 argue DoGIP
 * suits: a = a_in inside the union of nballs balls (host array [nballs][dim+1]:
 * center, radius > 0), a_out elsewhere, isotropic (M = a I, or m = a).  Rebuilds the
 * D of an element-wise operator (with its FP32 copy and the Jacobi diagonal) from
 * int_T a phi^W_i = a_out |T| w^_i + (a_in - a_out) int_T 1_B phi^W_i, the last
 * integral by sub-cell quadrature on the GPU: the reference cell is red-refined
 * (2D: 4 children; 3D: 8, the inner octahedron cut along its m02-m13 diagonal) where
 * a sub-simplex is cut by a ball boundary, down to `depth` levels (0..6).  A
 * sub-simplex with all vertices in one ball is inside; one whose bounding sphere
 * misses every ball is outside.  Inside sub-simplices and cut ones at the last level
 * take the collapsed Gauss rule of ng points per direction (1..8, see
 * dogip_quadrature) mapped onto them, the indicator evaluated at the points of cut
 * ones.  mean_points (optional host output): quadrature points evaluated per cell,
 * averaged.  The apply's cost does not change.  Synchronizes the stream.
 * DOGIP_E_STATE for a DOGIP_OP_GLOBAL_W or quadrature-point operator;
 * DOGIP_E_RANGE for double-grid orders above 8 (2D) or 6 (3D); DOGIP_E_INVALID unless
 * a_in and a_out are finite and positive (the elliptic form needs a positive
 * coefficient). */
int dogip_op_set_inclusions(dogip_op op, int nballs, const double* balls, double a_in, double a_out, int depth,
                            int ng, double* mean_points, dogip_stream stream);

/* ---- conventional quadrature-point operator (the comparison of Section 3.3) ----
 * The matrix-free evaluation over integration points that the paper sets against
 * DoGIP: per cell, the trial function's values (projection) or gradients (elliptic)
 * are interpolated to the quadrature points, multiplied by w_q |det R_T| a(x_q)
 * (elliptic: and R_T^-1 R_T^-T), and projected back.  Its cost grows with the number
 * of points, DoGIP's with W_T.
 *
 * dogip_quadrature: the reference rule, host output pts [n^dim][dim], wts [n^dim]:
 * the collapsed (Duffy) Gauss-Legendre rule with n points per direction, n = 1..16,
 * ordered with s outermost (x1 = s, x2 = t (1-s), x3 = v (1-s)(1-t)), exact for total
 * degree <= 2n - dim (so its weights sum to |T^| when 2n >= dim).
 * dogip_op_create_qp: coef is a device array [ncells][n^dim] (mesh cell order) of the
 * scalar coefficient at the mapped points x_q = X_0 + R_T xhat_q, read during the
 * call.  flags: DOGIP_OP_FP32 or 0.  tile_waves: as for dogip_op_create, 0 meaning 4
 * here.  The operator supports dogip_apply, dogip_diag,
 * dogip_pcg and the timer; dogip_op_set_coef, dogip_op_export_d and
 * dogip_grad_logcoef return DOGIP_E_STATE.  Orders: 2D k <= 5, 3D k <= 3
 * (projection) or 4 (elliptic), else DOGIP_E_RANGE.  Synchronizes the stream. */
int dogip_quadrature(int dim, int n, double* pts, double* wts);
int dogip_op_create_qp(dogip_space s, int n, const double* coef, unsigned flags, int tile_waves,
                       dogip_stream stream, dogip_op* out);

/* Rebuild D (and the FP32 copy and the Jacobi diagonal) from a new coefficient.  async. */
int dogip_op_set_coef(dogip_op op, int coef_kind, const double* coef, dogip_stream stream);
int dogip_op_get_info(dogip_op op, dogip_op_info* info);
/* Lanes of the workgroup that runs one tile of the FP64 (lanes64) and FP32 (lanes32)
 * applies, for tuning: a multiple of 64 dividing info.tile_cells, at most the kernel's
 * launch bound (512 FP64, 768 FP32 for the element-wise kernels), or 0 (the default) to
 * take, per kernel, the count that keeps the most waves resident per compute unit.  The
 * tile's cells are taken in ascending order in passes whatever the lanes, so results are
 * the same bit for bit.  DOGIP_E_RANGE for a count that does not divide the tile (checked
 * here) or exceeds the kernel's bound (checked at the next apply). */
int dogip_op_set_tile_lanes(dogip_op op, int lanes64, int lanes32);

/* Copy D to device memory [ncells][wt][nsym] in mesh cell order (FP64).  async.
 * DOGIP_E_STATE for a DOGIP_OP_GLOBAL_W operator (its D is not per cell). */
int dogip_op_export_d(dogip_op op, double* d_out, dogip_stream stream);

/* y <- A u (overwrite), with Dirichlet identity rows if the space has them.
 * u, y: device [ndofs] FP64, u != y.  prec: DOGIP_F64 or DOGIP_F32 (the latter
 * needs DOGIP_OP_FP32).  async; allocates nothing.  The result is bitwise
 * reproducible (no floating-point atomics outside a workgroup's own cells).
 * The operator owns a staging buffer used by every apply, diag, solve and
 * gradient call: calls on one operator must be ordered (one stream). */
int dogip_apply(dogip_op op, const double* u, double* y, int prec, dogip_stream stream);
/* For callers that cannot allocate device memory at the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dogip_apply with the
 * same kernels and the same result bit for bit, its staging buffer taken from a static
 * device array of DOGIP_NOALLOC_MAX_STAGE doubles (32 MiB) that each device holds until
 * the process ends, instead of the operator's own.  Calls no hipMalloc, hipFree or
 * allocating library routine, issues no memset, and does not record the kernel timer.
 * DOGIP_E_RANGE if the operator's info.stage_entries exceeds DOGIP_NOALLOC_MAX_STAGE.
 * Every call on a device shares that device's array: calls that overlap in time on one
 * device (other streams or host threads) race and must be ordered by the caller.
 * async. */
#define DOGIP_NOALLOC_MAX_STAGE (1 << 22)
int dogip_apply_noalloc(dogip_op op, const double* u, double* y, int prec, dogip_stream stream);
/* diag <- diagonal of A (1 on Dirichlet rows).  device [ndofs].  async.  Bitwise
 * reproducible like dogip_apply (fixed summation order; uses the staging buffer). */
int dogip_diag(dogip_op op, double* diag, dogip_stream stream);
/* Solve A x = b.  b, x: device [ndofs].  Returns DOGIP_OK, DOGIP_E_NOT_CONVERGED,
 * DOGIP_E_BREAKDOWN or DOGIP_E_NONFINITE; stats (may be NULL) are filled in all
 * four cases.  Synchronizes the stream.  Dirichlet rows of b must hold the
 * boundary values (zero for a homogeneous problem). */
int dogip_pcg(dogip_op op, const double* b, double* x, const dogip_solve_opts* opts,
              dogip_solve_stats* stats, dogip_stream stream);
/* g_T <- -(B^ lam_T) . D_T (B^ u_T) = -lam_T^T A_T u_T per cell (mesh order), with
 * boundary entries of u and lam taken as zero: the gradient of J with respect
 * to theta_T when D scales with exp(theta_T) and A lam = dJ/du.  u, lam: device
 * [ndofs]; g: device [ncells].  async. */
int dogip_grad_logcoef(dogip_op op, const double* u, const double* lam, double* g, dogip_stream stream);
/* (DOGIP_E_STATE for a DOGIP_OP_GLOBAL_W operator.) */
/* Kernel timer: when enabled, every apply records HIP events on the apply's
 * stream before its tile kernel, between the tile kernel and the shared-dof
 * finish kernel, and after the finish.  dogip_op_timer_read synchronizes on the
 * last event and returns the summed milliseconds of the tile kernels and of
 * the finish kernels and the number of applies recorded, then resets.  Any
 * output pointer may be NULL.  The events only time (created with
 * hipEventDisableSystemFence, so that recording them does not write back and
 * invalidate the caches inside the timed applies): waiting on them does not
 * make the applies' outputs visible to the host; synchronize the stream for
 * that. */
int dogip_op_timer_enable(dogip_op op, int enable);
int dogip_op_timer_read(dogip_op op, double* tile_ms_sum, double* finish_ms_sum, int64_t* count);
void dogip_op_destroy(dogip_op op);

/* ---- batch: many operators applied in one persistent launch ---- */

/* ops: host array of nops operators (each with DOGIP_OP_FP32 if FP32 applies
 * are wanted).  Vectors of the batch are the concatenation of the per-operator
 * vectors; offsets (host [nops+1]) are returned by dogip_batch_offsets.
 * The batch keeps its operators alive. */
int dogip_batch_create(const dogip_op* ops, int nops, dogip_stream stream, dogip_batch* out);
int dogip_batch_offsets(dogip_batch b, int64_t* offsets);
/* y <- blockdiag(A_1, .., A_n) u in one persistent kernel launch (work queue of
 * tiles, largest first).  async. */
int dogip_batch_apply(dogip_batch b, const double* u, double* y, int prec, dogip_stream stream);
/* Solve every system of the batch; each applies its own stopping test.  stats:
 * host [nops] (may be NULL).  Returns the worst status. */
int dogip_batch_pcg(dogip_batch b, const double* rhs, double* x, const dogip_solve_opts* opts,
                    dogip_solve_stats* stats, dogip_stream stream);
void dogip_batch_destroy(dogip_batch b);

#ifdef __cplusplus
}
#endif

#endif /* DOGIP_H */
