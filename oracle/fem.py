"""Standard FEM on simplices (oracle, test infrastructure).

Plain textbook FEM, independent of the double-grid machinery:

* Local-to-global map l_T (Section 2.1).  A Lagrange node of C_{N,k} on cell T
  with barycentric multi-index b (|b| = k) sits at sum_j (b_j / k) X_j.  Nodes of
  neighbouring cells coincide exactly when their sets {(vertex id, b_j) : b_j > 0}
  coincide, so that set is the node's global key; dofs are numbered by the
  sorted order of the keys.
* Affine map F_T(x^) = R_T x^ + S_T with R_T = [X_1 - X_0, ..., X_d - X_0]
  (Section 2.1); gradients by the chain rule eq. bas_deriv: grad phi = R_T^{-T} grad^ phi^.
* Element matrices by the collapsed Gauss rule of ``reference.collapsed_gauss``:
  weighted projection (eq. bilf_gp, eq. linsys_gp) A_T = J sum_q w_q m(x_q) phi phi^T;
  elliptic problem (eq. bilf_se, eq. linsys_se)
  A_T = J sum_q w_q G_q^T R^{-1} M(x_q) R^{-T} G_q.
* Assembly into CSR with scipy.sparse (duplicates summed, no threshold).
* Boundary dofs: nodes on a facet that belongs to a single cell.

Parity pins: the P1 five-point stencil, textbook P1/P2 mass matrices
(tests/golden), Neumann null space, mass sum, dim V = (kN+1)^d, manufactured
solution convergence rates, and the exact structural nnz of Tables 3-4.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import reference as ref

__all__ = [
    "Space",
    "make_space",
    "geometry",
    "unpack_sym",
    "element_matrices",
    "assemble",
    "load_vector",
    "structural_nnz",
    "quad_order",
]


def local_barycentric(d: int, k: int) -> np.ndarray:
    """Barycentric multi-indices b (|b| = k) of the local nodes, in the order of
    ``reference.lattice(d, k)``: b_0 = k - |a|, b_r = a_r."""
    a = np.array(ref.multi_indices(d, k), dtype=np.int64)
    return np.concatenate([k - a.sum(1, keepdims=True), a], axis=1)


class Space:
    """C_{N,k} on a mesh: cell_dofs [nel, V_T], dof coordinates, boundary dofs."""

    def __init__(self, coords, cells, k, cell_dofs, dof_coords, boundary):
        self.coords = coords
        self.cells = cells
        self.k = k
        self.d = cells.shape[1] - 1
        self.cell_dofs = cell_dofs
        self.dof_coords = dof_coords
        self.boundary = boundary
        self.ndofs = dof_coords.shape[0]

    @property
    def interior(self):
        mask = np.ones(self.ndofs, bool)
        mask[self.boundary] = False
        return np.nonzero(mask)[0]


def make_space(coords: np.ndarray, cells: np.ndarray, k: int) -> Space:
    nel, nv1 = cells.shape
    d = nv1 - 1
    b = local_barycentric(d, k)  # [V_T, d+1]
    vt = b.shape[0]
    cells64 = cells.astype(np.int64)
    big = np.iinfo(np.int64).max
    verts = np.where(b[None, :, :] > 0, cells64[:, None, :], big)  # [nel, V_T, d+1]
    mults = np.broadcast_to(b[None], verts.shape)
    order = np.argsort(verts, axis=2, kind="stable")
    sv = np.take_along_axis(verts, order, 2)
    sm = np.take_along_axis(mults, order, 2)
    sv = np.where(sv == big, -1, sv)
    sm = np.where(sv == -1, -1, sm)
    keys = np.concatenate([sv, sm], axis=2).reshape(nel * vt, 2 * nv1)
    uniq, first, inv = np.unique(keys, axis=0, return_index=True, return_inverse=True)
    cell_dofs = inv.reshape(nel, vt).astype(np.int64)
    ndofs = uniq.shape[0]

    # node coordinates sum_j (b_j / k) X_j, taken at the first occurrence
    X = coords[cells64]  # [nel, d+1, d]
    xyz = np.einsum("vj,ejx->evx", b / k, X).reshape(nel * vt, d)
    dof_coords = xyz[first]

    # boundary facets: facet j of a cell omits vertex j
    fac = np.stack([np.sort(np.delete(cells64, j, axis=1), axis=1) for j in range(nv1)], axis=1)
    _, finv, fcnt = np.unique(fac.reshape(-1, d), axis=0, return_inverse=True, return_counts=True)
    fbnd = (fcnt[finv] == 1).reshape(nel, nv1)
    # node lies on facet j iff b_j == 0
    on = (b[None, :, :] == 0) & fbnd[:, None, :]
    node_bnd = on.any(axis=2).reshape(-1)
    boundary = np.unique(cell_dofs.reshape(-1)[node_bnd])
    return Space(coords, cells, k, cell_dofs, dof_coords, boundary)


def geometry(coords: np.ndarray, cells: np.ndarray):
    """R_T [nel, d, d] (columns X_r - X_0), J = |det R_T|, R_T^{-1}, S_T = X_0."""
    X = coords[cells.astype(np.int64)]
    R = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    det = np.linalg.det(R)
    return R, np.abs(det), np.linalg.inv(R), X[:, 0, :]


def unpack_sym(packed: np.ndarray, d: int) -> np.ndarray:
    """Upper triangle row by row -> full symmetric [.., d, d]."""
    iu = np.triu_indices(d)
    full = np.zeros(packed.shape[:-1] + (d, d))
    full[..., iu[0], iu[1]] = packed
    full[..., iu[1], iu[0]] = packed
    return full


def quad_order(k: int, extra: int = 0) -> int:
    """Points per direction of the collapsed rule: exact for degree 2k integrands
    (2n - d >= 2k for d <= 3), plus ``extra`` for smooth varying coefficients."""
    return k + 2 + extra


def _coef_at(coef, d, nel, xq, kind):
    """Coefficient at physical quadrature points: scalar [nel, nq] or tensor [nel, nq, d, d]."""
    nq = xq.shape[1]
    if callable(coef):
        return coef(xq)
    c = np.asarray(coef, dtype=np.float64)
    if kind == "wp" or c.ndim == 1:
        if c.ndim != 1:
            raise ValueError("scalar coefficient expected")
        return np.broadcast_to(c[:, None], (nel, nq))
    if c.ndim == 2:  # packed symmetric
        c = unpack_sym(c, d)
    return np.broadcast_to(c[:, None, :, :], (nel, nq, d, d))


def element_matrices(space: Space, coef, kind: str, nquad: int | None = None) -> np.ndarray:
    """Quadrature element matrices A_T [nel, V_T, V_T] (eq. linsys_gp / linsys_se)."""
    d, k = space.d, space.k
    n = nquad or quad_order(k)
    pts, wts = ref.collapsed_gauss(d, n)
    R, J, Rinv, S = geometry(space.coords, space.cells)
    nel = R.shape[0]
    xq = S[:, None, :] + np.einsum("exr,qr->eqx", R, pts)
    c = _coef_at(coef, d, nel, xq, kind)
    if kind == "wp":
        phi = ref.eval_basis(d, k, pts)  # [nq, V_T]
        return np.einsum("e,q,eq,qk,ql->ekl", J, wts, c, phi, phi)
    if kind == "se":
        if c.ndim == 2:  # scalar (isotropic, Corollary) -> m I
            c = c[:, :, None, None] * np.eye(d)
        G = ref.eval_basis_grad(d, k, pts)  # [nq, d, V_T]
        K = np.einsum("erp,eqpt,est->eqrs", Rinv, c, Rinv)  # R^{-1} M R^{-T}
        return np.einsum("e,q,qrk,eqrs,qsl->ekl", J, wts, G, K, G)
    raise ValueError(kind)


def assemble(space: Space, Ae: np.ndarray) -> sp.csr_matrix:
    """Sum of P_T^T A_T P_T as CSR (duplicates summed, nothing dropped)."""
    cd = space.cell_dofs
    vt = cd.shape[1]
    rows = np.repeat(cd, vt, axis=1).reshape(-1)
    cols = np.tile(cd, (1, vt)).reshape(-1)
    A = sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(space.ndofs, space.ndofs)).tocsr()
    A.sum_duplicates()
    return A


def load_vector(space: Space, f, nquad: int | None = None) -> np.ndarray:
    """b_i = int f phi_i (constant f or callable of physical points [.., d])."""
    d, k = space.d, space.k
    n = nquad or quad_order(k, 2)
    pts, wts = ref.collapsed_gauss(d, n)
    R, J, Rinv, S = geometry(space.coords, space.cells)
    xq = S[:, None, :] + np.einsum("exr,qr->eqx", R, pts)
    fv = f(xq) if callable(f) else np.full(xq.shape[:2], float(f))
    phi = ref.eval_basis(d, k, pts)
    bT = np.einsum("e,q,eq,qk->ek", J, wts, fv, phi)
    return np.bincount(space.cell_dofs.reshape(-1), weights=bT.reshape(-1), minlength=space.ndofs)


def structural_nnz(space: Space) -> int:
    """Number of (i, j) dof pairs that share a cell (the CSR pattern without cancellation)."""
    cd = space.cell_dofs
    vt = cd.shape[1]
    rows = np.repeat(cd, vt, axis=1).reshape(-1)
    cols = np.tile(cd, (1, vt)).reshape(-1)
    pat = sp.coo_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(space.ndofs, space.ndofs)).tocsr()
    pat.sum_duplicates()
    return int(pat.nnz)


def simplex_volume_factor(d: int) -> float:
    """|T| = J / d!."""
    return 1.0 / math.factorial(d)
