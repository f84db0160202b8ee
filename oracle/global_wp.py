"""Global DoGIP for the weighted projection (oracle, test infrastructure).

Theorem 1: with V = C_{N,k} and the continuous double-grid space W = C_{N,2k}
(the product of two functions of V lies in W, lemma of Section 2.2), the
matrix of eq. linsys_gp factors as A = B^T A^DoGIP B with
  * A^DoGIP diagonal over the global W dofs: A^DoGIP_jj = int_Omega m phi^W_j,
  * B in R^{W x V} the interpolation of V at the W nodes: B_jl = phi^V_l(x^W_j).
Unlike the element-wise form (Theorem 2), each W dof shared by several cells is
stored once.  The remark after Tables 1-2 expects this to save memory at low k.

Written from the theorem as a literal product of a sparse B with a diagonal:
  * W numbering: ``fem.make_space`` at order 2k.
  * B: each cell contributes the rows of its W nodes (its reference B^ of
    Theorem 2) in the global numbering; a row shared by several cells is taken
    once (the cells agree on it, which ``interpolation_matrix`` checks).
  * A^DoGIP_jj: the sum over the cells holding W node j of int_T m phi^W_j, that
    is of the element-wise diagonal of Theorem 2 (``dogip.build_d``).

Pinned in tests/test_oracle_global.py by: equality with the quadrature-assembled
FEM matrix (the theorem), B u = p(x^W) for p linear (interpolation), the closed
form dim C_{N,2k} = (2kN + 1)^d on the unit meshes, sum_j A^DoGIP_jj = int m, and
the P2 vertex weights being zero (closed Newton-Cotes, m = 1).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dogip as odg
from . import fem
from . import reference as ref

__all__ = ["w_space", "interpolation_matrix", "build_d_global", "apply_global"]


def w_space(space: fem.Space) -> fem.Space:
    """The continuous double-grid space C_{N,2k} on the mesh of ``space``."""
    return fem.make_space(space.coords, space.cells, 2 * space.k)


def interpolation_matrix(space: fem.Space, wsp: fem.Space) -> sp.csr_matrix:
    """B [dim W, dim V] with B_jl = phi^V_l(x^W_j)."""
    B = ref.bhat(space.d, space.k, "wp")  # [W_T, V_T]
    nel, wt = wsp.cell_dofs.shape
    vt = space.cell_dofs.shape[1]
    rows = np.repeat(wsp.cell_dofs[:, :, None], vt, axis=2).reshape(-1)
    cols = np.repeat(space.cell_dofs[:, None, :], wt, axis=1).reshape(-1)
    vals = np.broadcast_to(B[None], (nel, wt, vt)).reshape(-1)
    # one entry per (row, col): the first cell's; every cell holding the row must agree
    key = rows * space.ndofs + cols
    uk, first, inv = np.unique(key, return_index=True, return_inverse=True)
    agree = np.abs(vals - vals[first][inv]).max(initial=0.0)
    if agree != 0.0:
        raise AssertionError(f"cells disagree on a row of B by {agree}")
    keep = vals[first] != 0.0
    return sp.csr_matrix((vals[first][keep], (rows[first][keep], cols[first][keep])),
                         shape=(wsp.ndofs, space.ndofs))


def build_d_global(space: fem.Space, wsp: fem.Space, coef) -> np.ndarray:
    """A^DoGIP_jj = int_Omega m phi^W_j [dim W], summed from the cells' integrals."""
    De = odg.build_d(space, coef, "wp")  # [nel, W_T]: int_T m phi^W_i
    return np.bincount(wsp.cell_dofs.reshape(-1), weights=De.reshape(-1), minlength=wsp.ndofs)


def apply_global(space: fem.Space, wsp: fem.Space, Dg: np.ndarray, u: np.ndarray,
                 B: sp.csr_matrix | None = None) -> np.ndarray:
    """y = B^T (A^DoGIP (B u)) (Theorem 1)."""
    B = interpolation_matrix(space, wsp) if B is None else B
    return B.T @ (Dg * (B @ u))
