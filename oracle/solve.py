"""Linear solvers for the oracle (test infrastructure).

The paper leaves the iterative solver open (Section 1, "a suitable iterative
solver").  Reading used here: conjugate gradients preconditioned by the Jacobi
diagonal, x_0 = 0, stopped when ||b - A x||_2 / ||b||_2 <= tol (recursively
updated residual).  The direct solve (scipy SuperLU) is the pin for CG.

Zero Dirichlet conditions: the interior block A_II is solved; boundary values are
zero.  The identity-row form used by the HIP path (rows and columns of boundary
dofs replaced by the identity) has the same interior solution.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["pcg", "direct_dirichlet", "dirichlet_matrix"]


def pcg(matvec, b: np.ndarray, diag: np.ndarray, tol: float, maxit: int = 100000):
    """Jacobi-preconditioned CG.  Returns (x, iterations, final relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = r / diag
    p = z.copy()
    rho = r @ z
    it = 0
    while it < maxit:
        if np.linalg.norm(r) <= tol * nb:
            break
        q = matvec(p)
        pq = p @ q
        if not (pq > 0.0):
            raise FloatingPointError("CG breakdown: p^T A p <= 0")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        z = r / diag
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it, float(np.linalg.norm(r) / nb)


def dirichlet_matrix(A: sp.csr_matrix, boundary: np.ndarray) -> sp.csr_matrix:
    """A with boundary rows/columns replaced by identity rows/columns."""
    n = A.shape[0]
    keep = np.ones(n)
    keep[boundary] = 0.0
    P = sp.diags(keep)
    E = sp.diags(1.0 - keep)
    return (P @ A @ P + E).tocsr()


def direct_dirichlet(A: sp.csr_matrix, b: np.ndarray, boundary: np.ndarray) -> np.ndarray:
    """Solve A_II x_I = b_I with x_B = 0 by sparse LU."""
    n = A.shape[0]
    mask = np.ones(n, bool)
    mask[boundary] = False
    I = np.nonzero(mask)[0]
    x = np.zeros(n)
    x[I] = spla.splu(A[I][:, I].tocsc()).solve(b[I])
    return x
