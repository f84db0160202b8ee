"""Adjoint gradient for per-cell log-coefficients (oracle, test infrastructure).

Problem (elliptic, zero Dirichlet): a_T = exp(theta_T), A(theta) u = b,
J(theta) = 0.5 ||u - u_obs||_2^2 over the dof vector.  With the adjoint solve
A lambda = u - u_obs (A symmetric) and dA/dtheta_T = A_T (the cell matrix scales
with a_T), dJ/dtheta_T = -lambda_T^T A_T u_T, both vectors with boundary
entries zero.  The cell matrices come from the quadrature assembly of ``fem``
(independent of B^), so this pins the DoGIP contraction -(B^ lambda).D(B^ u).
The gradient itself is pinned by central finite differences with direct solves.
"""

from __future__ import annotations

import numpy as np

from . import fem
from . import solve

__all__ = ["forward", "objective", "gradient", "fd_directional"]


def forward(space: fem.Space, theta: np.ndarray, b: np.ndarray):
    """u(theta) by direct solve; returns (u, A, cell matrices)."""
    Ae = fem.element_matrices(space, np.exp(theta), "se")
    A = fem.assemble(space, Ae)
    return solve.direct_dirichlet(A, b, space.boundary), A, Ae


def objective(space, theta, b, u_obs) -> float:
    u, _, _ = forward(space, theta, b)
    r = u - u_obs
    return 0.5 * float(r @ r)


def gradient(space, theta, b, u_obs):
    """(J, dJ/dtheta [nel], u, lambda)."""
    u, A, Ae = forward(space, theta, b)
    r = u - u_obs
    lam = solve.direct_dirichlet(A, r, space.boundary)
    um = u.copy()
    lm = lam.copy()
    um[space.boundary] = 0.0
    lm[space.boundary] = 0.0
    cd = space.cell_dofs
    g = -np.einsum("ek,ekl,el->e", lm[cd], Ae, um[cd])
    return 0.5 * float(r @ r), g, u, lam


def fd_directional(space, theta, b, u_obs, v, h=1e-6) -> float:
    """Central difference (J(theta + h v) - J(theta - h v)) / (2 h)."""
    return (objective(space, theta + h * v, b, u_obs) - objective(space, theta - h * v, b, u_obs)) / (2 * h)
