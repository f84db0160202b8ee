"""Element-wise DoGIP: D construction and the element loop (oracle, test infrastructure).

* Weighted projection, Theorem 2: A^DoGIP_T,ij = delta_ij int_T m phi^W_j.  For a
  coefficient constant on T this is m_T |T| w^_j; for a coefficient varying on T
  it is the same collapsed Gauss rule as the standard FEM assembly applied to
  m phi^W_j (the decomposition is linear in the integration functional, so it
  reproduces the quadrature-assembled matrix exactly).
* Elliptic problem, Theorem 4: A^DoGIP_T,rs,ii = (R_T^{-1} (int_T M phi^W_i) R_T^{-T})_rs
  with W = D_{N,2k-2} (reading of the theorem's W = D_{N,k} by the preceding
  lemma and by the W_T column of Tables 3-4).  For isotropic M = m I the block is
  m R^{-1} R^{-T} times the scalar integral (Corollary of Theorem 3).
* Algorithm 1: for every cell, gather u_T, compute B^^T D_T B^ u_T from the
  right and add it to the output.  The algorithm as printed omits the
  transpose on the left factor; eq. ep_dogip_mul fixes it as B^^T (adjoint).
  Cells are processed in batches with numpy; the scatter is np.bincount.

D layouts returned: [nel, W_T] (weighted projection) and [nel, W_T, d, d] (elliptic).
Pinned by the identity B^^T D B^ = A against ``fem`` (tests/test_oracle_dogip.py).
``apply_abs`` (the rounding scale of the parity checks) is pinned in
tests/test_oracle_apply_abs.py: it equals the assembled operator where nothing is
negative, lies between sum_T |A_T||u_T| and |A u| by the triangle inequality, is the
absolute textbook P1 stiffness on the reference simplex, and keeps Dirichlet rows.
``apply_abs_factored`` is the same scale for an apply that forms B^ u_T through the
factors of ``reference.bhat_factors`` (the gradient at the P_{k-1} nodes, then P_{k-1}
interpolation to the W nodes); pinned in tests/test_oracle_factored.py.
"""

from __future__ import annotations

import math

import numpy as np

from . import fem
from . import reference as ref

__all__ = ["build_d", "apply", "apply_dirichlet", "apply_abs", "apply_abs_factored", "diagonal", "energy_contraction"]


def build_d(space: fem.Space, coef, kind: str, nquad: int | None = None) -> np.ndarray:
    """D per cell.  ``coef``: [nel] scalar, [nel, d(d+1)/2] packed or [nel, d, d] tensor
    (elliptic only), or a callable of physical points (varying inside the cell)."""
    d, k = space.d, space.k
    q = ref.w_order(k, kind)
    R, J, Rinv, S = fem.geometry(space.coords, space.cells)
    nel = R.shape[0]
    vol = J / math.factorial(d)
    if callable(coef):
        n = nquad or fem.quad_order(k)
        pts, wts = ref.collapsed_gauss(d, n)
        xq = S[:, None, :] + np.einsum("exr,qr->eqx", R, pts)
        c = coef(xq)
        phiw = ref.eval_basis(d, q, pts)  # [nq, W_T]
        if kind == "wp":
            return np.einsum("e,q,eq,qi->ei", J, wts, c, phiw)
        if c.ndim == 2:
            c = c[:, :, None, None] * np.eye(d)
        integ = np.einsum("e,q,eqpt,qi->eipt", J, wts, c, phiw)  # int_T M phi_i
        return np.einsum("erp,eipt,est->eirs", Rinv, integ, Rinv)
    w = ref.what(d, q)
    c = np.asarray(coef, dtype=np.float64)
    if kind == "wp":
        return (c * vol)[:, None] * w[None, :]
    if kind != "se":
        raise ValueError(kind)
    if c.ndim == 1:
        c = c[:, None, None] * np.eye(d)
    elif c.ndim == 2:
        c = fem.unpack_sym(c, d)
    K = np.einsum("erp,ept,est->ers", Rinv, c, Rinv)
    return (vol[:, None, None, None] * w[None, :, None, None]) * K[:, None, :, :]


def _element_products(B, D, uT, kind):
    if kind == "wp":
        g = uT @ B.T                  # B^ u_T            [nb, W_T]
        h = D * g                     # A^DoGIP_T (.)      [nb, W_T]
        return h @ B                  # B^^T (.)          [nb, V_T]
    g = np.einsum("riv,ev->eir", B, uT)        # B^ u_T, [nb, W_T, d]
    h = np.einsum("eirs,eis->eir", D, g)       # D_T, per W node a d x d block
    return np.einsum("riv,eir->ev", B, h)      # B^^T


def apply(space: fem.Space, D: np.ndarray, u: np.ndarray, kind: str, batch: int = 65536) -> np.ndarray:
    """y = sum_T P_T^T B^^T D_T B^ P_T u (Algorithm 1, no boundary conditions)."""
    B = ref.bhat(space.d, space.k, kind)
    cd = space.cell_dofs
    y = np.zeros(space.ndofs)
    for s in range(0, cd.shape[0], batch):
        c = cd[s:s + batch]
        yT = _element_products(B, D[s:s + batch], u[c], kind)
        y += np.bincount(c.reshape(-1), weights=yT.reshape(-1), minlength=space.ndofs)
    return y


def apply_dirichlet(space: fem.Space, D: np.ndarray, u: np.ndarray, kind: str) -> np.ndarray:
    """Operator with zero-Dirichlet identity rows: y_I = (A (u with u_B = 0))_I, y_B = u_B."""
    ut = u.copy()
    ut[space.boundary] = 0.0
    y = apply(space, D, ut, kind)
    y[space.boundary] = u[space.boundary]
    return y


def apply_abs(space: fem.Space, D: np.ndarray, u: np.ndarray, kind: str, dirichlet: bool) -> np.ndarray:
    """|B^|^T |D| |B^| |u| per cell, summed: the scale of the rounding error of an apply."""
    B = np.abs(ref.bhat(space.d, space.k, kind))
    ua = np.abs(u).copy()
    if dirichlet:
        ua[space.boundary] = 0.0
    cd = space.cell_dofs
    y = np.zeros(space.ndofs)
    for s in range(0, cd.shape[0], 65536):
        c = cd[s:s + 65536]
        yT = _element_products(B, np.abs(D[s:s + 65536]), ua[c], kind)
        y += np.bincount(c.reshape(-1), weights=yT.reshape(-1), minlength=space.ndofs)
    if dirichlet:
        y[space.boundary] = np.abs(u[space.boundary])
    return y


def apply_abs_factored(space: fem.Space, D: np.ndarray, u: np.ndarray, dirichlet: bool) -> np.ndarray:
    """|B1|^T (I (x) |B2|)^T |D| (I (x) |B2|) |B1| |u| per cell, summed (elliptic problem):
    the rounding scale of an apply through the factors B^_r = B2 B1_r."""
    B1, B2 = ref.bhat_factors(space.d, space.k)
    B1, B2 = np.abs(B1), np.abs(B2)
    ua = np.abs(u).copy()
    if dirichlet:
        ua[space.boundary] = 0.0
    cd = space.cell_dofs
    y = np.zeros(space.ndofs)
    for s in range(0, cd.shape[0], 65536):
        c = cd[s:s + 65536]
        G = np.einsum("rjv,ev->erj", B1, ua[c])                 # |B1| |u_T|, per component and P_{k-1} node
        g = np.einsum("ij,erj->eir", B2, G)                     # |B2| (.) at the W nodes
        h = np.einsum("eirs,eis->eir", np.abs(D[s:s + 65536]), g)
        H = np.einsum("ij,eir->erj", B2, h)                     # |B2|^T (.)
        yT = np.einsum("rjv,erj->ev", B1, H)                    # |B1|^T (.)
        y += np.bincount(c.reshape(-1), weights=yT.reshape(-1), minlength=space.ndofs)
    if dirichlet:
        y[space.boundary] = np.abs(u[space.boundary])
    return y


def diagonal(space: fem.Space, D: np.ndarray, kind: str, dirichlet: bool) -> np.ndarray:
    """diag(B^^T D B^) summed over cells; identity rows on the Dirichlet boundary."""
    B = ref.bhat(space.d, space.k, kind)
    if kind == "wp":
        dT = np.einsum("iv,ei,iv->ev", B, D, B)
    else:
        dT = np.einsum("riv,eirs,siv->ev", B, D, B)
    out = np.bincount(space.cell_dofs.reshape(-1), weights=dT.reshape(-1), minlength=space.ndofs)
    if dirichlet:
        out[space.boundary] = 1.0
    return out


def energy_contraction(space: fem.Space, D: np.ndarray, u: np.ndarray, lam: np.ndarray, kind: str,
                       dirichlet: bool) -> np.ndarray:
    """Per cell (B^ lam_T) . D_T (B^ u_T) = lam_T^T A_T u_T (boundary entries masked)."""
    B = ref.bhat(space.d, space.k, kind)
    u = u.copy()
    lam = lam.copy()
    if dirichlet:
        u[space.boundary] = 0.0
        lam[space.boundary] = 0.0
    cd = space.cell_dofs
    yT = _element_products(B, D, u[cd], kind)
    return np.einsum("ev,ev->e", lam[cd], yT)
