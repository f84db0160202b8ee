"""Adjoint gradients of DoGIP solves behind torch.autograd.

For the elliptic problem with per-cell coefficient a_T = exp(theta_T) and zero
Dirichlet rows, u(theta, b) solves A(theta) u = b.  A is symmetric, so for a loss
L(u) the backward pass needs one adjoint solve A lam = dL/du; then
    dL/db = lam,
    dL/dtheta_T = -lam^T (dA/dtheta_T) u = -lam_T^T A_T u_T = -(B^ lam_T) . D_T (B^ u_T),
because A_T (and D_T) scale with exp(theta_T).  The contraction runs in the
library's HIP kernel (dogip_grad_logcoef); the solves run in its PCG.
"""

from __future__ import annotations

import torch

from .dogip import Operator

__all__ = ["DogipSolve", "solve"]


class DogipSolve(torch.autograd.Function):
    """u = A(theta)^-1 b.  Inputs: theta [ncells] (log-coefficients, mesh cell order),
    b [ndofs]; the operator is rebuilt from theta (D construction on the device)."""

    @staticmethod
    def forward(ctx, theta, b, op: Operator, tol: float, mode: str, maxit: int):
        theta = theta.detach().to(device="cuda", dtype=torch.float64).contiguous()
        op.set_coef(theta, "logscalar")
        u, st = op.pcg(b.detach().contiguous(), tol=tol, maxit=maxit, mode=mode, raise_on_error=False)
        if st["status"] not in (0, 6):
            raise RuntimeError(f"forward solve failed: {st}")
        ctx.save_for_backward(theta, u)
        ctx.op, ctx.tol, ctx.mode, ctx.maxit = op, tol, mode, maxit
        ctx.stats = st
        return u

    @staticmethod
    def backward(ctx, gu):
        theta, u = ctx.saved_tensors
        op = ctx.op
        op.set_coef(theta, "logscalar")  # the operator may have been reused since the forward
        lam, st = op.pcg(gu.detach().to(torch.float64).contiguous(), tol=ctx.tol, maxit=ctx.maxit, mode=ctx.mode,
                         raise_on_error=False)
        if st["status"] not in (0, 6):
            raise RuntimeError(f"adjoint solve failed: {st}")
        g = op.grad_logcoef(u, lam)
        return g, lam, None, None, None, None


def solve(theta, b, op: Operator, tol: float = 1e-12, mode: str = "f64", maxit: int = 50000):
    """Differentiable u(theta, b)."""
    return DogipSolve.apply(theta, b, op, tol, mode, maxit)
