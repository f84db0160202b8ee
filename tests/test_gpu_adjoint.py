"""Adjoint gradient through torch.autograd: against the oracle gradient (small mesh) and
against central finite differences on the full 2D 256^2 P3 inverse problem."""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import adjoint, fem
from workloads import theta_normal, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("mode", ["f64", "pmg"])
def test_autograd_matches_oracle_gradient(mode):
    """Forward and adjoint solves by Jacobi-PCG or by multigrid-preconditioned CG."""
    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.autograd import solve

    n, k = 8, 3
    coords, cells = unit_mesh(2, n, jitter=0.1, seed=2)
    nel = len(cells)
    osp = fem.make_space(coords, cells, k)
    b = fem.load_vector(osp, 1.0)
    b[osp.boundary] = 0.0
    u_star, _, _ = adjoint.forward(osp, theta_normal(nel, 11), b)
    u_obs = u_star + 0.01 * np.sqrt(np.mean(u_star ** 2)) * np.random.default_rng(3).standard_normal(osp.ndofs)
    u_obs[osp.boundary] = 0.0
    theta0 = theta_normal(nel, 4)
    J_o, g_o, _, lam_o = adjoint.gradient(osp, theta0, b, u_obs)

    sp = Space(Mesh(coords, cells), k, "se", "dirichlet")
    perm = match_dofs(sp.dof_coords(), osp.dof_coords)
    op = Operator(sp, torch.zeros(nel, dtype=torch.float64), "logscalar", fp32=False)
    theta = torch.from_numpy(theta0).cuda().requires_grad_(True)
    bt = torch.from_numpy(b[perm]).cuda().requires_grad_(True)
    u = solve(theta, bt, op, tol=1e-13, mode=mode)
    J = 0.5 * ((u - torch.from_numpy(u_obs[perm]).cuda()) ** 2).sum()
    J.backward()
    assert abs(J.item() - J_o) <= 1e-9 * J_o
    assert rel_err(theta.grad.cpu().numpy(), g_o) <= 1e-8
    assert rel_err(bt.grad.cpu().numpy(), lam_o[perm]) <= 1e-8


def test_adjoint_vs_finite_differences_full_size():
    """2D 256^2 P3, theta ~ N(0, 0.5^2), u_obs from a hidden theta* plus 1 % noise:
    dJ/dtheta . v against (J(theta + h v) - J(theta - h v)) / (2 h), h = 1e-6, 32 directions."""
    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.autograd import solve

    n, k = 256, 3
    sp = Space(Mesh.unit(2, n), k, "se", "dirichlet")
    nel = sp.ncells
    op = Operator(sp, torch.zeros(nel, dtype=torch.float64), "logscalar", fp32=False)
    wp = Operator(Space(sp.mesh, k, "wp", "none"), torch.ones(nel, dtype=torch.float64), "scalar", fp32=False)
    b = wp.apply(torch.ones(sp.ndofs, dtype=torch.float64, device="cuda"))
    b[torch.from_numpy(sp.boundary().astype(np.int64)).cuda()] = 0.0
    tol = 1e-14
    with torch.no_grad():
        u_star = solve(torch.from_numpy(theta_normal(nel, 99)).cuda(), b, op, tol=tol)
        rms = torch.sqrt(torch.mean(u_star ** 2))
        noise = torch.from_numpy(np.random.default_rng(5).standard_normal(sp.ndofs)).cuda()
        u_obs = u_star + 0.01 * rms * noise
        u_obs[torch.from_numpy(sp.boundary().astype(np.int64)).cuda()] = 0.0

    def J(th):
        u = solve(th, b, op, tol=tol)
        return 0.5 * ((u - u_obs) ** 2).sum()

    theta = torch.from_numpy(theta_normal(nel, 1)).cuda().requires_grad_(True)
    Jv = J(theta)
    Jv.backward()
    g = theta.grad.detach()
    rng = np.random.default_rng(7)
    h = 1e-6
    errs = []
    with torch.no_grad():
        for _ in range(32):
            v = torch.from_numpy(rng.standard_normal(nel)).cuda()
            fd = (J(theta.detach() + h * v) - J(theta.detach() - h * v)).item() / (2 * h)
            gv = torch.dot(g, v).item()
            errs.append(abs(fd - gv) / abs(gv))
    print(f"J={Jv.item():.6e} FD relative errors: max {max(errs):.2e} median {np.median(errs):.2e}", flush=True)
    assert max(errs) <= 1e-5
