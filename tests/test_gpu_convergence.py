"""The GPU solution against the exact solution of a boundary value problem (no oracle):
-div grad u = f on the unit square and cube, u = prod_j sin(pi x_j), zero Dirichlet data,
f = d pi^2 u.  The right-hand side is the projection operator's mass matrix (Theorem 2,
m = 1) applied to the nodal interpolant of f, so the discrete solution differs from u by
O(h^{k+1}) in the mean over the nodes; the nodal RMS error must fall at that rate under
refinement.  Solved with Jacobi-PCG in FP64 and with the mixed and multigrid modes."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nodal_rms_error(d, n, k, mode):
    from paper_1710_09913_amd import Mesh, Operator, Space

    mesh = Mesh.unit(d, n)
    se = Space(mesh, k, "se", "dirichlet")
    wp = Space(mesh, k, "wp", "none")
    x = se.dof_coords()
    assert np.array_equal(x, wp.dof_coords())  # the same numbering on one mesh and order
    uex = np.prod(np.sin(np.pi * x), axis=1)
    f = d * math.pi ** 2 * uex
    A = Operator(se, torch.ones(se.ncells, dtype=torch.float64), "scalar", fp32=True)
    M = Operator(wp, torch.ones(wp.ncells, dtype=torch.float64), "scalar", fp32=False)
    b = M.apply(torch.from_numpy(f).cuda())
    b[torch.from_numpy(se.boundary().astype(np.int64)).cuda()] = 0.0
    uh, st = A.pcg(b, tol=1e-12, maxit=50000, mode=mode)
    assert st["status"] == 0, st
    return float(np.sqrt(np.mean((uh.cpu().numpy() - uex) ** 2)))


@pytest.mark.parametrize("d,k,ns", [(2, 1, (8, 16, 32)), (2, 2, (8, 16, 32)), (2, 3, (4, 8, 16)), (3, 2, (4, 8, 16)),
                                    (3, 3, (4, 8, 16))])
@pytest.mark.parametrize("mode", ["f64", "mixed", "pmg_mixed"])
def test_nodal_error_rate(d, k, ns, mode):
    print(f"[convergence] d={d} k={k} {mode}", flush=True)
    errs = [_nodal_rms_error(d, n, k, mode) for n in ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"errors {errs}, rates {rates}", flush=True)
    # the asymptotic rate is k + 1 (k + 2 at the nodes for even k would only help)
    assert min(rates[-1:]) >= k + 1 - 0.3, rates


@pytest.mark.parametrize("d,k", [(2, 1), (2, 3), (2, 5), (3, 1), (3, 2), (3, 3)])
def test_constants_in_the_neumann_null_space(d, k):
    """Without boundary conditions the elliptic operator annihilates constants (the
    gradients of the basis sum to zero), on a jittered mesh with an anisotropic
    coefficient: |A 1| within the rounding of |B^|^T|D||B^| 1, in FP64 and FP32; and u^T A u
    > 0 for a random u (positive semidefinite, zero only on constants)."""
    from test_gpu_apply import Case

    c = Case(d, 6 if d == 2 else 3, k, "se", seed=5, bc="none")
    one = np.ones(c.space.ndofs)
    bound = c.abs_bound(one)
    info = c.space.info
    m = info["vt"] + info["nb"] * info["wt"] + info["nb"] + c.n_incident_max() + 3
    gam32 = 2 * m * 2.0 ** -24 / (1 - m * 2.0 ** -24)  # the FP32 bound of the apply tests
    for prec, tol in (("f64", 1e-12), ("f32", gam32)):
        y = c.op.apply(torch.from_numpy(one).cuda(), prec=prec).cpu().numpy()
        assert np.all(np.abs(y) <= tol * bound + 1e-300), (prec, float(np.abs(y).max()))
    u = np.random.default_rng(3).standard_normal(c.space.ndofs)
    assert float(u @ c.op.apply(torch.from_numpy(u).cuda()).cpu().numpy()) > 0.0
