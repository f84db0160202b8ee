"""Oracle solvers and adjoint gradient against direct solves and finite differences."""

import numpy as np
import pytest

from oracle import adjoint, dogip, fem, solve
from workloads import unit_mesh, coef_uniform, theta_normal, random_vector


def test_pcg_matches_direct_small_p2():
    """2D 16x16 P2 elliptic, a ~ U[1, 10], f = 1: Jacobi-PCG to 1e-10 equals the sparse LU
    solution within the residual bound kappa * tol."""
    coords, cells = unit_mesh(2, 16)
    sp = fem.make_space(coords, cells, 2)
    a = coef_uniform(len(cells), 1, 10, 0)
    A = fem.assemble(sp, fem.element_matrices(sp, a, "se"))
    b = fem.load_vector(sp, 1.0)
    b[sp.boundary] = 0.0
    Ab = solve.dirichlet_matrix(A, sp.boundary)
    x_lu = solve.direct_dirichlet(A, b, sp.boundary)
    D = dogip.build_d(sp, a, "se")
    diag = dogip.diagonal(sp, D, "se", True)
    x, it, rel = solve.pcg(lambda v: dogip.apply_dirichlet(sp, D, v, "se"), b, diag, 1e-10)
    assert rel <= 1e-10
    assert np.linalg.norm(b - Ab @ x) <= 1.01e-10 * np.linalg.norm(b)
    ev = np.linalg.eigvalsh(Ab.toarray())
    kappa = ev.max() / ev.min()
    assert np.linalg.norm(x - x_lu) <= 2 * kappa * 1e-10 * np.linalg.norm(x_lu)
    assert 10 < it < 500


def test_pcg_breakdown_on_indefinite():
    A = np.diag([1.0, -1.0, 2.0])
    with pytest.raises(FloatingPointError):
        solve.pcg(lambda v: A @ v, np.array([1.0, 1.0, 0.0]), np.ones(3), 1e-12)


@pytest.mark.parametrize("k", [2, 3])
def test_adjoint_gradient_vs_finite_differences(k):
    """dJ/dtheta from one adjoint solve matches central differences (h = 1e-6) in 8 random
    directions to 1e-5 relative."""
    coords, cells = unit_mesh(2, 4, jitter=0.1, seed=1)
    sp = fem.make_space(coords, cells, k)
    nel = len(cells)
    b = fem.load_vector(sp, 1.0)
    b[sp.boundary] = 0.0
    theta_star = theta_normal(nel, 9)
    u_star, _, _ = adjoint.forward(sp, theta_star, b)
    u_obs = u_star + 0.01 * np.sqrt(np.mean(u_star ** 2)) * np.random.default_rng(4).standard_normal(sp.ndofs)
    u_obs[sp.boundary] = 0.0
    theta = theta_normal(nel, 2)
    J, g, u, lam = adjoint.gradient(sp, theta, b, u_obs)
    rng = np.random.default_rng(7)
    for _ in range(8):
        v = rng.standard_normal(nel)
        fd = adjoint.fd_directional(sp, theta, b, u_obs, v)
        assert abs(fd - g @ v) <= 1e-5 * abs(g @ v) + 1e-12
    # the DoGIP contraction gives the same gradient as the quadrature cell matrices
    D = dogip.build_d(sp, np.exp(theta), "se")
    gd = -dogip.energy_contraction(sp, D, u, lam, "se", True)
    np.testing.assert_allclose(gd, g, rtol=1e-9, atol=1e-12 * np.abs(g).max())
