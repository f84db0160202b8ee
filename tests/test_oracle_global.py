"""Pins of the oracle's global weighted-projection DoGIP (Theorem 1)."""

import math

import numpy as np
import pytest

from oracle import dogip, fem, global_wp
from oracle import reference as ref
from workloads import coef_uniform, unit_mesh

CASES = [(2, 3, k) for k in (1, 2, 3, 4)] + [(3, 2, k) for k in (1, 2)] + [(3, 1, 3)]


def _setup(d, n, k, seed, jitter=0.15):
    coords, cells = unit_mesh(d, n, jitter=jitter, seed=seed)
    sp = fem.make_space(coords, cells, k)
    return sp, global_wp.w_space(sp), len(cells)


@pytest.mark.parametrize("d,n,k", CASES)
def test_theorem1_equals_assembled_matrix(d, n, k):
    """B^T A^DoGIP B = A (eq. linsys_gp, quadrature-assembled) to 1e-12 relative."""
    sp, wsp, nel = _setup(d, n, k, seed=20 + k)
    m = coef_uniform(nel, 1, 100, 4)
    A = fem.assemble(sp, fem.element_matrices(sp, m, "wp")).toarray()
    B = global_wp.interpolation_matrix(sp, wsp)
    Dg = global_wp.build_d_global(sp, wsp, m)
    Ag = (B.T @ (Dg[:, None] * B.toarray()))
    assert np.linalg.norm(Ag - A) <= 1e-12 * np.linalg.norm(A)
    u = np.random.default_rng(1).uniform(-1, 1, sp.ndofs)
    assert np.allclose(global_wp.apply_global(sp, wsp, Dg, u, B), A @ u, rtol=0, atol=1e-12 * np.abs(A).sum())


@pytest.mark.parametrize("d,n,k", CASES)
def test_interpolation_of_linear_functions(d, n, k):
    """B interpolates: for u the nodal values of p(x) = a + b.x (in every C_{N,k}),
    B u equals p at the W nodes."""
    sp, wsp, _ = _setup(d, n, k, seed=3)
    a, b = 0.7, np.arange(1, d + 1) * 0.37
    u = a + sp.dof_coords @ b
    w = global_wp.interpolation_matrix(sp, wsp) @ u
    assert np.abs(w - (a + wsp.dof_coords @ b)).max() <= 1e-13


@pytest.mark.parametrize("d,n,k", [(2, 4, 1), (2, 3, 3), (2, 2, 5), (3, 2, 1), (3, 2, 2)])
def test_global_dimension_closed_form(d, n, k):
    """dim C_{N,2k} = (2kN + 1)^d on the unit meshes, below the element-wise count sum_T W_T."""
    sp, wsp, nel = _setup(d, n, k, seed=0, jitter=0.0)
    assert wsp.ndofs == (2 * k * n + 1) ** d
    assert wsp.ndofs < nel * ref.dim_p(d, 2 * k)


def test_global_weights_integrate_the_coefficient():
    """sum_j A^DoGIP_jj = int m, and for m = 1 with k = 1 (W = P2): the vertex
    entries vanish (P2 vertex functions integrate to zero) and an edge entry is
    |T|/3 summed over the cells holding the edge."""
    sp, wsp, nel = _setup(2, 4, 1, seed=1, jitter=0.1)
    m = coef_uniform(nel, 1, 10, 2)
    R, J, _, _ = fem.geometry(sp.coords, sp.cells)
    vol = J / 2
    assert math.isclose(global_wp.build_d_global(sp, wsp, m).sum(), float((m * vol).sum()), rel_tol=1e-13)
    Dg = global_wp.build_d_global(sp, wsp, np.ones(nel))
    vert = np.zeros(wsp.ndofs, bool)
    vert[wsp.cell_dofs[:, [0, 2, 5]].reshape(-1)] = True  # lattice order of P2: (0,0),(0,1),(0,2),(1,0),(1,1),(2,0)
    assert np.abs(Dg[vert]).max() <= 1e-15
    edge_sum = np.bincount(wsp.cell_dofs[:, [1, 3, 4]].reshape(-1), weights=np.repeat(vol / 3, 3),
                           minlength=wsp.ndofs)
    assert np.allclose(Dg[~vert], edge_sum[~vert], rtol=1e-14, atol=0)


def test_same_operator_as_elementwise():
    """Theorems 1 and 2 give the same operator (the element-wise form splits each
    shared W dof's integral over its cells)."""
    sp, wsp, nel = _setup(3, 2, 2, seed=9)
    m = coef_uniform(nel, 1, 100, 5)
    u = np.random.default_rng(2).uniform(-1, 1, sp.ndofs)
    y1 = global_wp.apply_global(sp, wsp, global_wp.build_d_global(sp, wsp, m), u)
    y2 = dogip.apply(sp, dogip.build_d(sp, m, "wp"), u, "wp")
    assert np.linalg.norm(y1 - y2) <= 1e-13 * np.linalg.norm(y2)
