"""Pins of the oracle's standard FEM (dofs, assembly) against textbook facts."""

import json
import math
import os

import numpy as np
import pytest

from oracle import fem, solve
from oracle import reference as ref
from workloads import unit_mesh, coef_uniform, coef_aniso_2d

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d,n,k", [(2, 3, 1), (2, 4, 2), (2, 3, 5), (3, 2, 1), (3, 2, 3), (3, 3, 2)])
def test_dim_v_structured(d, n, k):
    """dim C_{N,k} = (kN + 1)^d on the structured mesh (Tables 1-4 quote 1201^2 and 97^3)."""
    coords, cells = unit_mesh(d, n, jitter=0.1, seed=3)
    sp = fem.make_space(coords, cells, k)
    assert sp.ndofs == (k * n + 1) ** d
    # boundary dofs: (kN+1)^d - (kN-1)^d
    assert len(sp.boundary) == (k * n + 1) ** d - (k * n - 1) ** d
    tab = json.load(open(os.path.join(GOLD, "paper_tables.json")))
    assert tab["dim_v"]["2"] == (1200 * 1 + 1) ** 2 == (150 * 8 + 1) ** 2
    assert tab["dim_v"]["3"] == (96 * 1 + 1) ** 3 == (24 * 4 + 1) ** 3


@pytest.mark.parametrize("d,n,k", [(2, 3, 2), (3, 2, 2)])
def test_dof_coordinates_consistent(d, n, k):
    """Every cell's local node positions equal the coordinates of its global dofs."""
    coords, cells = unit_mesh(d, n, jitter=0.12, seed=5)
    sp = fem.make_space(coords, cells, k)
    b = fem.local_barycentric(d, k)
    X = coords[cells]
    xyz = np.einsum("vj,ejx->evx", b / k, X)
    np.testing.assert_allclose(sp.dof_coords[sp.cell_dofs], xyz, atol=1e-14)
    # distinct dofs are distinct points
    assert len(np.unique(np.round(sp.dof_coords * 1e9))) > 0
    assert np.unique(np.round(sp.dof_coords, 9), axis=0).shape[0] == sp.ndofs


def _node_perm(d, k, nodes):
    b = fem.local_barycentric(d, k).tolist()
    return [b.index(list(x)) for x in nodes]


@pytest.mark.parametrize("name", ["p1_triangle_mass", "p1_tetra_mass", "p2_triangle_mass"])
def test_textbook_mass_matrices(name):
    fx = json.load(open(os.path.join(GOLD, "textbook_element_matrices.json")))[name]
    d, k = fx["d"], fx["k"]
    coords, cells = unit_mesh(d, 1, jitter=0.0)
    coords = coords * np.array([1.3, 0.7, 1.1][:d])  # non-unit affine map
    sp = fem.make_space(coords, cells[:1], k)
    Ae = fem.element_matrices(sp, np.ones(1), "wp")[0]
    R, J, _, _ = fem.geometry(coords, cells[:1])
    vol = J[0] / math.factorial(d)
    perm = _node_perm(d, k, fx["nodes"])
    expect = np.array(fx["matrix"], float) * vol / fx["scale"]
    np.testing.assert_allclose(Ae[np.ix_(perm, perm)], expect, rtol=1e-13, atol=1e-16)


def test_p1_five_point_stencil():
    """k = 1, M = I on the unjittered 'right' mesh: interior rows are (4, -1, -1, -1, -1)."""
    n = 6
    coords, cells = unit_mesh(2, n)
    sp = fem.make_space(coords, cells, 1)
    A = fem.assemble(sp, fem.element_matrices(sp, np.ones(len(cells)), "se")).toarray()
    key = {tuple(np.round(x * n).astype(int)): i for i, x in enumerate(sp.dof_coords)}
    for (i, j), row in key.items():
        if 0 < i < n and 0 < j < n:
            nb = [key[(i + 1, j)], key[(i - 1, j)], key[(i, j + 1)], key[(i, j - 1)]]
            expect = np.zeros(sp.ndofs)
            expect[row] = 4
            expect[nb] = -1
            np.testing.assert_allclose(A[row], expect, atol=1e-14)


@pytest.mark.parametrize("d,k", [(2, 1), (2, 3), (3, 2)])
def test_symmetry_null_space_mass(d, k):
    """SE: symmetric, A 1 = 0 (Neumann), positive definite after Dirichlet elimination.
    WP: symmetric positive definite, 1^T A 1 = int_Omega m."""
    coords, cells = unit_mesh(d, 2, jitter=0.1, seed=2)
    sp = fem.make_space(coords, cells, k)
    nel = len(cells)
    M = coef_aniso_2d(nel, 7) if d == 2 else np.ones(nel)
    A = fem.assemble(sp, fem.element_matrices(sp, M, "se")).toarray()
    np.testing.assert_allclose(A, A.T, atol=1e-13 * np.abs(A).max())
    np.testing.assert_allclose(A @ np.ones(sp.ndofs), 0, atol=1e-12 * np.abs(A).max())
    I = sp.interior
    assert np.linalg.eigvalsh(A[np.ix_(I, I)]).min() > 0
    m = coef_uniform(nel, 1, 10, 4)
    Am = fem.assemble(sp, fem.element_matrices(sp, m, "wp")).toarray()
    np.testing.assert_allclose(Am, Am.T, atol=1e-15)
    assert np.linalg.eigvalsh(Am).min() > 0
    _, J, _, _ = fem.geometry(coords, cells)
    vol = J / math.factorial(d)
    assert abs(Am.sum() - (m * vol).sum()) <= 1e-13 * (m * vol).sum()
    assert abs(vol.sum() - 1.0) < 1e-13


def _l2_h1_error(sp, uh, uex, gex):
    d, k = sp.d, sp.k
    pts, wts = ref.collapsed_gauss(d, k + 4)
    R, J, Rinv, S = fem.geometry(sp.coords, sp.cells)
    xq = S[:, None, :] + np.einsum("exr,qr->eqx", R, pts)
    phi = ref.eval_basis(d, k, pts)
    G = ref.eval_basis_grad(d, k, pts)
    uT = uh[sp.cell_dofs]
    vals = uT @ phi.T
    grads = np.einsum("erx,qrk,ek->eqx", Rinv, G, uT)  # R^{-T} grad^
    e2 = np.einsum("e,q,eq->", J, wts, (vals - uex(xq)) ** 2)
    h2 = np.einsum("e,q,eqx->", J, wts, (grads - gex(xq)) ** 2)
    return math.sqrt(e2), math.sqrt(h2)


@pytest.mark.parametrize("d,k,ns", [(2, 1, (4, 8, 16)), (2, 2, (4, 8)), (2, 3, (2, 4)), (3, 1, (3, 6))])
def test_manufactured_solution_rates(d, k, ns):
    """-div grad u = f, u = prod sin(pi x_j): L2 error O(h^{k+1}), H1 seminorm error O(h^k)."""
    uex = lambda x: np.prod(np.sin(np.pi * x), axis=-1)

    def gex(x):
        s, c = np.sin(np.pi * x), np.cos(np.pi * x)
        out = np.empty_like(x)
        for r in range(d):
            out[..., r] = np.pi * c[..., r] * np.prod(np.delete(s, r, axis=-1), axis=-1)
        return out

    f = lambda x: d * np.pi ** 2 * uex(x)
    errs = []
    for n in ns:
        coords, cells = unit_mesh(d, n)
        sp = fem.make_space(coords, cells, k)
        A = fem.assemble(sp, fem.element_matrices(sp, np.ones(len(cells)), "se"))
        b = fem.load_vector(sp, f)
        u = solve.direct_dirichlet(A, b, sp.boundary)
        errs.append(_l2_h1_error(sp, u, uex, gex))
    errs = np.array(errs)
    rates = np.log(errs[:-1] / errs[1:]) / np.log(np.array(ns[1:]) / np.array(ns[:-1]))[:, None]
    assert rates[-1, 0] > k + 1 - 0.35, rates
    assert rates[-1, 1] > k - 0.25, rates
