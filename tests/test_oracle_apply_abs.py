"""Pins of the oracle's componentwise rounding scale |B^|^T |D| |B^| |u| (``dogip.apply_abs``).

Every componentwise parity check of the GPU applies (FP64 to 1e-12 of this scale, FP32
within 2 gamma_m of it, the multigrid residual rows) takes its bound from this
function, so it is fixed here against facts that do not come from it:

* where B^, D and u have no negative entry (projection, P1 in 2D: the P1 basis at the
  P2 nodes is 0, 1/2 or 1, and the 2D weights of the P2 basis are 0 and 1/3), the scale
  is the operator itself, so it equals the quadrature-assembled matrix times u;
* the triangle inequality: it bounds |A u| from above and sum_T |A_T| |u_T| (element
  matrices of the standard assembly) from below;
* on the reference simplex with an isotropic coefficient, P1 elliptic, it is the
  absolute value of the textbook P1 stiffness matrix (each entry is one product,
  so nothing cancels);
* Dirichlet rows: a vector living on the boundary only gives zero interior rows and
  |u_B| on the boundary rows.
(Algorithm 1 and Theorems 2 and 4 define the operator whose rounding this bounds.)
"""

import json
import os

import numpy as np
import pytest

from oracle import dogip, fem
from oracle import reference as ref
from workloads import coef_aniso_3d, coef_uniform, random_vector, unit_mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_equals_operator_when_nothing_is_negative():
    """2D P1 projection, m > 0, u >= 0: apply_abs(u) = A u with A the assembled matrix."""
    d, k = 2, 1
    assert ref.bhat(d, k, "wp").min() >= 0.0
    assert ref.what(d, 2 * k).min() >= 0.0
    coords, cells = unit_mesh(d, 7, jitter=0.12, seed=4)
    sp = fem.make_space(coords, cells, k)
    m = coef_uniform(len(cells), 1.0, 100.0, 4)
    A = fem.assemble(sp, fem.element_matrices(sp, m, "wp"))
    assert A.data.min() >= 0.0
    D = dogip.build_d(sp, m, "wp")
    u = np.abs(random_vector(sp.ndofs, 4))
    got = dogip.apply_abs(sp, D, u, "wp", False)
    expect = A @ u
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=0.0)
    # and the signed operator gives the same numbers bit for bit (same products, no sign)
    np.testing.assert_array_equal(got, dogip.apply(sp, D, u, "wp"))


@pytest.mark.parametrize("d,n,k", [(3, 2, 3), (2, 4, 4)])
def test_triangle_inequality_bounds(d, n, k):
    """Signed random u, anisotropic tensors on a jittered mesh (elliptic, Dirichlet):
    sum_T |A_T| |u_T|  <=  apply_abs(u)  and  |A u| <= apply_abs(u), row by row."""
    coords, cells = unit_mesh(d, n, jitter=0.12, seed=7)
    sp = fem.make_space(coords, cells, k)
    nel = len(cells)
    c = coef_aniso_3d(nel, 7) if d == 3 else fem.unpack_sym(
        np.stack([np.full(nel, 3.0), np.full(nel, 0.8), np.full(nel, 1.5)], 1), 2)
    D = dogip.build_d(sp, c, "se")
    u = random_vector(sp.ndofs, 9)
    ab = dogip.apply_abs(sp, D, u, "se", True)
    y = dogip.apply_dirichlet(sp, D, u, "se")
    slack = 1e-12 * ab.max()
    assert np.all(np.abs(y) <= ab + slack)
    # lower bound from the element matrices of the standard quadrature assembly
    Ae = fem.element_matrices(sp, c, "se")
    ua = np.abs(u)
    ua[sp.boundary] = 0.0
    cd = sp.cell_dofs
    yT = np.einsum("ekl,el->ek", np.abs(Ae), ua[cd])
    low = np.bincount(cd.reshape(-1), weights=yT.reshape(-1), minlength=sp.ndofs)
    inner = sp.interior
    assert np.all(low[inner] <= ab[inner] + slack)
    # the bound is not vacuous: it exceeds |A u| somewhere by more than rounding
    assert np.max(ab[inner] - np.abs(y[inner])) > 1e-3 * ab.max()


@pytest.mark.parametrize("d,name", [(2, "p1_ref_triangle_stiffness"), (3, "p1_ref_tetra_stiffness")])
def test_reference_simplex_p1_is_abs_stiffness(d, name):
    """One reference simplex, P1 elliptic, a = 3: the columns of apply_abs are those of
    a |K| with K the textbook P1 stiffness of the reference simplex."""
    fx = json.load(open(os.path.join(GOLD, "textbook_element_matrices.json")))[name]
    coords = np.vstack([np.zeros(d), np.eye(d)])
    cells = np.arange(d + 1, dtype=np.int32)[None, :]
    sp = fem.make_space(coords, cells, 1)
    # dofs are the vertices; order them as the fixture (0, e_1, ..., e_d)
    perm = [int(np.argmin(np.linalg.norm(sp.dof_coords - x, axis=1))) for x in coords]
    a = 3.0
    D = dogip.build_d(sp, np.array([a]), "se")
    cols = np.stack([dogip.apply_abs(sp, D, e, "se", False) for e in np.eye(sp.ndofs)], axis=1)
    expect = a * np.abs(np.array(fx["matrix"], float)) / fx["scale"]
    np.testing.assert_allclose(cols[np.ix_(perm, perm)], expect, rtol=1e-14, atol=1e-15)
    # the signed operator is the stiffness itself (the same cell, the same D)
    sgn = np.stack([dogip.apply(sp, D, e, "se") for e in np.eye(sp.ndofs)], axis=1)
    np.testing.assert_allclose(sgn[np.ix_(perm, perm)], a * np.array(fx["matrix"], float) / fx["scale"],
                               rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2)])
def test_boundary_only_vector(d, k):
    """u = 0 on the interior: interior rows of the scale are exactly 0 (boundary columns
    drop out), and Dirichlet rows equal |u_B|."""
    coords, cells = unit_mesh(d, 3, jitter=0.1, seed=2)
    sp = fem.make_space(coords, cells, k)
    D = dogip.build_d(sp, coef_uniform(len(cells), 1.0, 10.0, 2), "se")
    u = np.zeros(sp.ndofs)
    u[sp.boundary] = random_vector(len(sp.boundary), 3)
    ab = dogip.apply_abs(sp, D, u, "se", True)
    assert np.all(ab[sp.interior] == 0.0)
    np.testing.assert_array_equal(ab[sp.boundary], np.abs(u[sp.boundary]))
    # without the Dirichlet mask the boundary values do reach interior rows
    assert np.abs(dogip.apply_abs(sp, D, u, "se", False)[sp.interior]).max() > 0.0
