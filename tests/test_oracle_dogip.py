"""The oracle's DoGIP element loop against the independent quadrature-assembled FEM
(the identity B^^T D B^ = A of Theorems 2 and 4)."""

import numpy as np
import pytest

from oracle import dogip, fem, solve
from oracle import reference as ref
from workloads import unit_mesh, coef_uniform, coef_aniso_2d, coef_aniso_3d


def _setup(d, n, k, seed):
    coords, cells = unit_mesh(d, n, jitter=0.15, seed=seed)
    return fem.make_space(coords, cells, k), len(cells)


def _dense(op, n):
    return np.stack([op(e) for e in np.eye(n)], axis=1)


CASES = [(2, 3, k) for k in (1, 2, 3, 4)] + [(3, 2, k) for k in (1, 2, 3)] + [(3, 1, 4)]


@pytest.mark.parametrize("d,n,k", CASES)
@pytest.mark.parametrize("kind", ["wp", "se"])
def test_identity_piecewise_constant(d, n, k, kind):
    """B^^T D B^ = A to 1e-12 relative (Frobenius) on jittered meshes, with per-cell
    anisotropic SPD tensors (elliptic) or scalars (projection)."""
    sp, nel = _setup(d, n, k, seed=11 + k)
    if kind == "wp":
        c = coef_uniform(nel, 1, 100, 3)
    else:
        c = coef_aniso_2d(nel, 3) if d == 2 else coef_aniso_3d(nel, 3)
    A = fem.assemble(sp, fem.element_matrices(sp, c, kind)).toarray()
    D = dogip.build_d(sp, c, kind)
    Ad = _dense(lambda e: dogip.apply(sp, D, e, kind), sp.ndofs)
    assert np.linalg.norm(Ad - A) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2)])
@pytest.mark.parametrize("kind", ["wp", "se"])
def test_identity_varying_coefficient(d, k, kind):
    """Coefficient varying inside cells: D from the same quadrature rule as A (Theorems 2/4
    with the integral evaluated numerically) still reproduces A."""
    sp, nel = _setup(d, 2, k, seed=5)

    def m(x):
        s = 2.0 + np.sin(3 * x[..., 0]) * np.cos(2 * x[..., -1])
        if kind == "wp":
            return s
        t = np.zeros(x.shape[:-1] + (d, d))
        for r in range(d):
            t[..., r, r] = s * (1 + r)
        t[..., 0, 1] = t[..., 1, 0] = 0.3 * s
        return t

    A = fem.assemble(sp, fem.element_matrices(sp, m, kind, nquad=k + 4)).toarray()
    D = dogip.build_d(sp, m, kind, nquad=k + 4)
    Ad = _dense(lambda e: dogip.apply(sp, D, e, kind), sp.ndofs)
    assert np.linalg.norm(Ad - A) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("kind", ["wp", "se"])
def test_diagonal_dirichlet_and_contraction(kind):
    d, k = 2, 3
    sp, nel = _setup(d, 3, k, seed=2)
    c = coef_uniform(nel, 1, 10, 1) if kind == "wp" else coef_aniso_2d(nel, 2)
    Ae = fem.element_matrices(sp, c, kind)
    A = fem.assemble(sp, Ae)
    D = dogip.build_d(sp, c, kind)
    dirichlet = kind == "se"
    diag = dogip.diagonal(sp, D, kind, dirichlet)
    Ab = solve.dirichlet_matrix(A, sp.boundary) if dirichlet else A
    np.testing.assert_allclose(diag, Ab.diagonal(), rtol=1e-12, atol=1e-14)
    u = np.random.default_rng(0).uniform(-1, 1, sp.ndofs)
    lam = np.random.default_rng(1).uniform(-1, 1, sp.ndofs)
    if dirichlet:
        y = dogip.apply_dirichlet(sp, D, u, kind)
        np.testing.assert_allclose(y, Ab @ u, rtol=1e-12, atol=1e-12 * np.abs(y).max())
    um, lm = u.copy(), lam.copy()
    if dirichlet:
        um[sp.boundary] = 0
        lm[sp.boundary] = 0
    cd = sp.cell_dofs
    expect = np.einsum("ek,ekl,el->e", lm[cd], Ae, um[cd])
    got = dogip.energy_contraction(sp, D, u, lam, kind, dirichlet)
    np.testing.assert_allclose(got, expect, rtol=1e-11, atol=1e-13 * np.abs(expect).max())


def test_d_is_indefinite_but_operator_spd():
    """The stored D has negative entries (w^ < 0 at q >= 2 in 3D) while B^^T D B^ stays SPD."""
    sp, nel = _setup(3, 1, 2, seed=0)
    D = dogip.build_d(sp, np.ones(nel), "se")
    assert (np.einsum("eirr->ei", D) < 0).any()
    A = _dense(lambda e: dogip.apply_dirichlet(sp, D, e, "se"), sp.ndofs)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    assert ref.what(3, 2).min() < 0
