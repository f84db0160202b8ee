"""Pins of the factored elliptic B^ (oracle): B^_r = B2 B1_r exactly, the factors' sparsity,
and the rounding scale apply_abs_factored.

* The identity is exact: the gradient of a P_k function is a P_{k-1} vector field, which
  P_{k-1} interpolation at the W nodes reproduces (Theorem 4's B^ is that gradient at the
  W nodes).  Checked in rational arithmetic against the oracle's B^ for every order the
  factored kernels cover, and for k = 1 (both lattices the centroid, B2 = [[1]]).
* apply_abs_factored equals apply_abs at k = 1 (the factors are B^ itself), dominates it
  for k >= 2 (|B2 B1| <= |B2||B1| entrywise), and equals a brute-force evaluation of its
  formula on one cell in rational arithmetic."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import dogip as odg
from oracle import fem
from oracle import reference as ref
from workloads import coef_aniso_3d, random_vector, unit_mesh


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (3, 1), (3, 2), (3, 3)])
def test_factors_reproduce_bhat_exactly(d, k):
    b1, b2 = ref.bhat_factors_exact(d, k)
    bh = ref.bhat_exact(d, k, "se")
    nj = len(b2[0])
    assert nj == ref.dim_p(d, k - 1) and len(b2) == ref.dim_p(d, 2 * k - 2)
    for r in range(d):
        for i in range(len(b2)):
            for l in range(ref.dim_p(d, k)):
                assert sum((b2[i][j] * b1[r][j][l] for j in range(nj)), Fraction(0)) == bh[r][i][l]


def test_factor_sparsity_3d_p3_and_2d_p5():
    """The multiply-add counts quoted for the factored kernels: nonzeros of B1 (and how many
    are +-1), of B2 outside its unit rows (W nodes on the P_{k-1} lattice), unit rows."""
    def cost(d, k):
        b1, b2 = ref.bhat_factors_exact(d, k)
        n1 = sum(1 for blk in b1 for row in blk for v in row if v != 0)
        pm1 = sum(1 for blk in b1 for row in blk for v in row if v in (1, -1))
        unit = sum(1 for row in b2 if sum(1 for v in row if v != 0) == 1 and max(row) == 1)
        n2 = sum(1 for row in b2 for v in row if v != 0) - unit
        return n1, pm1, n2, unit

    assert cost(3, 3) == (216, 36, 106, 10)
    assert cost(2, 5) == (436, 20, 255, 15)
    assert ref.nnz_counts(3, 3, "se") == (1014, 90)


def _case(d, n, k, seed):
    coords, cells = unit_mesh(d, n, jitter=0.1, seed=seed)
    sp = fem.make_space(coords, cells, k)
    a = coef_aniso_3d(len(cells), seed) if d == 3 else None
    if d == 2:
        rng = np.random.default_rng(seed)
        a = np.stack([rng.uniform(1, 3, len(cells)), rng.uniform(-0.5, 0.5, len(cells)), rng.uniform(1, 3, len(cells))], 1)
    D = odg.build_d(sp, fem.unpack_sym(a, d), "se")
    return sp, D


@pytest.mark.parametrize("d,n", [(2, 4), (3, 2)])
def test_abs_factored_equals_abs_at_k1(d, n):
    sp, D = _case(d, n, 1, 3)
    u = random_vector(sp.ndofs, seed=4)
    np.testing.assert_allclose(odg.apply_abs_factored(sp, D, u, True), odg.apply_abs(sp, D, u, "se", True),
                               rtol=1e-14, atol=0)


@pytest.mark.parametrize("d,n,k", [(2, 4, 3), (2, 3, 5), (3, 2, 2), (3, 2, 3)])
def test_abs_factored_dominates_abs(d, n, k):
    sp, D = _case(d, n, k, 5)
    u = random_vector(sp.ndofs, seed=6)
    a = odg.apply_abs(sp, D, u, "se", True)
    f = odg.apply_abs_factored(sp, D, u, True)
    assert np.all(f >= a * (1 - 1e-14))
    assert np.max(f / np.maximum(a, 1e-300)) > 1.01  # the factored scale is larger somewhere
    assert np.all(np.abs(odg.apply_dirichlet(sp, D, u, "se")) <= f * (1 + 1e-14))


def test_abs_factored_brute_force_one_cell():
    """One 3D P2 cell, every product written out in rationals from the exact factors."""
    coords, cells = unit_mesh(3, 1, jitter=0.0, seed=0)
    sp = fem.make_space(coords, cells[:1], 2)
    D = odg.build_d(sp, fem.unpack_sym(np.array([[2.0, 0.3, -0.2, 1.5, 0.1, 1.0]]), 3), "se")
    u = random_vector(sp.ndofs, seed=9)
    b1, b2 = ref.bhat_factors_exact(3, 2)
    uT = [abs(Fraction(float(u[g]))) for g in sp.cell_dofs[0]]
    nj, wt = len(b2[0]), len(b2)
    G = [[sum((abs(b1[r][j][l]) * uT[l] for l in range(len(uT))), Fraction(0)) for j in range(nj)] for r in range(3)]
    g = [[sum((abs(b2[i][j]) * G[r][j] for j in range(nj)), Fraction(0)) for r in range(3)] for i in range(wt)]
    Dc = D[0]
    h = [[sum((abs(Fraction(float(Dc[i, r, s]))) * g[i][s] for s in range(3)), Fraction(0)) for r in range(3)]
         for i in range(wt)]
    H = [[sum((abs(b2[i][j]) * h[i][r] for i in range(wt)), Fraction(0)) for j in range(nj)] for r in range(3)]
    y = [sum((abs(b1[r][j][l]) * H[r][j] for r in range(3) for j in range(nj)), Fraction(0)) for l in range(len(uT))]
    expect = np.zeros(sp.ndofs)
    for l, gdof in enumerate(sp.cell_dofs[0]):
        expect[gdof] += float(y[l])
    np.testing.assert_allclose(odg.apply_abs_factored(sp, D, u, False), expect, rtol=1e-13, atol=0)
