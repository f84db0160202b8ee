"""Pins of the oracle's reference-element quantities against the paper and closed forms."""

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import reference as ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TABLES = json.load(open(os.path.join(GOLD, "paper_tables.json")))


def _rows():
    for key, kind, d in (("wp_2d", "wp", 2), ("wp_3d", "wp", 3), ("se_2d", "se", 2), ("se_3d", "se", 3)):
        for row in TABLES[key]:
            yield pytest.param(kind, d, row, id=f"{key}-k{row[1]}")


@pytest.mark.parametrize("kind,d,row", list(_rows()))
def test_nnz_bhat_matches_tables(kind, d, row):
    """nnz B^ column of Tables 1-4 (exact integers), and the dimensions behind
    the mem A^DoGIP_T and mem A_T columns."""
    n, k = row[0], row[1]
    nnz, _ = ref.nnz_counts(d, k, kind)
    assert nnz == row[6]
    vt = ref.dim_p(d, k)
    wt = ref.dim_p(d, ref.w_order(k, kind))
    assert vt * vt == row[3]
    assert (wt if kind == "wp" else d * d * wt) == row[5]
    b = ref.bhat(d, k, kind)
    assert b.shape == ((wt, vt) if kind == "wp" else (d, wt, vt))


@pytest.mark.parametrize("d,q", [(2, 2), (3, 2), (2, 4)])
def test_newton_cotes_weights(d, q):
    """w^ equals the closed Newton-Cotes weights of the fixture (by node type)."""
    rule = next(r for r in json.load(open(os.path.join(GOLD, "newton_cotes.json")))["rules"]
                if r["d"] == d and r["q"] == q)
    w = ref.what_exact(d, q)
    nodes = ref.lattice(d, q)
    for x, wi in zip(nodes, w):
        a = [int(v * q) for v in x]
        b = sorted([q - sum(a)] + a, reverse=True)
        val = next(Fraction(s) for g, s in rule["groups"] if sorted(g, reverse=True) == b)
        assert wi == val


@pytest.mark.parametrize("d,q", [(2, 0), (2, 1), (2, 2), (2, 3), (2, 6), (3, 0), (3, 2), (3, 4)])
def test_weights_sum_and_quadrature(d, q):
    """sum w^ = 1, and the collapsed Gauss rule applied to the W basis gives the same weights."""
    w = ref.what_exact(d, q)
    assert sum(w) == 1
    pts, wts = ref.collapsed_gauss(d, q + 2)
    phi = ref.eval_basis(d, q, pts)
    wq = math.factorial(d) * (wts @ phi)
    np.testing.assert_allclose(wq, np.array([float(v) for v in w]), rtol=0, atol=1e-13)


@pytest.mark.parametrize("d,n", [(2, 1), (2, 4), (3, 2), (3, 5)])
def test_collapsed_gauss_exact_on_monomials(d, n):
    pts, wts = ref.collapsed_gauss(d, n)
    for a in ref.multi_indices(d, 2 * n - d):
        exact = float(ref.monomial_integral(a))
        got = wts @ np.prod(pts ** np.array(a), axis=1)
        assert abs(got - exact) <= 1e-14 * max(1.0, exact)


@pytest.mark.parametrize("d,k", [(2, 1), (2, 3), (2, 5), (3, 1), (3, 3)])
def test_nodal_basis_delta_and_partition(d, k):
    """Dirac delta property (Section 2.1) and partition of unity."""
    nodes = np.array([[float(v) for v in x] for x in ref.lattice(d, k)])
    phi = ref.eval_basis(d, k, nodes)
    np.testing.assert_allclose(phi, np.eye(len(nodes)), atol=1e-13)
    rng = np.random.default_rng(0)
    pts = rng.dirichlet(np.ones(d + 1), size=50)[:, 1:]
    np.testing.assert_allclose(ref.eval_basis(d, k, pts).sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(ref.eval_basis_grad(d, k, pts).sum(2), 0.0, atol=1e-11)


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 4), (3, 2), (3, 3)])
def test_bhat_rows_partition_and_reproduction(d, k):
    """Rows of the WP B^ sum to 1 (constants are reproduced); rows of the SE B^ sum
    to 0; the SE B^ applied to the nodal values of x_r gives e_r (linear reproduction)."""
    bw = ref.bhat_exact(d, k, "wp")
    assert all(sum(row) == 1 for row in bw)
    bs = ref.bhat_exact(d, k, "se")
    vn = ref.lattice(d, k)
    for r in range(d):
        for row in bs[r]:
            assert sum(row) == 0
            for s in range(d):
                assert sum(c * x[s] for c, x in zip(row, vn)) == (1 if s == r else 0)


def test_bhat_wp_reproduces_quadratics_at_w_nodes():
    """B^ interpolates P_k exactly: the nodal values of x1^2 x2 on V map to its values on W."""
    d, k = 2, 3
    b = ref.bhat_exact(d, k, "wp")
    vn, wn = ref.lattice(d, k), ref.lattice(d, 2 * k)
    f = lambda x: x[0] ** 2 * x[1]
    for row, xw in zip(b, wn):
        assert sum(c * f(x) for c, x in zip(row, vn)) == f(xw)


def test_k1_elliptic_bhat_is_p1_gradient():
    """k = 1, elliptic: W = D_{N,0} (one node) and B^ holds the gradients of the P1
    hat functions: (-1, ..., -1) for the node at the origin, e_r for the node at e_r."""
    for d in (2, 3):
        b = ref.bhat(d, 1, "se")
        assert b.shape == (d, 1, d + 1)
        for l, x in enumerate(ref.lattice(d, 1)):
            xs = [int(v) for v in x]
            expect = [-1] * d if sum(xs) == 0 else xs
            np.testing.assert_array_equal(b[:, 0, l], expect)
