"""Pins of the oracle's sub-cell quadrature D for a coefficient with jumps inside cells."""

import itertools
import math

import numpy as np
import pytest

from oracle import dogip, fem, subcell
from oracle import reference as ref
from workloads import unit_mesh


@pytest.mark.parametrize("d", [2, 3])
def test_red_refinement_tiles_the_parent(d):
    """The children of a red refinement have equal volumes summing to the parent's, and
    their vertices are the parent's vertices and edge midpoints."""
    rng = np.random.default_rng(0)
    v = rng.uniform(-1, 1, size=(d + 1, d))
    vol = lambda s: abs(np.linalg.det((s[1:] - s[0]).T)) / math.factorial(d)  # noqa: E731
    ch = subcell.red_children(v)
    assert len(ch) == 2 ** d
    assert np.allclose([vol(c) for c in ch], vol(v) / 2 ** d, rtol=1e-12)
    allowed = [v[i] for i in range(d + 1)] + [(v[i] + v[j]) / 2 for i in range(d + 1) for j in range(i + 1, d + 1)]
    for c in ch:
        for p in c:
            assert min(np.abs(p - a).max() for a in allowed) < 1e-15


@pytest.mark.parametrize("d,k,kind", [(2, 2, "se"), (2, 2, "wp"), (3, 2, "se"), (3, 1, "wp")])
def test_uncut_cells_match_the_closed_form(d, k, kind):
    """A ball covering the whole domain (a = a_in everywhere) and a ball far away
    (a = a_out everywhere) give Theorem 4 / 2 with a constant coefficient."""
    coords, cells = unit_mesh(d, 2, jitter=0.1, seed=3)
    sp = fem.make_space(coords, cells, k)
    nel = len(cells)
    big = np.array([[0.5] * d + [10.0]])
    far = np.array([[50.0] * d + [1.0]])
    for balls, a in ((big, 7.0), (far, 3.0)):
        D = subcell.build_d_subcell(sp, balls, 7.0, 3.0, kind, depth=2, ng=3)
        D0 = dogip.build_d(sp, np.full(nel, a), kind)
        assert np.abs(D - D0).max() <= 1e-13 * np.abs(D0).max()


@pytest.mark.parametrize("d", [2, 3])
def test_total_integral_converges_to_the_ball_volume(d):
    """sum_{T,i} int_T a phi^W_i = int_Omega a = a_out + (a_in - a_out) |B| for a ball
    inside the unit domain; the error stays within |a_in - a_out| times the volume of
    the cut leaves and shrinks with the depth."""
    coords, cells = unit_mesh(d, 2 if d == 2 else 1, jitter=0.0)
    sp = fem.make_space(coords, cells, 1)
    c, r = np.array([0.45, 0.55, 0.5][:d]), 0.3
    exact_ball = math.pi * r ** 2 if d == 2 else 4.0 / 3.0 * math.pi * r ** 3
    a_in, a_out = 5.0, 1.0
    errs = []
    for depth in (1, 2, 3, 4) if d == 2 else (1, 2, 3):
        D = subcell.build_d_subcell(sp, np.array([[*c, r]]), a_in, a_out, "wp", depth=depth, ng=2)
        total = D.sum()
        err = abs(total - (a_out * 1.0 + (a_in - a_out) * exact_ball))
        # bound: cut leaves at this depth, each of volume |T| / 2^(d depth)
        cut = 0.0
        for e in range(len(cells)):
            X = coords[cells[e]]
            R = (X[1:] - X[0]).T
            J = abs(np.linalg.det(R))

            def count(v, level):
                cls = subcell.classify(X[0] + v @ R.T, np.array([[*c, r]]))
                if cls != 2:
                    return 0.0
                if level == depth:
                    return J * abs(np.linalg.det((v[1:] - v[0]).T)) / math.factorial(d)
                return sum(count(ch, level + 1) for ch in subcell.red_children(v))

            cut += count(np.vstack([np.zeros(d), np.eye(d)]), 0)
        assert err <= (a_in - a_out) * cut + 1e-12
        errs.append(err)
    assert errs[-1] < errs[0] / 3


def test_leaf_rule_is_exact_for_the_w_basis_on_inside_cells():
    """On a sub-simplex wholly inside a ball the mapped rule integrates phi^W exactly:
    a ball containing the cell reproduces w^_i |T^| per node."""
    d, q = 3, 4
    X = np.vstack([np.zeros(d), np.eye(d)]) * 0.1
    s, _ = subcell.subcell_integrals(X, np.array([[0.0, 0.0, 0.0, 5.0]]), q, depth=2, ng=(q + d + 2) // 2)
    assert np.abs(s - ref.what(d, q) / math.factorial(d)).max() <= 1e-15


def _cut_leaf_volume(X, balls, depth):
    """Reference-cell volume of the cut sub-simplices at the last level."""
    d = X.shape[1]
    R = (X[1:] - X[0]).T

    def count(v, level):
        cls = subcell.classify(X[0] + v @ R.T, balls)
        if cls != 2:
            return 0.0
        if level == depth:
            return abs(np.linalg.det((v[1:] - v[0]).T)) / math.factorial(d)
        return sum(count(ch, level + 1) for ch in subcell.red_children(v))

    return count(np.vstack([np.zeros(d), np.eye(d)]), 0)


def _ball_orthant_moment(alpha, r):
    """int over {x >= 0, |x| < r} of x^alpha: r^(|a|+n)/(|a|+n) * 2^(1-n) prod Gamma((a_i+1)/2) / Gamma((|a|+n)/2)
    (polar coordinates; the sphere part is the orthant share of the Dirichlet integral)."""
    n, s = len(alpha), sum(alpha)
    g = math.prod(math.gamma((a + 1) / 2) for a in alpha) / math.gamma((s + n) / 2)
    return r ** (s + n) / (s + n) * 2.0 ** (1 - n) * g


def _ball_moment(alpha, c, r):
    """int over the full ball |x - c| < r of x^alpha, expanding (c + y)^alpha; odd powers of
    y integrate to zero, even ones are 2^n times the orthant moment."""
    n = len(alpha)
    total = 0.0
    for beta in itertools.product(*[range(a + 1) for a in alpha]):
        if any(b % 2 for b in beta):
            continue
        coef = math.prod(math.comb(a, b) * ci ** (a - b) for a, b, ci in zip(alpha, beta, c))
        total += coef * 2.0 ** n * _ball_orthant_moment(beta, r)
    return total


@pytest.mark.parametrize("d,q", [(2, 4), (3, 4), (2, 2)])
@pytest.mark.parametrize("where", ["vertex", "inside"])
def test_cut_cell_node_integrals_reproduce_exact_moments(d, q, where):
    """One cut cell, the reference simplex, against exact values that do not use the
    oracle's basis: the W basis reproduces polynomials of degree <= q, so
    sum_i I_i x_i^alpha = int_T 1_B x^alpha for every |alpha| <= q, and these W_T moments
    determine the node integrals I_i.  The exact moments are closed forms: a ball centred
    at the vertex 0 whose sphere stays inside T (T cut to the orthant sector of the ball),
    and a ball inside T around the incentre (T cut to the whole ball).  The oracle's error
    is bounded by twice the volume of the cut leaves (|x^alpha| <= 1 on T, positive
    weights) and shrinks with the depth."""
    X = np.vstack([np.zeros(d), np.eye(d)])
    if where == "vertex":
        r = 0.5  # < 1/sqrt(d): the far facet x_1 + .. + x_d = 1 is not reached
        balls = np.array([[0.0] * d + [r]])
        exact = {a: _ball_orthant_moment(a, r) for a in ref.multi_indices(d, q)}
    else:
        rin = 1.0 / (d + math.sqrt(d))  # inradius of the reference simplex, incentre (rin, .., rin)
        c, r = np.full(d, rin), 0.8 * rin
        balls = np.array([[*c, r]])
        exact = {a: _ball_moment(a, c, r) for a in ref.multi_indices(d, q)}
    nodes = np.array(ref.lattice(d, q), dtype=np.float64)
    ng = (q + d + 1) // 2 + 1  # 2 ng - d >= q: exact on inside leaves
    errs = []
    for depth in ((2, 4, 6) if d == 2 else (2, 3, 4)):
        s, _ = subcell.subcell_integrals(X, balls, q, depth, ng)
        bound = 2.0 * _cut_leaf_volume(X, balls, depth) + 1e-14
        worst = 0.0
        for a, m in exact.items():
            mom = float(s @ np.prod(nodes ** np.array(a), axis=1))
            assert abs(mom - m) <= bound, (depth, a, mom, m, bound)
            worst = max(worst, abs(mom - m))
        errs.append(worst)
    assert errs[-1] < errs[0] / 3
