"""Reference-element quantities of the element-wise DoGIP (oracle, test infrastructure).

Everything here is computed in exact rational arithmetic (``fractions.Fraction``)
and converted to float64 once at the end.

* Reference simplex T^ = conv{0, e_1, ..., e_d}, |T^| = 1/d!  (Section 2.1).
* Lagrange nodes of P_p: the equispaced lattice a/p, |a| <= p.  A space of
  order 0 (the discontinuous double-grid space D_{N,0} of the elliptic problem
  at k = 1) has one node, the centroid.
* Nodal basis: coefficients in the monomial basis from the exact inverse of the
  Vandermonde matrix, so that phi_l(x_j) = delta_lj (Dirac delta property,
  Section 2.1).
* B^ for the weighted projection (Theorem 2): B^_jl = phi^_l(x^_W^j), with
  W = C_{N,2k}.
* B^ for the elliptic problem (Theorem 4): B^_rik = d phi^_k / d x^_r at
  x^_W^i, with W = D_{N,2k-2}.  The derivative is taken with respect to the
  reference coordinate: the inverse Jacobians sit in D (reading of the
  theorem's formula, which writes d/dx_r, against its proof).
* w^_i = (1/|T^|) int_T^ phi^W_i: the weights of the closed Newton-Cotes rule on
  the W lattice, obtained from the moment equations
  sum_i x_i^alpha w_i = (1/|T^|) int_T^ x^alpha for all |alpha| <= q,
  with int_T^ x^alpha = prod_r alpha_r! / (|alpha| + d)!.

* Factored elliptic B^ (Section 4's outlook: a cheaper interpolation-projection operator):
  the gradient of a P_k function is a vector field of degree k-1, so it is fixed by its
  values at the P_{k-1} lattice and reproduced at the W nodes by P_{k-1} interpolation:
  B^_r = B2 B1_r with B1_rjl = d phi^_l / d x^_r (x^_{k-1, j}) and B2_ij = phi^{k-1}_j(x^_W^i).

Pins (tests/test_oracle_reference.py): nnz B^ and the count of entries equal to
+-1 for every row of Tables 1-4; closed Newton-Cotes weights of the P2 triangle
and tetrahedron; sum of weights; partition of unity; the collapsed Gauss rule
against the exact monomial integrals.
"""

from __future__ import annotations

import itertools
import math
from fractions import Fraction
from functools import lru_cache

import numpy as np

__all__ = [
    "multi_indices",
    "lattice",
    "dim_p",
    "w_order",
    "basis_coefficients",
    "bhat_exact",
    "bhat",
    "bhat_factors_exact",
    "bhat_factors",
    "what_exact",
    "what",
    "nnz_counts",
    "monomial_integral",
    "collapsed_gauss",
    "eval_basis",
    "eval_basis_grad",
]


def multi_indices(d: int, p: int):
    """All alpha in N^d with |alpha| <= p, in lexicographic order."""
    return [a for a in itertools.product(range(p + 1), repeat=d) if sum(a) <= p]


def dim_p(d: int, p: int) -> int:
    """dim P_p in d variables = C(p + d, d)."""
    return math.comb(p + d, d)


def w_order(k: int, kind: str) -> int:
    """Polynomial order q of the double-grid space: 2k (weighted projection,
    lemma of Section 2.2) or 2k - 2 (elliptic problem, lemma of Section 2.3)."""
    if kind == "wp":
        return 2 * k
    if kind == "se":
        return 2 * k - 2
    raise ValueError(kind)


@lru_cache(maxsize=None)
def lattice(d: int, p: int):
    """Lagrange nodes of P_p on T^ as tuples of Fractions (the centroid for p = 0)."""
    if p == 0:
        return (tuple(Fraction(1, d + 1) for _ in range(d)),)
    return tuple(tuple(Fraction(ar, p) for ar in a) for a in multi_indices(d, p))


def _mono(x, alpha):
    v = Fraction(1)
    for xr, ar in zip(x, alpha):
        if ar:
            v *= xr ** ar
    return v


def _mono_grad(x, alpha, r):
    ar = alpha[r]
    if ar == 0:
        return Fraction(0)
    v = Fraction(ar)
    for s, (xs, a) in enumerate(zip(x, alpha)):
        e = a - 1 if s == r else a
        if e:
            v *= xs ** e
    return v


def _inverse(mat):
    """Exact Gauss-Jordan inverse of a square list-of-lists of Fractions."""
    n = len(mat)
    a = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(mat)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        inv = 1 / a[c][c]
        a[c] = [v * inv for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[c])]
    return [row[n:] for row in a]


def _solve(mat, rhs):
    """Exact solution of mat x = rhs (mat square, Fractions)."""
    n = len(mat)
    a = [list(row) + [rhs[i]] for i, row in enumerate(mat)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c] != 0)
        a[c], a[piv] = a[piv], a[c]
        inv = 1 / a[c][c]
        a[c] = [v * inv for v in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                f = a[r][c]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[c])]
    return [row[n] for row in a]


@lru_cache(maxsize=None)
def basis_coefficients(d: int, p: int):
    """C with phi_l(x) = sum_m C[m][l] x^alpha_m (alpha_m = multi_indices(d, p)[m]).

    C is the exact inverse of the Vandermonde matrix V[j][m] = (x_j)^alpha_m.
    """
    nodes = lattice(d, p)
    alphas = multi_indices(d, p)
    vand = [[_mono(x, a) for a in alphas] for x in nodes]
    return tuple(tuple(row) for row in _inverse(vand))


@lru_cache(maxsize=None)
def bhat_exact(d: int, k: int, kind: str):
    """Exact B^: [W_T][V_T] for 'wp', [d][W_T][V_T] for 'se' (nested tuples of Fractions)."""
    q = w_order(k, kind)
    wnodes = lattice(d, q)
    alphas = multi_indices(d, k)
    c = basis_coefficients(d, k)
    vt = len(alphas)
    if kind == "wp":
        out = []
        for x in wnodes:
            mono = [_mono(x, a) for a in alphas]
            out.append(tuple(sum((mono[m] * c[m][l] for m in range(vt)), Fraction(0)) for l in range(vt)))
        return tuple(out)
    outr = []
    for r in range(d):
        rows = []
        for x in wnodes:
            mg = [_mono_grad(x, a, r) for a in alphas]
            rows.append(tuple(sum((mg[m] * c[m][l] for m in range(vt)), Fraction(0)) for l in range(vt)))
        outr.append(tuple(rows))
    return tuple(outr)


def bhat(d: int, k: int, kind: str) -> np.ndarray:
    """B^ as float64: shape (W_T, V_T) for 'wp', (d, W_T, V_T) for 'se'."""
    b = bhat_exact(d, k, kind)
    return np.array([[[float(v) for v in row] for row in blk] for blk in b]) if kind == "se" \
        else np.array([[float(v) for v in row] for row in b])


@lru_cache(maxsize=None)
def bhat_factors_exact(d: int, k: int):
    """Exact factors of the elliptic B^: (B1 [d][P_{k-1} nodes][V_T], B2 [W_T][P_{k-1} nodes]).
    The gradient of phi^_l at the P_{k-1} lattice, and the P_{k-1} nodal basis at the W
    nodes (P_{2k-2} lattice); for k = 1 both lattices are the centroid and B2 = [[1]]."""
    p = k - 1
    jnodes = lattice(d, p)
    alphas = multi_indices(d, k)
    c = basis_coefficients(d, k)
    vt = len(alphas)
    b1 = []
    for r in range(d):
        rows = []
        for x in jnodes:
            mg = [_mono_grad(x, a, r) for a in alphas]
            rows.append(tuple(sum((mg[m] * c[m][l] for m in range(vt)), Fraction(0)) for l in range(vt)))
        b1.append(tuple(rows))
    wnodes = lattice(d, 2 * k - 2)
    if p == 0:
        b2 = tuple((Fraction(1),) for _ in wnodes)
    else:
        pa = multi_indices(d, p)
        pc = basis_coefficients(d, p)
        nj = len(pa)
        b2 = tuple(tuple(sum((_mono(x, pa[m]) * pc[m][j] for m in range(nj)), Fraction(0)) for j in range(nj))
                   for x in wnodes)
    return tuple(b1), b2


def bhat_factors(d: int, k: int):
    """The factors of bhat_factors_exact as float64 arrays (d, NJ, V_T) and (W_T, NJ)."""
    b1, b2 = bhat_factors_exact(d, k)
    return (np.array([[[float(v) for v in row] for row in blk] for blk in b1]),
            np.array([[float(v) for v in row] for row in b2]))


def _flatten(b):
    if isinstance(b, Fraction):
        yield b
    else:
        for v in b:
            yield from _flatten(v)


def nnz_counts(d: int, k: int, kind: str):
    """(nnz B^, number of entries of B^ equal to +1 or -1), counted exactly."""
    vals = list(_flatten(bhat_exact(d, k, kind)))
    nnz = sum(1 for v in vals if v != 0)
    pm1 = sum(1 for v in vals if v == 1 or v == -1)
    return nnz, pm1


def monomial_integral(alpha) -> Fraction:
    """int_T^ x^alpha dx = prod_r alpha_r! / (|alpha| + d)! over T^ = conv{0, e_1..e_d}."""
    num = 1
    for a in alpha:
        num *= math.factorial(a)
    return Fraction(num, math.factorial(sum(alpha) + len(alpha)))


@lru_cache(maxsize=None)
def what_exact(d: int, q: int):
    """w^_i = int_T^ phi^W_i / |T^| for the P_q lattice (closed Newton-Cotes weights)."""
    nodes = lattice(d, q)
    if q == 0:
        return (Fraction(1),)
    alphas = multi_indices(d, q)
    fact = math.factorial(d)
    # moment equations: sum_i (x_i)^alpha_m w_i = int x^alpha_m / |T^|
    mat = [[_mono(x, a) for x in nodes] for a in alphas]
    rhs = [monomial_integral(a) * fact for a in alphas]
    return tuple(_solve(mat, rhs))


def what(d: int, q: int) -> np.ndarray:
    return np.array([float(v) for v in what_exact(d, q)])


def collapsed_gauss(d: int, n: int):
    """Collapsed (Duffy) Gauss-Legendre rule on T^ with n points per direction.

    2D: x1 = s, x2 = t (1 - s), Jacobian (1 - s).
    3D: x1 = s, x2 = t (1 - s), x3 = v (1 - s)(1 - t), Jacobian (1 - s)^2 (1 - t).
    Exact for polynomials of total degree <= 2n - d.  Returns (points [nq, d], weights [nq]).
    """
    g, w = np.polynomial.legendre.leggauss(n)
    g = (g + 1.0) / 2.0
    w = w / 2.0
    if d == 2:
        s, t = np.meshgrid(g, g, indexing="ij")
        ws, wt = np.meshgrid(w, w, indexing="ij")
        pts = np.stack([s, t * (1 - s)], -1).reshape(-1, 2)
        wts = (ws * wt * (1 - s)).reshape(-1)
    elif d == 3:
        s, t, v = np.meshgrid(g, g, g, indexing="ij")
        ws, wt, wv = np.meshgrid(w, w, w, indexing="ij")
        pts = np.stack([s, t * (1 - s), v * (1 - s) * (1 - t)], -1).reshape(-1, 3)
        wts = (ws * wt * wv * (1 - s) ** 2 * (1 - t)).reshape(-1)
    else:
        raise ValueError(d)
    return pts, wts


def _coef_ld(d: int, p: int) -> np.ndarray:
    c = basis_coefficients(d, p)
    return np.array([[np.longdouble(str(v.numerator)) / np.longdouble(str(v.denominator)) for v in row]
                     for row in c], dtype=np.longdouble)


def eval_basis(d: int, p: int, pts: np.ndarray) -> np.ndarray:
    """phi^_l(x) at float points, shape [npts, dim P_p]; monomial sums in extended precision."""
    if p == 0:
        return np.ones((pts.shape[0], 1))
    alphas = np.array(multi_indices(d, p))
    x = pts.astype(np.longdouble)
    mono = np.prod(x[:, None, :] ** alphas[None, :, :], axis=2)
    return (mono @ _coef_ld(d, p)).astype(np.float64)


def eval_basis_grad(d: int, p: int, pts: np.ndarray) -> np.ndarray:
    """d phi^_l / d x^_r at float points, shape [npts, d, dim P_p]."""
    alphas = np.array(multi_indices(d, p))
    x = pts.astype(np.longdouble)
    c = _coef_ld(d, p)
    out = np.empty((pts.shape[0], d, alphas.shape[0]))
    for r in range(d):
        e = alphas.copy()
        e[:, r] = np.maximum(e[:, r] - 1, 0)
        mono = np.prod(x[:, None, :] ** e[None, :, :], axis=2) * alphas[None, :, r]
        out[:, r, :] = (mono @ c).astype(np.float64)
    return out
