"""D for a coefficient discontinuous inside the cells, by sub-cell quadrature (oracle,
test infrastructure).

The paper argues (Sections 2 and 3.3) that DoGIP suits coefficients with jumps inside
elements: the integrals int_T M phi^W_i are computed once, with as many integration
points as the jump needs (decomposing the element into sub-elements integrated
separately, as the finite cell method does), while the apply keeps its fixed cost.
The paper does not fix the decomposition; the reading taken here:

  * coefficient a(x) = a_in inside a union of balls |x - c_j| < r_j, a_out elsewhere
    (scalar; M = a I for the elliptic problem, m = a for the projection);
  * int_T a phi^W_i = a_out |T| w^_i + (a_in - a_out) int_T 1_B phi^W_i;
  * the second integral on the reference cell: the simplex is red-refined (2D: 4
    children, corner triangles and the middle one; 3D: 8 children, four corner
    tetrahedra and the inner octahedron cut along the m02-m13 diagonal) down to
    ``depth`` levels, but only where a sub-simplex is cut: one whose vertices all
    lie in one ball is inside (balls are convex), one whose bounding sphere misses
    every ball is outside; every other one is cut;
  * an inside sub-simplex, and a cut one at the last level, is integrated with the
    collapsed Gauss rule of ``ng`` points per direction mapped onto it; the
    indicator 1_B is evaluated at each point of a cut sub-simplex (1 on inside ones);
  * D_T,i from Theorem 4 / Theorem 2 with that integral.

Pinned in tests/test_oracle_subcell.py by: cells wholly inside or outside the balls
give the closed form a |T| w^_i; the children of a red refinement tile the parent
(volumes); sum_{T,i} int_T a phi^W_i = int_Omega a converges to the exact ball
volume, within the bound |a_in - a_out| * (volume of the cut leaves); and the node
integrals of one cut cell reproduce the exact moments int_T 1_B x^alpha, |alpha| <= q
(closed forms for a ball at a vertex and a ball inside the cell), within twice the
volume of the cut leaves.
"""

from __future__ import annotations

import math

import numpy as np

from . import fem
from . import reference as ref

__all__ = ["red_children", "classify", "subcell_integrals", "build_d_subcell"]


def red_children(v: np.ndarray) -> list[np.ndarray]:
    """Red refinement of a simplex with vertex rows v [d+1, d]."""
    d = v.shape[1]
    m = {(i, j): (v[i] + v[j]) / 2 for i in range(d + 1) for j in range(i + 1, d + 1)}
    if d == 2:
        return [np.array(t) for t in ([v[0], m[0, 1], m[0, 2]], [m[0, 1], v[1], m[1, 2]],
                                      [m[0, 2], m[1, 2], v[2]], [m[0, 1], m[1, 2], m[0, 2]])]
    return [np.array(t) for t in (
        [v[0], m[0, 1], m[0, 2], m[0, 3]], [m[0, 1], v[1], m[1, 2], m[1, 3]],
        [m[0, 2], m[1, 2], v[2], m[2, 3]], [m[0, 3], m[1, 3], m[2, 3], v[3]],
        [m[0, 1], m[0, 2], m[0, 3], m[1, 3]], [m[0, 1], m[0, 2], m[1, 2], m[1, 3]],
        [m[0, 2], m[0, 3], m[1, 3], m[2, 3]], [m[0, 2], m[1, 2], m[1, 3], m[2, 3]])]


def classify(P: np.ndarray, balls: np.ndarray) -> int:
    """0 outside every ball, 1 inside one ball, 2 cut (physical vertices P [d+1, d])."""
    c, r = balls[:, :-1], balls[:, -1]
    dist = np.linalg.norm(P[None, :, :] - c[:, None, :], axis=2)  # [nballs, d+1]
    if np.any(np.all(dist < r[:, None], axis=1)):
        return 1
    g = P.mean(axis=0)
    rho = np.linalg.norm(P - g, axis=1).max()
    if np.all(np.linalg.norm(c - g, axis=1) - rho >= r):
        return 0
    return 2


def subcell_integrals(X: np.ndarray, balls: np.ndarray, q: int, depth: int, ng: int):
    """int_T^ 1_B(X_0 + R_T xhat) phi^W_i(xhat) dxhat for the W nodes of order q (reference
    cell), and the number of points evaluated.  X: the cell's vertices [d+1, d]."""
    d = X.shape[1]
    R = (X[1:] - X[0]).T
    pts, wts = ref.collapsed_gauss(d, ng)
    out = np.zeros(ref.dim_p(d, q))
    npts = 0

    def leaf(v, pointwise):
        nonlocal npts
        Rs = (v[1:] - v[0]).T
        xh = v[0] + pts @ Rs.T
        w = wts * abs(np.linalg.det(Rs))
        npts += len(w)
        if pointwise:
            xp = X[0] + xh @ R.T
            inside = (np.linalg.norm(xp[:, None, :] - balls[None, :, :-1], axis=2) < balls[None, :, -1]).any(axis=1)
            w = w * inside
        out[:] += w @ ref.eval_basis(d, q, xh)

    def walk(v, level):
        cls = classify(X[0] + v @ R.T, balls)
        if cls == 0:
            return
        if cls == 1:
            leaf(v, False)
        elif level == depth:
            leaf(v, True)
        else:
            for ch in red_children(v):
                walk(ch, level + 1)

    walk(np.vstack([np.zeros(d), np.eye(d)]), 0)
    return out, npts


def build_d_subcell(space: fem.Space, balls, a_in: float, a_out: float, kind: str, depth: int, ng: int):
    """D per cell (layouts of dogip.build_d) for the inclusion coefficient."""
    d, k = space.d, space.k
    q = ref.w_order(k, kind)
    balls = np.asarray(balls, dtype=np.float64)
    R, J, Rinv, _ = fem.geometry(space.coords, space.cells)
    vol = J / math.factorial(d)
    w = ref.what(d, q)
    nel = len(space.cells)
    integ = np.empty((nel, len(w)))
    for e in range(nel):
        X = space.coords[space.cells[e]]
        s, _ = subcell_integrals(X, balls, q, depth, ng)
        integ[e] = a_out * vol[e] * w + (a_in - a_out) * J[e] * s
    if kind == "wp":
        return integ
    K = np.einsum("erp,esp->ers", Rinv, Rinv)  # R^-1 R^-T
    return integ[:, :, None, None] * K[:, None, :, :]
