"""Memory and operation counts of Section 3 (oracle, test infrastructure).

* CSR memory model: mem A = 2 nnz A + nrows A.
* DoGIP storage per cell, nnz A^DoGIP_T: W_T for the weighted projection and
  d^2 W_T for the elliptic problem (the tables store full d x d blocks).
* eq. memory_eff: nnz A^DoGIP_T * dim M / mem A, with dim M = 2N^2 or 6N^3 cells.
* eq. comp_eff: [2 (nnz B^ - nnz_{+-1} B^) + nnz A^DoGIP_T] * dim M / nnz A.
* Structural nnz of the standard matrix on the structured mesh family: counted
  on small meshes by ``fem.structural_nnz`` and extended to the paper's N by the
  exact polynomial (degree d in N) through those counts, checked on one extra N.
"""

from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

from . import fem
from . import reference as ref

__all__ = [
    "dims",
    "mem_csr",
    "mem_dogip_cell",
    "n_cells",
    "memory_eff",
    "comp_eff",
    "structural_nnz_poly",
]


def dims(d: int, k: int, kind: str):
    """(V_T, W_T)."""
    return ref.dim_p(d, k), ref.dim_p(d, ref.w_order(k, kind))


def n_cells(d: int, n: int) -> int:
    return 2 * n * n if d == 2 else 6 * n ** 3


def mem_csr(nnz: int, nrows: int) -> int:
    return 2 * nnz + nrows


def mem_dogip_cell(d: int, k: int, kind: str) -> int:
    _, wt = dims(d, k, kind)
    return wt if kind == "wp" else d * d * wt


def memory_eff(d, k, kind, n, mem_a) -> float:
    return mem_dogip_cell(d, k, kind) * n_cells(d, n) / mem_a


def comp_eff(d, k, kind, n, nnz_a) -> float:
    nnz, pm1 = ref.nnz_counts(d, k, kind)
    return (2 * (nnz - pm1) + mem_dogip_cell(d, k, kind)) * n_cells(d, n) / nnz_a


def _lagrange_eval(xs, ys, x):
    tot = Fraction(0)
    for i, (xi, yi) in enumerate(zip(xs, ys)):
        term = Fraction(yi)
        for j, xj in enumerate(xs):
            if j != i:
                term *= Fraction(x - xj, xi - xj)
        tot += term
    return tot


@lru_cache(maxsize=None)
def _count(d, k, n):
    from workloads import unit_mesh  # seeded input generator, no method arithmetic
    coords, cells = unit_mesh(d, n)
    return fem.structural_nnz(fem.make_space(coords, cells, k))


def structural_nnz_poly(d: int, k: int, n: int, base: int = 3) -> int:
    """Structural nnz on the N-mesh from the degree-d polynomial through N = base..base+d,
    after checking it reproduces the count at N = base + d + 1."""
    xs = list(range(base, base + d + 1))
    ys = [_count(d, k, x) for x in xs]
    check = base + d + 1
    if _lagrange_eval(xs, ys, check) != _count(d, k, check):
        raise AssertionError("structural nnz is not polynomial on the sampled range")
    val = _lagrange_eval(xs, ys, n)
    if val.denominator != 1:
        raise AssertionError("non-integer extrapolation")
    return int(val)
