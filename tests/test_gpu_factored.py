"""The apply through the factored elliptic B^ (DOGIP_VARIANT_FACTORED) against the CPU
oracle.

Rounding bound.  The kernel forms G = B1 u_T (sums of at most V_T terms), per W node
g = B2_i G (at most n1 = dim P_{k-1} terms), h = D_i g (d terms), H = sum_i B2_i^T h (at
most W_T terms) and y_T = B1^T H (at most d n1 terms); with the cells per dof and the
roundings of the inputs,
  |y - y_exact| <= 2 gamma_m |B1|^T (I x |B2|)^T |D| (I x |B2|) |B1| |u|,
  m = V_T + n1 + d + W_T + d n1 + n_inc + 3,
the scale being the oracle's apply_abs_factored (pinned in test_oracle_factored.py)."""

import math

import numpy as np
import pytest

from helpers import rel_err
from oracle import dogip as odg
from workloads import random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _factored():
    from paper_1710_09913_amd.capi import DOGIP_VARIANT_FACTORED

    return DOGIP_VARIANT_FACTORED


def _gamma(c, unit):
    info = c.space.info
    d, k = c.d, c.k
    n1 = math.comb(k - 1 + d, d)
    m = info["vt"] + n1 + d + info["wt"] + d * n1 + c.n_incident_max() + 3
    return m * unit / (1 - m * unit)


CASES = [(2, 9, 2, 1), (2, 9, 3, 1), (2, 7, 4, 2), (2, 9, 5, 1), (3, 3, 2, 1), (3, 3, 3, 1), (2, 33, 3, 16),
         (3, 7, 3, 24), (3, 9, 2, 48)]


@pytest.mark.parametrize("d,n,k,tw", CASES)
def test_factored_apply_within_rounding_bound(d, n, k, tw):
    """FP64 and FP32 on jittered meshes with an anisotropic tensor, several tiles (64-cell
    tiles, and multi-pass 1024-3072-cell tiles with ragged last tiles)."""
    from test_gpu_apply import Case

    c = Case(d, n, k, "se", seed=30 + k, tile_waves=tw, variant=_factored())
    assert c.op.info["variant"] == _factored()
    u = random_vector(c.space.ndofs, seed=31)
    yo = c.oracle_apply(u)
    bound = c.from_oracle(odg.apply_abs_factored(c.osp, c.D, c.to_oracle(u), c.dirichlet))
    y64 = c.op.apply(_gpu(u)).cpu().numpy()
    assert np.all(np.abs(y64 - yo) <= 2 * _gamma(c, 2.0 ** -53) * bound + 1e-300)
    assert rel_err(y64, yo) <= 1e-13
    y32 = c.op.apply(_gpu(u), prec="f32").cpu().numpy()
    assert np.all(np.abs(y32 - yo) <= 2 * _gamma(c, 2.0 ** -24) * bound + 1e-300)
    err = rel_err(y32, yo)
    print(f"factored fp32 normwise relative error {err:.3e}")
    assert err < 1e-5
    # bitwise reproducible, and independent of the lanes of a multi-pass tile
    assert torch.equal(c.op.apply(_gpu(u)), c.op.apply(_gpu(u)))
    if c.op.info["tile_cells"] > 512:
        ref64 = c.op.apply(_gpu(u))
        c.op.set_tile_lanes(256, 256)
        assert torch.equal(c.op.apply(_gpu(u)), ref64)
        c.op.set_tile_lanes(0, 0)


def test_factored_raw_indefinite_d():
    """A random indefinite D per W node (RAW_D, negative entries)."""
    from test_gpu_apply import Case

    from paper_1710_09913_amd import Mesh, Space
    from workloads import unit_mesh

    coords, cells = unit_mesh(3, 3, jitter=0.1, seed=4)
    s = Space(Mesh(coords, cells), 3, "se", "none")
    raw = np.random.default_rng(6).uniform(-1, 1, size=(len(cells), s.info["wt"], s.info["nsym"]))
    c = Case(3, 3, 3, "se", seed=4, jitter=0.1, bc="none", coef=raw, coef_kind="raw_d", variant=_factored())
    u = random_vector(c.space.ndofs, seed=32)
    yo = c.oracle_apply(u)
    bound = c.from_oracle(odg.apply_abs_factored(c.osp, c.D, c.to_oracle(u), c.dirichlet))
    for prec, unit in (("f64", 2.0 ** -53), ("f32", 2.0 ** -24)):
        y = c.op.apply(_gpu(u), prec=prec).cpu().numpy()
        assert np.all(np.abs(y - yo) <= 2 * _gamma(c, unit) * bound + 1e-300), prec


def test_factored_mixed_pcg_matches_unrolled():
    """Mixed Jacobi-PCG and the multigrid solve with the factored apply reach the FP64
    tolerance and the unrolled operator's solution."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    sp = Space(Mesh.unit(2, 24), 5, "se", "dirichlet")
    a = torch.ones(sp.ncells, dtype=torch.float64)
    opf = Operator(sp, a, "scalar", fp32=True, variant=_factored())
    opu = Operator(sp, a, "scalar", fp32=True)
    b = opu.apply(_gpu(random_vector(sp.ndofs, seed=33)))
    xu, _ = opu.pcg(b, tol=1e-10, maxit=20000, mode="f64")
    for mode in ("f64", "mixed", "pmg_mixed"):
        x, st = opf.pcg(b, tol=1e-10, maxit=20000, mode=mode)
        assert st["status"] == 0 and st["relres_true"] <= 1.05e-10, (mode, st)
        assert rel_err(x.cpu().numpy(), xu.cpu().numpy()) <= 1e-7, mode


def test_factored_refusals():
    from paper_1710_09913_amd import Batch, Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    for d, k, kind in ((2, 1, "se"), (2, 3, "wp"), (3, 4, "se")):
        sp = Space(Mesh.unit(d, 2), k, kind, "dirichlet" if kind == "se" else "none")
        with pytest.raises(DogipError):
            Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True, variant=_factored())
    sp = Space(Mesh.unit(2, 4), 3, "se", "dirichlet")
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True, variant=_factored())
    with pytest.raises(DogipError):
        Batch([op])
