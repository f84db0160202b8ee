"""Tiles larger than a workgroup: a tile of te cells is taken in passes of as many cells
as the workgroup has lanes (Algorithm 1 over the tile's cells, the partial sums of every
pass added in the tile's LDS in ascending cell order).  Against the CPU oracle with
several tiles and a ragged last tile and pass; bitwise independence of the lanes; the
diagonal and the adjoint contraction in passes; refusals of lane counts."""

import numpy as np
import pytest

from helpers import rel_err
from oracle import dogip as odg
from workloads import random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _gamma32(c):
    info = c.space.info
    m = info["vt"] + info["nb"] * info["wt"] + info["nb"] + c.n_incident_max() + 3
    return m * 2.0 ** -24 / (1 - m * 2.0 ** -24)


# (dim, n, k, kind, tile_waves): 3D 7^3 = 2058 cells in 1536-cell tiles (the last one 522
# cells: one full pass of 512 lanes and a pass of 10 cells), 3D 5^3 P2 (750 cells, one
# ragged tile), 2D 33^2 P3 (2178 cells) in 768-cell tiles, 2D projection P4 in 1024-cell tiles
CASES = [(3, 7, 3, "se", 24), (3, 5, 2, "se", 24), (3, 7, 2, "wp", 12), (2, 33, 3, "se", 12), (2, 25, 4, "wp", 16)]


@pytest.mark.parametrize("d,n,k,kind,tw", CASES)
def test_multipass_tiles_match_oracle(d, n, k, kind, tw):
    from test_gpu_apply import Case

    c = Case(d, n, k, kind, seed=21, tile_waves=tw)
    te = c.op.info["tile_cells"]
    assert 512 < te <= 64 * tw
    u = random_vector(c.space.ndofs, seed=5)
    yo = c.oracle_apply(u)
    bound = c.abs_bound(u)
    y64 = c.op.apply(_gpu(u)).cpu().numpy()
    assert np.all(np.abs(y64 - yo) <= 1e-12 * bound + 1e-300)
    y32 = c.op.apply(_gpu(u), prec="f32").cpu().numpy()
    assert np.all(np.abs(y32 - yo) <= 2 * _gamma32(c) * bound + 1e-300)
    # the Jacobi diagonal in passes against the oracle's
    diag = c.op.diag().cpu().numpy()
    assert rel_err(diag, c.from_oracle(odg.diagonal(c.osp, c.D, kind, c.dirichlet))) <= 1e-12


@pytest.mark.parametrize("d,n,k,kind,tw", [(3, 7, 3, "se", 24), (2, 33, 3, "se", 12)])
def test_lanes_do_not_change_results(d, n, k, kind, tw):
    """Every admissible lane count gives the same FP64 and FP32 results bit for bit (the
    passes add a tile's cells in ascending order), with and without the CG energy."""
    from test_gpu_apply import Case

    c = Case(d, n, k, kind, seed=22, tile_waves=tw)
    te = c.op.info["tile_cells"]
    u = _gpu(random_vector(c.space.ndofs, seed=6))
    ref64 = c.op.apply(u)
    ref32 = c.op.apply(u, prec="f32")
    for lanes in [x for x in (64, 128, 192, 256, 384, 512, 768) if te % x == 0]:
        c.op.set_tile_lanes(lanes if lanes <= 512 else 0, lanes)
        print(f"[lanes] te={te} lanes={lanes}", flush=True)
        if lanes <= 512:
            assert torch.equal(c.op.apply(u), ref64), lanes
        assert torch.equal(c.op.apply(u, prec="f32"), ref32), lanes
    c.op.set_tile_lanes(0, 0)
    assert torch.equal(c.op.apply(u), ref64)


def test_lanes_refused():
    from test_gpu_apply import Case

    from paper_1710_09913_amd.capi import DogipError

    c = Case(3, 4, 3, "se", seed=23, tile_waves=24)
    assert c.op.info["tile_cells"] == 1536
    u = _gpu(random_vector(c.space.ndofs, seed=7))
    y = c.op.apply(u)
    for bad in ((100, 0), (0, 100), (-64, 0), (1024, 0), (0, 1024 + 512)):
        with pytest.raises(DogipError):
            c.op.set_tile_lanes(*bad)
    c.op.set_tile_lanes(768, 0)  # divides the tile, above the FP64 kernel's 512 lanes: refused at launch
    with pytest.raises(DogipError):
        c.op.apply(u)
    c.op.set_tile_lanes(0, 0)
    assert torch.equal(c.op.apply(u), y)


def test_multipass_grad_matches_oracle():
    """The adjoint contraction g_T = -(B^ lam_T) . D_T (B^ u_T) in passes over 1536-cell
    tiles: against the oracle, and bit for bit against 64-cell tiles (no sums across
    cells)."""
    from test_gpu_apply import Case

    theta = np.random.default_rng(3).normal(0, 0.5, size=6 * 6 ** 3)
    c1 = Case(3, 6, 3, "se", seed=24, tile_waves=1, coef=theta, coef_kind="logscalar")
    c2 = Case(3, 6, 3, "se", seed=24, tile_waves=24, coef=theta, coef_kind="logscalar")
    assert c2.op.info["tile_cells"] == 1536
    D = odg.build_d(c2.osp, np.exp(theta), "se")
    u = random_vector(c1.space.ndofs, seed=8)
    lam = random_vector(c1.space.ndofs, seed=9)
    g1 = c1.op.grad_logcoef(_gpu(u), _gpu(lam))
    g2 = c2.op.grad_logcoef(_gpu(u), _gpu(lam))
    assert torch.equal(g1, g2)
    go = -odg.energy_contraction(c2.osp, D, c2.to_oracle(u), c2.to_oracle(lam), "se", True)
    assert rel_err(g2.cpu().numpy(), go) <= 1e-11


def test_multipass_mixed_pcg_matches_f64():
    """Mixed Jacobi-PCG (the FP32 apply with FP32 vectors and the fused energy) and the
    FP64 solve on 1536-cell tiles reach the same solution."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    sp = Space(Mesh.unit(3, 8), 3, "se", "dirichlet")
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True, tile_waves=24)
    assert op.info["tile_cells"] == 1536
    b = op.apply(_gpu(random_vector(sp.ndofs, seed=10)))
    x64, s64 = op.pcg(b, tol=1e-10, maxit=5000, mode="f64")
    for mode in ("mixed", "mixed_v64", "pmg_mixed"):
        x, st = op.pcg(b, tol=1e-10, maxit=5000, mode=mode)
        assert st["status"] == 0 and st["relres_true"] <= 1.05e-10, (mode, st)
        assert rel_err(x.cpu().numpy(), x64.cpu().numpy()) <= 1e-7, mode
