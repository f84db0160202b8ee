"""The matrix-core FP32 apply of the 3D P3 elliptic operator (DOGIP_VARIANT_MFMA) against
the CPU oracle.

Rounding bound.  B^ of 3D P3 is exact in bfloat16 and the vector operand is split into
three bfloat16 terms exactly, so every product is exact and the error comes from the
FP32 sums (and the FP32 copies of u and D).  Each output of the first product g = B^ u_T
is three chained 16x16x32 matrix-core steps, each adding 32 products and the running
sum: at most 3 (32 + 1) FP32 additions.  The second product y_T = B^^T h takes five
K-blocks of 32, three terms each: at most 15 (32 + 1).  With the 3 FMAs of h = D_T g,
the cells per dof (FP64 additions) and 3 roundings of the inputs,
  |y32 - y| <= 2 gamma_m |B^|^T |D| |B^| |u|,  m = 99 + 495 + 3 + n_inc + 3.
"""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import dogip as odg
from oracle import fem, solve, subcell
from workloads import coef_lognormal, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def _gamma_mfma(n_inc):
    m = 3 * 33 + 15 * 33 + 3 + n_inc + 3
    return m * 2.0 ** -24 / (1 - m * 2.0 ** -24)


def _mfma():
    from paper_1710_09913_amd.capi import DOGIP_VARIANT_MFMA

    return DOGIP_VARIANT_MFMA


@pytest.mark.parametrize("n,tile_waves,coef", [(3, 1, "sym"), (5, 1, "sym"), (5, 8, "sym"), (4, 2, "raw_d")])
def test_mfma_f32_within_rounding_bound(n, tile_waves, coef):
    """Several tiles with a ragged last wave (5^3 x 6 = 750 cells), an anisotropic tensor
    per cell or a random indefinite D per W node (RAW_D, negative entries)."""
    from test_gpu_apply import Case

    from paper_1710_09913_amd import Mesh, Space

    kw = {}
    if coef == "raw_d":
        coords, cells = unit_mesh(3, n, jitter=0.1, seed=4)
        s = Space(Mesh(coords, cells), 3, "se", "none")
        raw = np.random.default_rng(6).uniform(-1, 1, size=(len(cells), s.info["wt"], s.info["nsym"]))
        kw = dict(bc="none", coef=raw, coef_kind="raw_d", jitter=0.1)
    c = Case(3, n, 3, "se", seed=4, tile_waves=tile_waves, variant=_mfma(), **kw)
    assert c.op.info["variant"] == _mfma()
    u = random_vector(c.space.ndofs, seed=8)
    y32 = c.op.apply(_gpu(u), prec="f32").cpu().numpy()
    yo = c.oracle_apply(u)
    bound = c.abs_bound(u)
    gam = _gamma_mfma(c.n_incident_max())
    assert np.all(np.abs(y32 - yo) <= 2 * gam * bound + 1e-300)
    err = rel_err(y32, yo)
    print(f"mfma fp32 normwise relative error {err:.3e}")
    assert err < 1e-5
    # the FP64 apply of this variant is the unrolled vector kernel: bit for bit on the same tiles
    c2 = Case(3, n, 3, "se", seed=4, tile_waves=tile_waves, variant=1, **kw)
    assert c.op.info["tile_cells"] == c2.op.info["tile_cells"]
    assert torch.equal(c.op.apply(_gpu(u)), c2.op.apply(_gpu(u)))
    # against the FP32 vector kernel: both within their bounds of the exact result
    y32v = c2.op.apply(_gpu(u), prec="f32").cpu().numpy()
    assert np.all(np.abs(y32 - y32v) <= 4 * gam * bound + 1e-300)


def test_mfma_mixed_pcg_matches_direct():
    """Mixed Jacobi-PCG with the matrix-core FP32 apply reaches the FP64 tolerance and the
    oracle's direct solution (3D 4^3 P3, jittered, lognormal coefficient)."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    coords, cells = unit_mesh(3, 4, jitter=0.1, seed=3)
    a = coef_lognormal(coords, cells, 3)
    sp = Space(Mesh(coords, cells), 3, "se", "dirichlet")
    op = Operator(sp, torch.from_numpy(a), "scalar", fp32=True, variant=_mfma())
    osp = fem.make_space(coords, cells, 3)
    perm = match_dofs(sp.dof_coords(), osp.dof_coords)
    A = fem.assemble(osp, fem.element_matrices(osp, a, "se"))
    b = fem.load_vector(osp, 1.0)
    b[osp.boundary] = 0.0
    x_lu = solve.direct_dirichlet(A, b, osp.boundary)
    Ab = solve.dirichlet_matrix(A, osp.boundary).toarray()
    ev = np.linalg.eigvalsh(Ab)
    kappa = ev.max() / ev.min()
    for mode in ("mixed", "mixed_v64", "pmg_mixed"):
        print(f"[mfma pcg] {mode}", flush=True)
        x, st = op.pcg(_gpu(b[perm]), tol=1e-10, maxit=5000, mode=mode)
        assert st["status"] == 0 and st["relres_true"] <= 1.05e-10, (mode, st)
        assert rel_err(x.cpu().numpy(), x_lu[perm]) <= 2 * kappa * 1e-10, mode


def test_mfma_inclusions():
    """D by sub-cell quadrature is written in the variant's FP32 layout too: the FP32
    apply after dogip_op_set_inclusions is within the bound of the oracle's sub-cell D."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    coords, cells = unit_mesh(3, 3, jitter=0.05, seed=7)
    sp = Space(Mesh(coords, cells), 3, "se", "dirichlet")
    op = Operator(sp, torch.ones(len(cells), dtype=torch.float64), "scalar", fp32=True, variant=_mfma())
    balls = np.array([[0.4, 0.5, 0.45, 0.3], [0.8, 0.2, 0.7, 0.2]])
    op.set_inclusions(balls, 50.0, 1.0, depth=2, ng=3)
    osp = fem.make_space(coords, cells, 3)
    perm = match_dofs(sp.dof_coords(), osp.dof_coords)
    D = subcell.build_d_subcell(osp, balls, 50.0, 1.0, "se", depth=2, ng=3)
    u = random_vector(sp.ndofs, seed=2)
    uo = np.empty_like(u)
    uo[perm] = u
    yo = odg.apply_dirichlet(osp, D, uo, "se")[perm]
    bound = odg.apply_abs(osp, D, uo, "se", True)[perm]
    y32 = op.apply(_gpu(u), prec="f32").cpu().numpy()
    n_inc = int(np.bincount(osp.cell_dofs.reshape(-1)).max())
    assert np.all(np.abs(y32 - yo) <= 2 * _gamma_mfma(n_inc) * bound + 1e-300)
    y64 = op.apply(_gpu(u)).cpu().numpy()
    assert rel_err(y64, yo) <= 1e-11


def test_mfma_refusals():
    """The variant is refused outside 3D P3 elliptic, for the global form, and by batches."""
    from paper_1710_09913_amd import Batch, Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    sp2 = Space(Mesh.unit(3, 2), 2, "se", "dirichlet")
    with pytest.raises(DogipError):
        Operator(sp2, torch.ones(sp2.ncells, dtype=torch.float64), "scalar", fp32=True, variant=_mfma())
    sp3 = Space(Mesh.unit(3, 2), 3, "se", "dirichlet")
    op = Operator(sp3, torch.ones(sp3.ncells, dtype=torch.float64), "scalar", fp32=True, variant=_mfma())
    with pytest.raises(DogipError):
        Batch([op])


def test_mfma_fullsize_sampled_rows():
    """3D 64^3 P3 with the lognormal coefficient (the benchmark operator): sampled FP32 rows
    of the matrix-core apply within the bound, and bitwise-reproducible repeated applies."""
    from test_gpu_fullsize import NSAMPLE, FullCase

    from paper_1710_09913_amd import Operator

    print("[mfma full] 3D 64^3 P3", flush=True)
    c = FullCase(3, 64, 3, "se")
    del c.op
    torch.cuda.empty_cache()
    c.op = Operator(c.space, torch.from_numpy(c.coef), c.coef_kind, fp32=True, variant=_mfma())
    y32 = c.op.apply(c.ug, prec="f32")
    assert torch.equal(y32, c.op.apply(c.ug, prec="f32"))
    y32 = y32.cpu().numpy()
    rng = np.random.default_rng(17)
    s = np.sort(np.setdiff1d(rng.choice(c.space.ndofs, NSAMPLE, replace=False), c.bnd))
    yo, ab = c.sampled_rows(s)
    assert np.all(np.abs(y32[s] - yo) <= 2 * _gamma_mfma(c.n_incident_max()) * ab + 1e-300)
    print(f"mfma fp32 sampled normwise relative error {rel_err(y32[s], yo):.3e}")
