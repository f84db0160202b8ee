"""GPU parity of the global weighted-projection form (Theorem 1): one D value per dof of
C_{N,2k}, against the oracle's literal B^T diag(D) B."""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import fem, global_wp
from workloads import coef_uniform, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


class GCase:
    def __init__(self, d, n, k, seed=0, jitter=0.12, tile_waves=0, variant=0, coef=None, coef_kind="scalar"):
        from paper_1710_09913_amd import Mesh, Operator, Space

        print(f"[global] d={d} n={n} k={k} seed={seed} tile_waves={tile_waves} variant={variant}", flush=True)
        self.coords, self.cells = unit_mesh(d, n, jitter=jitter, seed=seed)
        nel = len(self.cells)
        self.coef = coef_uniform(nel, 1.0, 100.0, seed) if coef is None else coef
        self.space = Space(Mesh(self.coords, self.cells), k, "wp", "none")
        self.op = Operator(self.space, torch.from_numpy(np.ascontiguousarray(self.coef)), coef_kind, fp32=True,
                           tile_waves=tile_waves, variant=variant, global_w=True)
        self.osp = fem.make_space(self.coords, self.cells, k)
        self.wsp = global_wp.w_space(self.osp)
        self.B = global_wp.interpolation_matrix(self.osp, self.wsp)
        if coef_kind == "raw_d":
            raw = self.coef.reshape(nel, -1)
            self.Dg = np.bincount(self.wsp.cell_dofs.reshape(-1), weights=raw.reshape(-1), minlength=self.wsp.ndofs)
        else:
            self.Dg = global_wp.build_d_global(self.osp, self.wsp, self.coef)
        self.perm = match_dofs(self.space.dof_coords(), self.osp.dof_coords)

    def oracle(self, u):
        uo = np.empty_like(u)
        uo[self.perm] = u
        return global_wp.apply_global(self.osp, self.wsp, self.Dg, uo, self.B)[self.perm]

    def abs_bound(self, u):
        uo = np.empty_like(u)
        uo[self.perm] = np.abs(u)
        Ba = abs(self.B)
        return (Ba.T @ (np.abs(self.Dg) * (Ba @ uo)))[self.perm]


def _gpu(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


CASES = [(2, 5, k) for k in (1, 2, 3, 4, 5, 6, 8)] + [(3, 3, 1), (3, 3, 2), (3, 2, 3), (3, 1, 4)]


@pytest.mark.parametrize("d,n,k", CASES)
def test_global_f64_parity(d, n, k):
    c = GCase(d, n, k, seed=k)
    u = random_vector(c.space.ndofs, seed=k)
    y = c.op.apply(_gpu(u)).cpu().numpy()
    yo = c.oracle(u)
    assert rel_err(y, yo) <= 1e-11
    assert np.all(np.abs(y - yo) <= 1e-12 * c.abs_bound(u) + 1e-300)
    assert c.op.info["ndofs_w"] == c.wsp.ndofs
    assert c.op.info["bytes_d64"] == 8 * c.wsp.ndofs
    from paper_1710_09913_amd.capi import DOGIP_VARIANT_LOOPED

    if c.op.info["variant"] != DOGIP_VARIANT_LOOPED:
        c2 = GCase(d, n, k, seed=k, variant=DOGIP_VARIANT_LOOPED)
        assert rel_err(c2.op.apply(_gpu(u)).cpu().numpy(), yo) <= 1e-11


@pytest.mark.parametrize("d,n,k", [(2, 6, 1), (2, 5, 3), (3, 3, 2)])
def test_global_equals_elementwise(d, n, k):
    """Theorems 1 and 2 give one operator: the global and element-wise applies agree."""
    from paper_1710_09913_amd import Operator

    c = GCase(d, n, k, seed=3)
    el = Operator(c.space, torch.from_numpy(c.coef), "scalar", fp32=True)
    u = _gpu(random_vector(c.space.ndofs, seed=4))
    y1, y2 = c.op.apply(u), el.apply(u)
    assert float(torch.linalg.norm(y1 - y2) / torch.linalg.norm(y2)) <= 1e-13
    assert el.info["bytes_d64"] > c.op.info["bytes_d64"]


@pytest.mark.parametrize("d,n,k", [(2, 5, 2), (2, 5, 5), (3, 3, 2)])
def test_global_f32_bound(d, n, k):
    c = GCase(d, n, k, seed=7)
    u = random_vector(c.space.ndofs, seed=8)
    y32 = c.op.apply(_gpu(u), prec="f32").cpu().numpy()
    info = c.space.info
    inc = int(np.bincount(c.osp.cell_dofs.reshape(-1)).max())
    m = info["vt"] + info["wt"] + 1 + inc + 3
    gam = m * 2.0 ** -24 / (1 - m * 2.0 ** -24)
    assert np.all(np.abs(y32 - c.oracle(u)) <= 2 * gam * c.abs_bound(u) + 1e-300)


@pytest.mark.parametrize("d,n,k", [(2, 5, 3), (3, 3, 2)])
def test_global_diagonal_and_pcg(d, n, k):
    """Jacobi diagonal sum_j B_jl^2 D_j, and PCG on the projection system against a direct solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    c = GCase(d, n, k, seed=5)
    diag = c.op.diag().cpu().numpy()
    do = (c.B.multiply(c.B)).T @ c.Dg
    assert rel_err(diag, do[c.perm]) <= 1e-12
    for _ in range(3):
        np.testing.assert_array_equal(c.op.diag().cpu().numpy(), diag)
    xs = random_vector(c.space.ndofs, seed=6)
    b = c.oracle(xs)
    x, st = c.op.pcg(_gpu(b), tol=1e-10, mode="f64")
    A = sp.csr_matrix(c.B.T @ sp.diags(c.Dg) @ c.B)
    bo = np.empty_like(b)
    bo[c.perm] = b
    xd = spla.spsolve(A, bo)[c.perm]
    assert st["status"] == 0 and st["relres_true"] <= 1e-10
    assert rel_err(x.cpu().numpy(), xd) <= 1e-7
    x32, st32 = c.op.pcg(_gpu(b), tol=1e-10, mode="mixed")
    assert st32["status"] == 0 and st32["relres_true"] <= 1e-10


def test_global_raw_d_is_summed():
    """Raw per-cell values: the global D of a W dof is the sum of its cells' values."""
    d, n, k = 2, 4, 2
    coords, cells = unit_mesh(d, n, jitter=0.1, seed=1)
    from paper_1710_09913_amd import Mesh, Space

    wt = Space(Mesh(coords, cells), k, "wp", "none").info["wt"]
    raw = np.random.default_rng(3).uniform(-1, 1, size=(len(cells), wt))
    c = GCase(d, n, k, seed=1, jitter=0.1, coef=raw, coef_kind="raw_d")
    u = random_vector(c.space.ndofs, seed=2)
    assert rel_err(c.op.apply(_gpu(u)).cpu().numpy(), c.oracle(u)) <= 1e-11


@pytest.mark.parametrize("tw", [1, 2, 4, 8])
def test_global_tile_invariance_and_reproducible(tw):
    c = GCase(2, 12, 2, seed=9, tile_waves=tw)
    u = random_vector(c.space.ndofs, seed=9)
    y1 = c.op.apply(_gpu(u))
    y2 = c.op.apply(_gpu(u))
    assert torch.equal(y1, y2)
    assert rel_err(y1.cpu().numpy(), c.oracle(u)) <= 1e-11


def test_global_errors():
    from paper_1710_09913_amd import Batch, Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    mesh = Mesh.unit(2, 4)
    se = Space(mesh, 2, "se", "dirichlet")
    ones = torch.ones(se.ncells, dtype=torch.float64)
    with pytest.raises(DogipError):
        Operator(se, ones, "scalar", global_w=True)
    wp = Space(mesh, 2, "wp", "none")
    op = Operator(wp, ones, "scalar", global_w=True)
    with pytest.raises(DogipError):
        op.export_d()
    u = torch.ones(wp.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(DogipError):
        op.grad_logcoef(u, u)
    with pytest.raises(DogipError):
        Batch([op])
