"""GPU parity of the HIP apply, diagonal, D construction and adjoint contraction
against the CPU oracle, through the C interface."""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import dogip as odg
from oracle import fem
from oracle import reference as ref
from workloads import coef_aniso_2d, coef_aniso_3d, coef_uniform, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _coef(kind, d, nel, seed):
    if kind == "wp":
        return coef_uniform(nel, 1.0, 100.0, seed), "scalar"
    return (coef_aniso_2d(nel, seed) if d == 2 else coef_aniso_3d(nel, seed)), "sym"


class Case:
    """One problem built on both sides, with the dof permutation between them."""

    def __init__(self, d, n, k, kind, seed=0, jitter=0.12, tile_waves=1, variant=0, bc=None, coef=None,
                 coef_kind=None):
        from paper_1710_09913_amd import Mesh, Operator, Space

        print(f"[case] d={d} n={n} k={k} kind={kind} seed={seed} tile_waves={tile_waves} variant={variant}",
              flush=True)
        self.d, self.k, self.kind = d, k, kind
        self.coords, self.cells = unit_mesh(d, n, jitter=jitter, seed=seed)
        nel = len(self.cells)
        if coef is None:
            coef, coef_kind = _coef(kind, d, nel, seed)
        self.coef, self.coef_kind = coef, coef_kind
        self.dirichlet = (kind == "se") if bc is None else bc == "dirichlet"
        self.space = Space(Mesh(self.coords, self.cells), k, kind, "dirichlet" if self.dirichlet else "none")
        self.op = Operator(self.space, torch.from_numpy(np.ascontiguousarray(coef)), coef_kind, fp32=True,
                           tile_waves=tile_waves, variant=variant)
        self.osp = fem.make_space(self.coords, self.cells, k)
        self.perm = match_dofs(self.space.dof_coords(), self.osp.dof_coords)
        if coef_kind == "raw_d":
            self.D = _unpack_d(coef, kind, d)
        else:
            self.D = odg.build_d(self.osp, coef if coef_kind != "sym" else fem.unpack_sym(coef, d), kind)

    def to_oracle(self, v):
        out = np.empty_like(v)
        out[self.perm] = v
        return out

    def from_oracle(self, v):
        return v[self.perm]

    def oracle_apply(self, u_prod, D=None):
        D = self.D if D is None else D
        uo = self.to_oracle(u_prod)
        f = odg.apply_dirichlet if self.dirichlet else odg.apply
        return self.from_oracle(f(self.osp, D, uo, self.kind))

    def abs_bound(self, u_prod):
        uo = self.to_oracle(u_prod)
        return self.from_oracle(odg.apply_abs(self.osp, self.D, uo, self.kind, self.dirichlet))

    def n_incident_max(self):
        return int(np.bincount(self.osp.cell_dofs.reshape(-1)).max())


def _unpack_d(raw, kind, d):
    if kind == "wp":
        return raw[:, :, 0]
    return fem.unpack_sym(raw, d)


def _gpu(v):
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


APPLY_CASES = (
    [(2, 9, k, kind) for k in (1, 2, 3, 4, 5, 6, 8) for kind in ("wp", "se")]
    + [(3, 3, k, kind) for k in (1, 2, 3) for kind in ("wp", "se")]
    + [(3, 2, 4, "se"), (3, 2, 4, "wp")]
)


@pytest.mark.parametrize("d,n,k,kind", APPLY_CASES)
def test_apply_f64_parity(d, n, k, kind):
    """FP64 apply = oracle Algorithm 1 (with identity Dirichlet rows for the elliptic
    problem): 1e-11 normwise and 1e-12 of |B^|^T|D||B^||u| componentwise."""
    c = Case(d, n, k, kind, seed=k)
    u = random_vector(c.space.ndofs, seed=k)
    y = c.op.apply(_gpu(u)).cpu().numpy()
    yo = c.oracle_apply(u)
    assert rel_err(y, yo) <= 1e-11
    bound = c.abs_bound(u)
    assert np.all(np.abs(y - yo) <= 1e-12 * bound + 1e-300)
    # the other element-kernel variant gives the same result
    from paper_1710_09913_amd.capi import DOGIP_VARIANT_LOOPED

    if c.op.info["variant"] != DOGIP_VARIANT_LOOPED:
        c2 = Case(d, n, k, kind, seed=k, variant=DOGIP_VARIANT_LOOPED)
        y2 = c2.op.apply(_gpu(u)).cpu().numpy()
        assert rel_err(y2, yo) <= 1e-11


@pytest.mark.parametrize("d,n,k,kind", [(2, 9, 1, "se"), (2, 9, 3, "se"), (2, 9, 5, "wp"), (2, 9, 5, "se"),
                                        (3, 3, 2, "se"), (3, 3, 3, "se"), (2, 6, 8, "se")])
def test_apply_f32_within_rounding_bound(d, n, k, kind):
    """FP32 apply: |y32 - y| <= 2 gamma_m |B^|^T|D||B^||u| with gamma_m = m u32 / (1 - m u32),
    m = V_T + nb W_T + nb + (max cells per dof) + 3 roundings of the inputs."""
    c = Case(d, n, k, kind, seed=10 + k)
    u = random_vector(c.space.ndofs, seed=3)
    y32 = c.op.apply(_gpu(u), prec="f32").cpu().numpy()
    yo = c.oracle_apply(u)
    info = c.space.info
    m = info["vt"] + info["nb"] * info["wt"] + info["nb"] + c.n_incident_max() + 3
    gam = m * 2.0 ** -24 / (1 - m * 2.0 ** -24)
    bound = c.abs_bound(u)
    assert np.all(np.abs(y32 - yo) <= 2 * gam * bound + 1e-300)
    err = rel_err(y32, yo)
    print(f"fp32 normwise relative error {err:.3e}")
    assert err < 1e-4


@pytest.mark.parametrize("d,n,k,kind", [(2, 9, 3, "se"), (3, 3, 3, "se"), (2, 9, 2, "wp")])
def test_general_per_node_d(d, n, k, kind):
    """A random indefinite D per W node (no piecewise-constant structure) is applied exactly."""
    from paper_1710_09913_amd import Mesh, Space

    coords, cells = unit_mesh(d, n, jitter=0.1, seed=2)
    s = Space(Mesh(coords, cells), k, kind, "none")
    raw = np.random.default_rng(5).uniform(-1, 1, size=(len(cells), s.info["wt"], s.info["nsym"]))
    c = Case(d, n, k, kind, seed=2, jitter=0.1, bc="none", coef=raw, coef_kind="raw_d")
    u = random_vector(c.space.ndofs, seed=9)
    y = c.op.apply(_gpu(u)).cpu().numpy()
    assert rel_err(y, c.oracle_apply(u)) <= 1e-11
    d_out = c.op.export_d().cpu().numpy()
    np.testing.assert_array_equal(d_out, raw)


@pytest.mark.parametrize("d,n,k,kind", [(2, 7, 2, "wp"), (2, 7, 4, "se"), (3, 3, 3, "se"), (3, 2, 2, "wp")])
def test_build_d_and_diagonal(d, n, k, kind):
    c = Case(d, n, k, kind, seed=4)
    dg = c.op.export_d().cpu().numpy()
    if kind == "wp":
        do = c.D[:, :, None]
    else:
        iu = np.triu_indices(d)
        do = c.D[:, :, iu[0], iu[1]]
    assert rel_err(dg, do) <= 1e-14
    diag = c.op.diag().cpu().numpy()
    expect = c.from_oracle(odg.diagonal(c.osp, c.D, kind, c.dirichlet))
    assert rel_err(diag, expect) <= 1e-12


@pytest.mark.parametrize("tile_waves", [1, 8])
def test_diagonal_bitwise_reproducible(tile_waves):
    """The Jacobi diagonal adds the cells' terms in a fixed order (wave by wave inside a
    tile, staged partial sums across tiles): repeated builds agree bit for bit."""
    c = Case(3, 8, 3, "se", seed=11, tile_waves=tile_waves)
    assert c.op.info["ntiles"] > 1 and c.op.info["nshared"] > 0
    d1 = c.op.diag().cpu().numpy()
    expect = c.from_oracle(odg.diagonal(c.osp, c.D, "se", c.dirichlet))
    assert rel_err(d1, expect) <= 1e-12
    for _ in range(20):
        np.testing.assert_array_equal(c.op.diag().cpu().numpy(), d1)


@pytest.mark.parametrize("d,n,k", [(2, 8, 3), (3, 3, 2)])
def test_grad_contraction(d, n, k):
    theta = np.random.default_rng(1).normal(0, 0.5, size=2 * n * n if d == 2 else 6 * n ** 3)
    c = Case(d, n, k, "se", seed=6, coef=theta, coef_kind="logscalar")
    c.D = odg.build_d(c.osp, np.exp(theta), "se")
    u = random_vector(c.space.ndofs, seed=1)
    lam = random_vector(c.space.ndofs, seed=2)
    g = c.op.grad_logcoef(_gpu(u), _gpu(lam)).cpu().numpy()
    go = -odg.energy_contraction(c.osp, c.D, c.to_oracle(u), c.to_oracle(lam), "se", True)
    assert rel_err(g, go) <= 1e-11


@pytest.mark.parametrize("tw", [1, 2, 4, 8])
def test_tile_size_invariance(tw):
    """Tiles of 64..512 cells (many shared dofs, ragged last tile) give the same apply."""
    c = Case(2, 13, 3, "se", seed=3, tile_waves=tw)
    u = random_vector(c.space.ndofs, seed=4)
    y = c.op.apply(_gpu(u)).cpu().numpy()
    assert rel_err(y, c.oracle_apply(u)) <= 1e-11
    assert c.op.info["tile_cells"] == 64 * tw


def test_degenerate_inputs():
    """One cell; zero input; boundary-only input; a vector of ones in the projection."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    m = Mesh(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 2]]))
    s = Space(m, 3, "wp", "none")
    op = Operator(s, torch.tensor([2.0]), "scalar")
    one = torch.ones(s.ndofs, dtype=torch.float64, device="cuda")
    total = float(torch.dot(one, op.apply(one)))
    assert abs(total - 2.0 * 0.5) <= 1e-14  # 1^T A 1 = int m
    c = Case(2, 6, 2, "se", seed=1)
    z = torch.zeros(c.space.ndofs, dtype=torch.float64, device="cuda")
    assert float(c.op.apply(z).abs().max()) == 0.0
    ub = np.zeros(c.space.ndofs)
    bnd = c.space.boundary()
    ub[bnd] = 1.0 + np.arange(len(bnd))
    y = c.op.apply(_gpu(ub)).cpu().numpy()
    np.testing.assert_array_equal(y[bnd], ub[bnd])
    inner = np.setdiff1d(np.arange(c.space.ndofs), bnd)
    assert np.abs(y[inner]).max() == 0.0


def test_apply_errors():
    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    s = Space(Mesh.unit(2, 2), 2, "se", "dirichlet")
    op = Operator(s, torch.ones(8, dtype=torch.float64), "scalar", fp32=False)
    u = torch.ones(s.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(DogipError):
        op.apply(u, u)  # in place
    with pytest.raises(DogipError):
        op.apply(u, prec="f32")  # no FP32 copy
    with pytest.raises(DogipError):
        Operator(Space(Mesh.unit(2, 2), 2, "wp", "none"), torch.ones(8, 3, dtype=torch.float64), "sym")


def test_apply_bitwise_reproducible():
    """No floating-point atomics across workgroups: repeated applies agree bit for bit."""
    c = Case(3, 3, 3, "se", seed=7, tile_waves=1)
    u = _gpu(random_vector(c.space.ndofs, seed=8))
    y1 = c.op.apply(u).cpu().numpy()
    for _ in range(3):
        np.testing.assert_array_equal(c.op.apply(u).cpu().numpy(), y1)
    z1 = c.op.apply(u, prec="f32").cpu().numpy()
    np.testing.assert_array_equal(c.op.apply(u, prec="f32").cpu().numpy(), z1)
