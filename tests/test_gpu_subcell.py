"""GPU parity of D built by sub-cell quadrature for a coefficient with jumps inside the
cells (inclusions) against the oracle's sub-cell integration."""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import dogip as odg
from oracle import fem, subcell
from workloads import random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _balls(d, seed, n=3):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 0.8, size=(n, d))
    r = rng.uniform(0.12, 0.3, size=(n, 1))
    return np.hstack([c, r])


def _pack(D, kind, d):
    if kind == "wp":
        return D[:, :, None]
    iu = np.triu_indices(d)
    return D[:, :, iu[0], iu[1]]


CASES = ([(2, 4, k, "se", 3, 3) for k in (1, 2, 3, 4, 5)] + [(2, 4, k, "wp", 3, 3) for k in (1, 2, 3, 4)]
         + [(3, 2, k, "se", 2, 2) for k in (1, 2, 3, 4)] + [(3, 2, k, "wp", 2, 2) for k in (1, 2)])


@pytest.mark.parametrize("d,n,k,kind,depth,ng", CASES)
def test_subcell_d_and_apply_parity(d, n, k, kind, depth, ng):
    from paper_1710_09913_amd import Mesh, Operator, Space

    print(f"[subcell] d={d} n={n} k={k} kind={kind} depth={depth} ng={ng}", flush=True)
    coords, cells = unit_mesh(d, n, jitter=0.1, seed=k)
    balls = _balls(d, seed=k)
    sp = Space(Mesh(coords, cells), k, kind, "dirichlet" if kind == "se" else "none")
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True)
    mp = op.set_inclusions(balls, 9.0, 1.5, depth=depth, ng=ng)
    osp = fem.make_space(coords, cells, k)
    Do = subcell.build_d_subcell(osp, balls, 9.0, 1.5, kind, depth=depth, ng=ng)
    De = op.export_d().cpu().numpy()
    assert np.abs(De - _pack(Do, kind, d)).max() <= 1e-12 * np.abs(Do).max()
    npts = [subcell.subcell_integrals(coords[cells[e]], balls, 2 * k if kind == "wp" else 2 * k - 2, depth, ng)[1]
            for e in range(len(cells))]
    assert abs(mp - np.mean(npts)) <= 1e-9 * max(1.0, np.mean(npts))
    perm = match_dofs(sp.dof_coords(), osp.dof_coords)
    u = random_vector(sp.ndofs, seed=3)
    y = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    uo = np.empty_like(u)
    uo[perm] = u
    yo = (odg.apply_dirichlet if kind == "se" else odg.apply)(osp, Do, uo, kind)[perm]
    assert rel_err(y, yo) <= 1e-11


def test_subcell_solve_and_reset():
    """PCG on the inclusion operator, and set_coef restoring the smooth D."""
    from paper_1710_09913_amd import Mesh, Operator, Space

    sp = Space(Mesh.unit(2, 16), 3, "se", "dirichlet")
    ones = torch.ones(sp.ncells, dtype=torch.float64)
    op = Operator(sp, ones, "scalar", fp32=True)
    u = torch.from_numpy(random_vector(sp.ndofs, seed=1)).cuda()
    y0 = op.apply(u)
    op.set_inclusions(_balls(2, 7, n=5), 100.0, 1.0, depth=3, ng=3)
    b = op.apply(u)
    for mode in ("f64", "mixed"):
        x, st = op.pcg(b, tol=1e-10, mode=mode)
        assert st["status"] == 0 and st["relres_true"] <= 1e-10
    op.set_coef(ones)
    assert float(torch.linalg.norm(op.apply(u) - y0) / torch.linalg.norm(y0)) <= 1e-14


def test_subcell_errors():
    from paper_1710_09913_amd import Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    sp = Space(Mesh.unit(2, 3), 2, "se", "dirichlet")
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar")
    good = np.array([[0.5, 0.5, 0.2]])
    with pytest.raises(DogipError):
        op.set_inclusions(good, 2.0, 1.0, depth=7)
    with pytest.raises(DogipError):
        op.set_inclusions(good, 2.0, 1.0, ng=0)
    with pytest.raises(DogipError):
        op.set_inclusions(np.array([[0.5, 0.5, -0.1]]), 2.0, 1.0)
    with pytest.raises(ValueError):
        op.set_inclusions(np.array([[0.5, 0.5]]), 2.0, 1.0)
    # the coefficient must be positive on both sides (the coarse levels take its logarithm)
    from paper_1710_09913_amd.capi import DOGIP_E_INVALID

    for a_in, a_out in ((0.0, 1.0), (2.0, -1.0), (float("nan"), 1.0)):
        with pytest.raises(DogipError) as e:
            op.set_inclusions(good, a_in, a_out)
        assert e.value.code == DOGIP_E_INVALID
    wp = Space(Mesh.unit(2, 3), 1, "wp", "none")
    g = Operator(wp, torch.ones(wp.ncells, dtype=torch.float64), "scalar", global_w=True)
    with pytest.raises(DogipError):
        g.set_inclusions(good, 2.0, 1.0)
