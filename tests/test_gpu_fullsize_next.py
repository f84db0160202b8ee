"""Parity of the quadrature-point operator and of the sub-cell quadrature D at the
benchmark size (3D 64^3 x 6 Kuhn tets, P3 elliptic, zero Dirichlet), in the launch
configuration the benchmark times, on sampled outputs:

  * quadrature-point apply (4 points per direction, the per-cell lognormal value at every
    point): rows of A u at sampled dofs against the oracle's quadrature-assembled rows on
    the sub-mesh around them;
  * inclusions (a = 100 in 64 balls, depth 3, 3^3 points per leaf): D of sampled cells
    against the oracle's sub-cell integration, and the symmetry of the resulting apply.
"""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import fem, subcell
from workloads import coef_lognormal, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, K = 64, 3


@pytest.fixture(scope="module")
def big():
    from paper_1710_09913_amd import Mesh, Space

    print(f"[fullsize-next] 3D {N}^3 P{K} elliptic", flush=True)
    coords, cells = unit_mesh(3, N)
    coef = coef_lognormal(coords, cells, 0)
    space = Space(Mesh.unit(3, N), K, "se", "dirichlet")
    yield {"coords": coords, "cells": cells, "coef": coef, "space": space, "cd": space.cell_dofs(),
           "bnd": space.boundary()}
    torch.cuda.empty_cache()


def _sub_space(b, cells_sel):
    verts, local = np.unique(b["cells"][cells_sel], return_inverse=True)
    osp = fem.make_space(b["coords"][verts], local.reshape(len(cells_sel), -1).astype(b["cells"].dtype), K)
    pid = np.unique(b["cd"][cells_sel])
    perm = match_dofs(b["space"].dof_coords()[pid], osp.dof_coords)
    return osp, pid, perm


def test_quadrature_point_apply_sampled_rows(big):
    from paper_1710_09913_amd import Operator

    b, n = big, 4
    sp = b["space"]
    nq = n ** 3
    samples = torch.from_numpy(b["coef"]).cuda()[:, None].expand(sp.ncells, nq).contiguous()
    op = Operator.quadrature(sp, n, samples)
    del samples
    u = random_vector(sp.ndofs, 0)
    y = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    rng = np.random.default_rng(5)
    s = np.sort(np.setdiff1d(rng.choice(sp.ndofs, 120, replace=False), b["bnd"]))
    sel = np.nonzero(np.isin(b["cd"], s).any(axis=1))[0]
    osp, pid, perm = _sub_space(b, sel)
    A = fem.assemble(osp, fem.element_matrices(osp, b["coef"][sel], "se", nquad=n)).tocsr()
    uo = np.zeros(osp.ndofs)
    uo[perm] = u[pid]
    uo[perm[np.isin(pid, b["bnd"])]] = 0.0
    yo = (A @ uo)[perm[np.searchsorted(pid, s)]]
    assert rel_err(y[s], yo) <= 1e-11
    assert np.abs(y[s] - yo).max() <= 1e-11 * np.abs(yo).max()


def test_inclusions_d_sampled_cells_and_symmetry(big):
    from paper_1710_09913_amd import Operator

    b = big
    sp = b["space"]
    rng = np.random.default_rng(11)
    balls = np.hstack([rng.uniform(0.05, 0.95, size=(64, 3)), rng.uniform(0.04, 0.1, size=(64, 1))])
    op = Operator(sp, torch.ones(sp.ncells, dtype=torch.float64), "scalar", fp32=True)
    op.set_inclusions(balls, 100.0, 1.0, depth=3, ng=3)
    De = op.export_d().cpu().numpy()
    # sampled cells, half of them among the cells a ball boundary cuts
    X = b["coords"][b["cells"]]
    cen = X.mean(axis=1)
    dist = np.linalg.norm(cen[:, None, :] - balls[None, :, :3], axis=2) - balls[None, :, 3]
    near = np.nonzero(np.abs(dist).min(axis=1) < 0.02)[0]
    pick = np.concatenate([rng.choice(near, 24, replace=False), rng.choice(sp.ncells, 24, replace=False)])
    osp, _, _ = _sub_space(b, pick)
    Do = subcell.build_d_subcell(osp, balls, 100.0, 1.0, "se", depth=3, ng=3)
    iu = np.triu_indices(3)
    Dp = Do[:, :, iu[0], iu[1]]
    assert np.abs(De[pick] - Dp).max() <= 1e-12 * np.abs(Dp).max()
    u = torch.from_numpy(random_vector(sp.ndofs, 3)).cuda()
    v = torch.from_numpy(random_vector(sp.ndofs, 4)).cuda()
    au, av = op.apply(u), op.apply(v)
    lhs, rhs = float(torch.dot(v, au)), float(torch.dot(u, av))
    assert abs(lhs - rhs) <= 1e-12 * float(torch.linalg.norm(v) * torch.linalg.norm(au))
