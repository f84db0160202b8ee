"""Batched persistent launches against the single-operator path and the oracle."""

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import dogip as odg
from oracle import fem
from workloads import batch_spec, coef_uniform, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problems(count, seed, n_lo=4, n_hi=20, tile_waves=None, kind="se"):
    from paper_1710_09913_amd import Mesh, Operator, Space

    spec = batch_spec(count, seed, n_lo=n_lo, n_hi=n_hi)
    ops, meshes = [], []
    for i, (n, k, sub) in enumerate(spec):
        coords, cells = unit_mesh(2, n, jitter=0.1, seed=seed + i)
        a = coef_uniform(len(cells), 1.0, 10.0, seed, sub)
        sp = Space(Mesh(coords, cells), k, kind, "dirichlet" if kind == "se" else "none")
        tw = tile_waves[i % len(tile_waves)] if tile_waves else 0
        ops.append(Operator(sp, torch.from_numpy(a), "scalar", fp32=True, tile_waves=tw))
        meshes.append((coords, cells, a, k))
    print(f"[batch] {count} problems, sizes {[o.ndofs for o in ops]}", flush=True)
    return ops, meshes


@pytest.mark.parametrize("kind", ["se", "wp"])
def test_batch_apply_equals_single_applies(kind):
    from paper_1710_09913_amd import Batch

    ops, _ = _problems(12, 3, tile_waves=[1, 2, 4], kind=kind)
    b = Batch(ops)
    u = torch.from_numpy(random_vector(b.ndofs, 1)).cuda()
    for prec in ("f64", "f32"):
        y = b.apply(u, prec=prec)
        for i, op in enumerate(ops):
            lo, hi = b.offsets[i], b.offsets[i + 1]
            yi = op.apply(u[lo:hi].contiguous(), prec=prec)
            assert torch.equal(y[lo:hi], yi), (prec, i)


def test_batch_apply_matches_oracle():
    from paper_1710_09913_amd import Batch

    ops, meshes = _problems(6, 5)
    b = Batch(ops)
    u = random_vector(b.ndofs, 2)
    y = b.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    for i, (op, (coords, cells, a, k)) in enumerate(zip(ops, meshes)):
        lo, hi = b.offsets[i], b.offsets[i + 1]
        osp = fem.make_space(coords, cells, k)
        perm = match_dofs(op.space.dof_coords(), osp.dof_coords)
        uo = np.empty(hi - lo)
        uo[perm] = u[lo:hi]
        yo = odg.apply_dirichlet(osp, odg.build_d(osp, a, "se"), uo, "se")[perm]
        assert rel_err(y[lo:hi], yo) <= 1e-11


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_batch_pcg(mode):
    """Every problem of the batch reaches the tolerance on its own FP64 residual and agrees
    with the single-operator solve."""
    from paper_1710_09913_amd import Batch

    ops, _ = _problems(16, 7, n_lo=6, n_hi=32)
    b = Batch(ops)
    rhs = torch.ones(b.ndofs, dtype=torch.float64, device="cuda")
    for i, op in enumerate(ops):
        lo = int(b.offsets[i])
        rhs[torch.from_numpy(op.space.boundary().astype(np.int64) + lo).cuda()] = 0.0
    x, stats = b.pcg(rhs, tol=1e-9, maxit=4000, mode=mode)
    for i, op in enumerate(ops):
        lo, hi = b.offsets[i], b.offsets[i + 1]
        st = stats[i]
        assert st["status"] == 0 and st["relres_true"] <= 1e-9, (i, st)
        xi, si = op.pcg(rhs[lo:hi].contiguous(), tol=1e-9, maxit=4000)
        assert rel_err(x[lo:hi].cpu().numpy(), xi.cpu().numpy()) <= 1e-6
        assert abs(st["iters"] - si["iters"]) <= 0.1 * si["iters"] + 20


def test_batch_errors():
    from paper_1710_09913_amd import Batch, Mesh, Operator, Space
    from paper_1710_09913_amd.capi import DogipError

    s3 = Space(Mesh.unit(3, 2), 2, "se", "dirichlet")
    op3 = Operator(s3, torch.ones(48, dtype=torch.float64), "scalar")
    with pytest.raises(DogipError):
        Batch([op3])
    s5 = Space(Mesh.unit(2, 3), 5, "se", "dirichlet")
    op5 = Operator(s5, torch.ones(18, dtype=torch.float64), "scalar")
    with pytest.raises(DogipError):
        Batch([op5])
    ops, _ = _problems(2, 1)
    b = Batch(ops)
    rhs = torch.ones(b.ndofs, dtype=torch.float64, device="cuda")
    with pytest.raises(DogipError):
        b.pcg(rhs, x=torch.zeros_like(rhs))


def test_batch_fullsize_in_bench_configuration():
    """The batch workload at its full size (256 problems, 34.6M dofs, tuned tiles, one
    persistent launch): the batched apply equals each problem's own apply bit for bit
    on a sample of problems, in FP64 and FP32, and the smallest problems match the
    oracle's Algorithm 1."""
    import bench

    ops, bt, coefs = bench.c5_problems(0)
    print(f"[batch full] {len(ops)} problems, {bt.ndofs} dofs", flush=True)
    u = torch.from_numpy(random_vector(bt.ndofs, 4)).cuda()
    rng = np.random.default_rng(9)
    pick = rng.choice(len(ops), 16, replace=False)
    for prec in ("f64", "f32"):
        y = bt.apply(u, prec=prec)
        for i in pick:
            lo, hi = int(bt.offsets[i]), int(bt.offsets[i + 1])
            assert torch.equal(y[lo:hi], ops[i].apply(u[lo:hi].contiguous(), prec=prec)), (prec, i)
    y = bt.apply(u).cpu().numpy()
    uh = u.cpu().numpy()
    for i in np.argsort([op.ndofs for op in ops])[:3]:
        op = ops[i]
        lo, hi = int(bt.offsets[i]), int(bt.offsets[i + 1])
        n = int(round(np.sqrt(op.space.ncells / 2)))
        coords, cells = unit_mesh(2, n)
        osp = fem.make_space(coords, cells, op.space.info["k"])
        perm = match_dofs(op.space.dof_coords(), osp.dof_coords)
        uo = np.empty(hi - lo)
        uo[perm] = uh[lo:hi]
        yo = odg.apply_dirichlet(osp, odg.build_d(osp, coefs[i], "se"), uo, "se")[perm]
        assert rel_err(y[lo:hi], yo) <= 1e-11
