"""The allocation-free apply (dogip_apply_noalloc) through the C interface: the same
result bit for bit as dogip_apply on two calls in a row, the second on a smaller
operator (the static staging buffer keeps the first call's contents), FP64 and FP32;
against the CPU oracle on the small problem; and the refusal of an operator whose
staging exceeds the static buffer."""

import ctypes as C

import numpy as np
import pytest

from helpers import match_dofs, rel_err
from oracle import dogip as odg
from oracle import fem
from workloads import coef_lognormal, coef_uniform, random_vector, unit_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _call(op, u, y, prec):
    from paper_1710_09913_amd import capi

    L = capi.lib()
    p = capi.DOGIP_F64 if prec == "f64" else capi.DOGIP_F32
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.dogip_apply_noalloc(op.h, C.c_void_p(u.data_ptr()), C.c_void_p(y.data_ptr()), p, s)
    msg = L.dogip_last_error().decode()
    return rc, msg


def _same_as_apply(op, n, seed, prec):
    u = torch.from_numpy(random_vector(n, seed)).cuda()
    y_ref = op.apply(u, prec=prec)
    y = torch.full_like(u, float("nan"))
    rc, msg = _call(op, u, y, prec)
    torch.cuda.synchronize()
    assert rc == 0, msg
    assert torch.equal(y, y_ref), f"{prec}: differs from dogip_apply (max {float((y - y_ref).abs().max())})"
    return u, y


def test_noalloc_apply_two_calls_then_refusal():
    from paper_1710_09913_amd import Mesh, Operator, Space, capi

    torch.cuda.set_device(0)
    # first call: the 3D 64^3 P3 elliptic operator with its default 512-cell tiles
    print("[noalloc] 3D 64^3 P3 se, default tiles", flush=True)
    coords, cells = unit_mesh(3, 64)
    coef = coef_lognormal(coords, cells, 0)
    big_space = Space(Mesh.unit(3, 64), 3, "se", "dirichlet")
    big = Operator(big_space, torch.from_numpy(coef), "scalar", fp32=True)
    assert 0 < big.info["stage_entries"] <= capi.DOGIP_NOALLOC_MAX_STAGE
    for prec in ("f64", "f32"):
        _same_as_apply(big, big_space.ndofs, 1, prec)

    # second call: a smaller operator (2D 12^2 P2, jittered), also against the oracle
    print("[noalloc] 2D 12^2 P2 se, jittered", flush=True)
    c2, e2 = unit_mesh(2, 12, jitter=0.12, seed=3)
    a2 = coef_uniform(len(e2), 1.0, 10.0, 3)
    sp = Space(Mesh(c2, e2), 2, "se", "dirichlet")
    small = Operator(sp, torch.from_numpy(a2), "scalar", fp32=True, tile_waves=1)
    assert small.info["stage_entries"] < big.info["stage_entries"]
    for prec in ("f64", "f32"):
        u, y = _same_as_apply(small, sp.ndofs, 2, prec)
        if prec == "f64":
            osp = fem.make_space(c2, e2, 2)
            perm = match_dofs(sp.dof_coords(), osp.dof_coords)
            uo = np.empty(sp.ndofs)
            uo[perm] = u.cpu().numpy()
            yo = odg.apply_dirichlet(osp, odg.build_d(osp, a2, "se"), uo, "se")[perm]
            assert rel_err(y.cpu().numpy(), yo) <= 1e-12

    # the first operator again after the smaller one
    _same_as_apply(big, big_space.ndofs, 4, "f64")

    # 64-cell tiles on the 64^3 P3 space stage more partial sums than the buffer holds
    print("[noalloc] 3D 64^3 P3 se, 64-cell tiles (refused)", flush=True)
    del big
    torch.cuda.empty_cache()
    wide = Operator(big_space, torch.from_numpy(coef), "scalar", fp32=False, tile_waves=1)
    assert wide.info["stage_entries"] > capi.DOGIP_NOALLOC_MAX_STAGE
    u = torch.from_numpy(random_vector(big_space.ndofs, 5)).cuda()
    y = torch.zeros_like(u)
    rc, msg = _call(wide, u, y, "f64")
    torch.cuda.synchronize()
    assert rc == capi.DOGIP_E_RANGE and "static scratch" in msg, (rc, msg)
    assert int(torch.count_nonzero(y)) == 0
