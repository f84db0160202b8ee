"""Python handles over libdogip.  Device memory and streams come from torch; every
step of the method runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import capi
from .capi import check, lib

__all__ = ["Mesh", "Space", "Operator", "Batch", "stream_ptr", "quadrature_rule", "KIND", "BC", "COEF"]

KIND = {"wp": capi.DOGIP_WP, "se": capi.DOGIP_SE}
BC = {"none": capi.DOGIP_BC_NONE, "dirichlet": capi.DOGIP_BC_DIRICHLET0}
COEF = {"scalar": capi.DOGIP_COEF_SCALAR, "sym": capi.DOGIP_COEF_SYM, "logscalar": capi.DOGIP_COEF_LOGSCALAR,
        "raw_d": capi.DOGIP_COEF_RAW_D}
PREC = {"f64": capi.DOGIP_F64, "f32": capi.DOGIP_F32}
SOLVE = {"f64": capi.DOGIP_SOLVE_F64, "mixed": capi.DOGIP_SOLVE_MIXED, "mixed_restart": capi.DOGIP_SOLVE_MIXED_RESTART,
         "pmg": capi.DOGIP_SOLVE_PMG, "pmg_mixed": capi.DOGIP_SOLVE_PMG_MIXED,
         "mixed_v64": capi.DOGIP_SOLVE_MIXED_V64}


def stream_ptr(stream=None) -> int:
    """hipStream_t of a torch stream (default: the current stream of the current device)."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t, dtype=None, n=None) -> int:
    import torch

    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return t.data_ptr()


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def quadrature_rule(dim: int, n: int):
    """Reference points [n^dim, dim] and weights [n^dim] of the quadrature-point operator
    (collapsed Gauss-Legendre, n points per direction)."""
    pts = np.empty((n ** dim, dim))
    wts = np.empty(n ** dim)
    check(lib().dogip_quadrature(dim, n, pts.ctypes.data_as(C.c_void_p), wts.ctypes.data_as(C.c_void_p)))
    return pts, wts


class Mesh:
    """dogip_mesh: simplex mesh (host copy inside the library)."""

    def __init__(self, coords, cells, _handle=None):
        if _handle is not None:
            self.h = _handle
        else:
            xyz, px = _host(coords, np.float64)
            cl, pc = _host(cells, np.int32)
            h = C.c_void_p()
            check(lib().dogip_mesh_create(xyz.shape[1], xyz.shape[0], px, cl.shape[0], pc, C.byref(h)))
            self.h = h
        d, nv, nc = C.c_int(), C.c_int64(), C.c_int64()
        check(lib().dogip_mesh_info(self.h, C.byref(d), C.byref(nv), C.byref(nc)))
        self.dim, self.nv, self.nc = d.value, nv.value, nc.value

    @classmethod
    def unit(cls, dim: int, n: int) -> "Mesh":
        h = C.c_void_p()
        check(lib().dogip_mesh_unit(dim, n, C.byref(h)))
        return cls(None, None, _handle=h)

    def copy(self):
        xyz = np.empty((self.nv, self.dim))
        cells = np.empty((self.nc, self.dim + 1), np.int32)
        check(lib().dogip_mesh_copy(self.h, xyz.ctypes.data_as(C.c_void_p), cells.ctypes.data_as(C.c_void_p)))
        return xyz, cells

    def __del__(self):
        if getattr(self, "h", None) and capi._lib is not None:
            capi._lib.dogip_mesh_destroy(self.h)
            self.h = None


class Space:
    """dogip_space: C_{N,k} with the double-grid space of the problem kind."""

    def __init__(self, mesh: Mesh, k: int, kind: str = "se", bc: str = "dirichlet"):
        h = C.c_void_p()
        check(lib().dogip_space_create(mesh.h, k, KIND[kind], BC[bc], C.byref(h)))
        self.h = h
        self.mesh = mesh
        info = capi.SpaceInfo()
        check(lib().dogip_space_get_info(self.h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in capi.SpaceInfo._fields_}
        self.ndofs = info.ndofs
        self.ncells = info.ncells
        self.kind = kind

    def dof_coords(self):
        out = np.empty((self.ndofs, self.info["dim"]))
        check(lib().dogip_space_dof_coords(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def cell_dofs(self):
        out = np.empty((self.ncells, self.info["vt"]), np.int32)
        check(lib().dogip_space_cell_dofs(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def boundary(self):
        out = np.empty(self.info["nboundary"], np.int32)
        check(lib().dogip_space_boundary(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def bhat(self):
        i = self.info
        b = np.empty((i["nb"], i["wt"], i["vt"]))
        w = np.empty(i["wt"])
        check(lib().dogip_space_bhat(self.h, b.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)))
        return b, w

    def bhat_factors(self):
        """The factors of the elliptic B^ applied by DOGIP_VARIANT_FACTORED: b1 [dim][n1][vt]
        (gradient of the basis at the P_{k-1} lattice), b2 [wt][n1] (P_{k-1} basis at the W
        nodes)."""
        i = self.info
        n1 = math.comb(i["k"] - 1 + i["dim"], i["dim"])
        b1 = np.empty((i["dim"], n1, i["vt"]))
        b2 = np.empty((i["wt"], n1))
        check(lib().dogip_space_bhat_factors(self.h, b1.ctypes.data_as(C.c_void_p), b2.ctypes.data_as(C.c_void_p)))
        return b1, b2

    def __del__(self):
        if getattr(self, "h", None) and capi._lib is not None:
            capi._lib.dogip_space_destroy(self.h)
            self.h = None


class Operator:
    """dogip_op: D on the device plus tiles and the Jacobi diagonal."""

    def __init__(self, space: Space, coef, coef_kind: str = "scalar", fp32: bool = True, tile_waves: int = 0,
                 variant: int = 0, stream=None, global_w: bool = False):
        """global_w: the global projection form (Theorem 1), one D value per dof of
        C_{N,2k} instead of one per cell and node (projection spaces only)."""
        import torch

        self.space = space
        self.ndofs = space.ndofs
        coef = coef.to(device="cuda", dtype=torch.float64).contiguous()
        self._check_coef(coef, coef_kind)
        h = C.c_void_p()
        flags = (capi.DOGIP_OP_FP32 if fp32 else 0) | (capi.DOGIP_OP_GLOBAL_W if global_w else 0)
        check(lib().dogip_op_create(space.h, COEF[coef_kind], _dev_ptr(coef), flags, tile_waves, variant,
                                    stream_ptr(stream), C.byref(h)))
        self.h = h
        self.refresh_info()

    @classmethod
    def quadrature(cls, space: "Space", n: int, samples, fp32: bool = True, tile_waves: int = 0, stream=None):
        """The conventional quadrature-point operator (dogip_op_create_qp): samples
        [ncells, n^dim] of the scalar coefficient at the mapped points of
        ``quadrature_rule(dim, n)``."""
        import torch

        nq = n ** space.info["dim"]
        samples = samples.to(device="cuda", dtype=torch.float64).contiguous()
        if samples.numel() != nq * space.ncells:
            raise ValueError(f"samples have {samples.numel()} values, expected {nq * space.ncells}")
        self = cls.__new__(cls)
        self.space = space
        self.ndofs = space.ndofs
        h = C.c_void_p()
        check(lib().dogip_op_create_qp(space.h, n, _dev_ptr(samples), capi.DOGIP_OP_FP32 if fp32 else 0, tile_waves,
                                       stream_ptr(stream), C.byref(h)))
        self.h = h
        self.refresh_info()
        return self

    def _check_coef(self, coef, coef_kind):
        i = self.space.info
        per = {"scalar": 1, "logscalar": 1, "sym": i["nsym"], "raw_d": i["wt"] * i["nsym"]}[coef_kind]
        if coef_kind == "sym" and self.space.kind == "wp":
            return  # rejected by the library with DOGIP_E_RANGE
        if coef.numel() != per * i["ncells"]:
            raise ValueError(f"coefficient has {coef.numel()} values, expected {per * i['ncells']}")

    def refresh_info(self):
        info = capi.OpInfo()
        check(lib().dogip_op_get_info(self.h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in capi.OpInfo._fields_}

    def set_inclusions(self, balls, a_in: float, a_out: float, depth: int = 3, ng: int = 3, stream=None):
        """D for a = a_in inside the balls ([nballs, dim+1]: center, radius), a_out elsewhere,
        by sub-cell quadrature (dogip_op_set_inclusions); returns the mean number of
        quadrature points evaluated per cell."""
        b = np.ascontiguousarray(balls, dtype=np.float64)
        if b.ndim != 2 or b.shape[1] != self.space.info["dim"] + 1:
            raise ValueError("balls must be [nballs, dim + 1]")
        mp = C.c_double()
        check(lib().dogip_op_set_inclusions(self.h, b.shape[0], b.ctypes.data_as(C.c_void_p), float(a_in),
                                            float(a_out), depth, ng, C.byref(mp), stream_ptr(stream)))
        return mp.value

    def set_coef(self, coef, coef_kind: str = "scalar", stream=None):
        import torch

        coef = coef.to(device="cuda", dtype=torch.float64).contiguous()
        self._check_coef(coef, coef_kind)
        check(lib().dogip_op_set_coef(self.h, COEF[coef_kind], _dev_ptr(coef), stream_ptr(stream)))
        torch.cuda.current_stream().synchronize()

    def set_tile_lanes(self, lanes64: int = 0, lanes32: int = 0):
        """Lanes of the workgroup that takes one tile of the FP64 / FP32 apply (0: chosen for
        occupancy); the results do not depend on it."""
        check(lib().dogip_op_set_tile_lanes(self.h, int(lanes64), int(lanes32)))

    def apply(self, u, y=None, prec: str = "f64", stream=None):
        import torch

        if y is None:
            y = torch.empty_like(u)
        check(lib().dogip_apply(self.h, _dev_ptr(u, torch.float64, self.ndofs), _dev_ptr(y, torch.float64, self.ndofs),
                                PREC[prec], stream_ptr(stream)))
        return y

    def apply_noalloc(self, u, y, prec: str = "f64", stream=None):
        """dogip_apply_noalloc: the apply with the library's static staging buffer (no
        device allocation in the call); y must be given."""
        import torch

        check(lib().dogip_apply_noalloc(self.h, _dev_ptr(u, torch.float64, self.ndofs),
                                        _dev_ptr(y, torch.float64, self.ndofs), PREC[prec], stream_ptr(stream)))
        return y

    def diag(self, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(self.ndofs, dtype=torch.float64, device="cuda")
        check(lib().dogip_diag(self.h, _dev_ptr(out, torch.float64, self.ndofs), stream_ptr(stream)))
        return out

    def export_d(self, stream=None):
        import torch

        i = self.space.info
        out = torch.empty((i["ncells"], i["wt"], i["nsym"]), dtype=torch.float64, device="cuda")
        check(lib().dogip_op_export_d(self.h, _dev_ptr(out), stream_ptr(stream)))
        return out

    def pcg(self, b, x=None, tol=1e-8, maxit=20000, mode="f64", inner_tol=0.0, max_outer=20, check_every=16,
            stream=None, raise_on_error=True):
        """Solve A x = b (dogip_pcg); returns (x, stats).  mode: "f64" (Jacobi-PCG),
        "mixed" (FP32 apply and vectors, FP64 residual replacement), "mixed_v64" (the
        same with r, p and A p in FP64: only the apply is FP32), "mixed_restart"
        (FP64 refinement around restarted FP32 solves), "pmg" / "pmg_mixed" (flexible CG
        preconditioned by a multigrid V-cycle over the orders k..1 and, for the elliptic
        problem on a unit mesh, over halved meshes; FP64 or FP32 applies inside the
        cycle).  x, when given, is the start and is overwritten."""
        import torch

        x0 = x is not None
        if x is None:
            x = torch.zeros_like(b)
        o = capi.SolveOpts(tol=tol, maxit=maxit, mode=SOLVE[mode],
                           inner_tol=inner_tol, max_outer=max_outer, check_every=check_every, x0_given=int(x0))
        st = capi.SolveStats()
        rc = lib().dogip_pcg(self.h, _dev_ptr(b, torch.float64, self.ndofs), _dev_ptr(x, torch.float64, self.ndofs),
                             C.byref(o), C.byref(st), stream_ptr(stream))
        stats = {f: getattr(st, f) for f, _ in capi.SolveStats._fields_ if f != "pad0"}
        if raise_on_error and rc != capi.DOGIP_OK:
            check(rc)
        return x, stats

    def grad_logcoef(self, u, lam, g=None, stream=None):
        import torch

        if g is None:
            g = torch.empty(self.space.ncells, dtype=torch.float64, device="cuda")
        check(lib().dogip_grad_logcoef(self.h, _dev_ptr(u, torch.float64, self.ndofs),
                                       _dev_ptr(lam, torch.float64, self.ndofs),
                                       _dev_ptr(g, torch.float64, self.space.ncells), stream_ptr(stream)))
        return g

    def timer_enable(self, on=True):
        check(lib().dogip_op_timer_enable(self.h, int(on)))

    def timer_read(self):
        """(tile kernel ms, finish kernel ms, applies) summed since the last read."""
        ms, fin, n = C.c_double(), C.c_double(), C.c_int64()
        check(lib().dogip_op_timer_read(self.h, C.byref(ms), C.byref(fin), C.byref(n)))
        return ms.value, fin.value, n.value

    def __del__(self):
        if getattr(self, "h", None) and capi._lib is not None:
            capi._lib.dogip_op_destroy(self.h)
            self.h = None


class Batch:
    """dogip_batch: operators applied and solved together in persistent launches."""

    def __init__(self, ops, stream=None):
        self.ops = list(ops)
        arr = (C.c_void_p * len(self.ops))(*[o.h.value for o in self.ops])
        h = C.c_void_p()
        check(lib().dogip_batch_create(arr, len(self.ops), stream_ptr(stream), C.byref(h)))
        self.h = h
        offs = (C.c_int64 * (len(self.ops) + 1))()
        check(lib().dogip_batch_offsets(self.h, offs))
        self.offsets = np.array(list(offs), dtype=np.int64)
        self.ndofs = int(self.offsets[-1])

    def apply(self, u, y=None, prec="f64", stream=None):
        import torch

        if y is None:
            y = torch.empty_like(u)
        check(lib().dogip_batch_apply(self.h, _dev_ptr(u, torch.float64, self.ndofs),
                                      _dev_ptr(y, torch.float64, self.ndofs), PREC[prec], stream_ptr(stream)))
        return y

    def pcg(self, b, x=None, tol=1e-8, maxit=20000, mode="f64", inner_tol=0.0, max_outer=20, check_every=16,
            stream=None, raise_on_error=True):
        import torch

        x0 = x is not None
        if x is None:
            x = torch.zeros_like(b)
        o = capi.SolveOpts(tol=tol, maxit=maxit, mode=SOLVE[mode],
                           inner_tol=inner_tol, max_outer=max_outer, check_every=check_every, x0_given=int(x0))
        st = (capi.SolveStats * len(self.ops))()
        rc = lib().dogip_batch_pcg(self.h, _dev_ptr(b, torch.float64, self.ndofs),
                                   _dev_ptr(x, torch.float64, self.ndofs), C.byref(o), st, stream_ptr(stream))
        stats = [{f: getattr(s, f) for f, _ in capi.SolveStats._fields_ if f != "pad0"} for s in st]
        if raise_on_error and rc != capi.DOGIP_OK:
            check(rc)
        return x, stats

    def __del__(self):
        if getattr(self, "h", None) and capi._lib is not None:
            capi._lib.dogip_batch_destroy(self.h)
            self.h = None
