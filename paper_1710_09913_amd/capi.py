"""ctypes declarations of libdogip (include/dogip.h), one Python name per C function.

Argument marshalling only: every computation happens in the library.  Loading
fails loudly when libdogip.so has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DOGIP_LIBRARY selects another build of the same library (for instance a tuning variant)
LIB_PATH = os.environ.get("DOGIP_LIBRARY") or os.path.join(HERE, "libdogip.so")

# status codes and enums (include/dogip.h)
DOGIP_OK = 0
DOGIP_E_INVALID = 1
DOGIP_E_RANGE = 2
DOGIP_E_NULL = 3
DOGIP_E_HIP = 4
DOGIP_E_NOMEM = 5
DOGIP_E_NOT_CONVERGED = 6
DOGIP_E_BREAKDOWN = 7
DOGIP_E_NONFINITE = 8
DOGIP_E_STATE = 9
DOGIP_WP = 0
DOGIP_SE = 1
DOGIP_BC_NONE = 0
DOGIP_BC_DIRICHLET0 = 1
DOGIP_COEF_SCALAR = 0
DOGIP_COEF_SYM = 1
DOGIP_COEF_LOGSCALAR = 2
DOGIP_COEF_RAW_D = 3
DOGIP_F64 = 0
DOGIP_F32 = 1
DOGIP_SOLVE_F64 = 0
DOGIP_SOLVE_MIXED = 1
DOGIP_SOLVE_MIXED_RESTART = 2
DOGIP_SOLVE_PMG = 3
DOGIP_SOLVE_PMG_MIXED = 4
DOGIP_SOLVE_MIXED_V64 = 5
DOGIP_OP_FP32 = 1
DOGIP_OP_GLOBAL_W = 2
DOGIP_VARIANT_AUTO = 0
DOGIP_VARIANT_UNROLLED = 1
DOGIP_VARIANT_LOOPED = 2
DOGIP_VARIANT_MFMA = 3
DOGIP_VARIANT_FACTORED = 4
DOGIP_NOALLOC_MAX_STAGE = 1 << 22


class SpaceInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("k", C.c_int32), ("kind", C.c_int32), ("bc", C.c_int32),
                ("ncells", C.c_int64), ("ndofs", C.c_int64), ("nboundary", C.c_int64),
                ("vt", C.c_int32), ("wt", C.c_int32), ("nsym", C.c_int32), ("nb", C.c_int32),
                ("nnz_bhat", C.c_int64), ("nnz_pm1_bhat", C.c_int64)]


class OpInfo(C.Structure):
    _fields_ = [("tile_cells", C.c_int32), ("variant", C.c_int32), ("has_fp32", C.c_int32), ("nq", C.c_int32),
                ("ntiles", C.c_int64), ("tile_dofs_total", C.c_int64), ("nshared", C.c_int64),
                ("max_tile_dofs", C.c_int64), ("bytes_d64", C.c_int64), ("bytes_d32", C.c_int64),
                ("bytes_index", C.c_int64), ("alg_bytes_f64", C.c_double), ("alg_bytes_f32", C.c_double),
                ("alg_flops", C.c_double), ("ndofs_w", C.c_int64),
                ("stage_entries", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("mode", C.c_int32), ("inner_tol", C.c_double),
                ("max_outer", C.c_int32), ("check_every", C.c_int32), ("x0_given", C.c_int32), ("pad0", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("outer", C.c_int32), ("pad0", C.c_int32),
                ("relres", C.c_double), ("relres_true", C.c_double), ("seconds", C.c_double)]


H = C.c_void_p  # opaque handles
P = C.c_void_p  # device or host pointers
PH = C.POINTER(C.c_void_p)

# name -> (restype, argtypes), in header order
SIGNATURES = {
    "dogip_last_error": (C.c_char_p, []),
    "dogip_version": (C.c_int, []),
    "dogip_device_count": (C.c_int, []),
    "dogip_check_tables": (C.c_int, [C.POINTER(C.c_int64)]),
    "dogip_mesh_create": (C.c_int, [C.c_int, C.c_int64, P, C.c_int64, P, PH]),
    "dogip_mesh_unit": (C.c_int, [C.c_int, C.c_int, PH]),
    "dogip_mesh_info": (C.c_int, [H, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dogip_mesh_copy": (C.c_int, [H, P, P]),
    "dogip_mesh_destroy": (None, [H]),
    "dogip_space_create": (C.c_int, [H, C.c_int, C.c_int, C.c_int, PH]),
    "dogip_space_get_info": (C.c_int, [H, C.POINTER(SpaceInfo)]),
    "dogip_space_dof_coords": (C.c_int, [H, P]),
    "dogip_space_cell_dofs": (C.c_int, [H, P]),
    "dogip_space_boundary": (C.c_int, [H, P]),
    "dogip_space_bhat": (C.c_int, [H, P, P]),
    "dogip_space_bhat_factors": (C.c_int, [H, P, P]),
    "dogip_space_destroy": (None, [H]),
    "dogip_op_create": (C.c_int, [H, C.c_int, P, C.c_uint, C.c_int, C.c_int, P, PH]),
    "dogip_quadrature": (C.c_int, [C.c_int, C.c_int, P, P]),
    "dogip_op_set_inclusions": (C.c_int, [H, C.c_int, P, C.c_double, C.c_double, C.c_int, C.c_int,
                                          C.POINTER(C.c_double), P]),
    "dogip_op_create_qp": (C.c_int, [H, C.c_int, P, C.c_uint, C.c_int, P, PH]),
    "dogip_op_set_coef": (C.c_int, [H, C.c_int, P, P]),
    "dogip_op_set_tile_lanes": (C.c_int, [H, C.c_int, C.c_int]),
    "dogip_op_get_info": (C.c_int, [H, C.POINTER(OpInfo)]),
    "dogip_op_export_d": (C.c_int, [H, P, P]),
    "dogip_apply": (C.c_int, [H, P, P, C.c_int, P]),
    "dogip_apply_noalloc": (C.c_int, [H, P, P, C.c_int, P]),
    "dogip_diag": (C.c_int, [H, P, P]),
    "dogip_pcg": (C.c_int, [H, P, P, C.POINTER(SolveOpts), C.POINTER(SolveStats), P]),
    "dogip_grad_logcoef": (C.c_int, [H, P, P, P, P]),
    "dogip_op_timer_enable": (C.c_int, [H, C.c_int]),
    "dogip_op_timer_read": (C.c_int, [H, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "dogip_op_destroy": (None, [H]),
    "dogip_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, P, PH]),
    "dogip_batch_offsets": (C.c_int, [H, C.POINTER(C.c_int64)]),
    "dogip_batch_apply": (C.c_int, [H, P, P, C.c_int, P]),
    "dogip_batch_pcg": (C.c_int, [H, P, P, C.POINTER(SolveOpts), C.POINTER(SolveStats), P]),
    "dogip_batch_destroy": (None, [H]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libdogip.so is not built ({LIB_PATH}); run python -m paper_1710_09913_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DogipError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc != DOGIP_OK:
        raise DogipError(rc, lib().dogip_last_error().decode())
    return rc
