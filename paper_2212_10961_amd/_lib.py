"""ctypes view of the C ABI declared in include/grf.h (argument marshalling only).

The shared library is the in-tree ``libgrf.so`` built by ``build.py``.  Loading fails
loudly when it is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libgrf.so"

GRF_OK, GRF_EINVAL, GRF_ENOMEM, GRF_EDEVICE, GRF_EUNSUPPORTED = 0, -1, -2, -3, -4
GRF_COV_GAUSSIAN, GRF_COV_EXPONENTIAL, GRF_COV_MATERN = 0, 1, 2
GRF_AUTO, GRF_DIRECT_F32, GRF_DIRECT_F64 = -1, 0, 1
GRF_SEP_BF16, GRF_SEP_F16, GRF_SEP_BF16_X3, GRF_SEP_F16_X3 = 2, 3, 4, 5
GRF_DIRECT_F32_BINNED, GRF_DIRECT_F32_POINTWISE = 6, 7
GRF_MAX_THRESHOLDS = 15
GRF_MAX_FACIES = 64
GRF_PLURI_APPLY_WS_BYTES = 512
GRF_PLAN_GRAPH, GRF_PLAN_AUTOTUNE = 1, 2
GRF_NOALLOC_SCRATCH_BYTES = 32 << 20

METHODS = {
    "auto": GRF_AUTO, "direct_f32": GRF_DIRECT_F32, "direct_f64": GRF_DIRECT_F64,
    "sep_bf16": GRF_SEP_BF16, "sep_f16": GRF_SEP_F16, "sep_bf16_x3": GRF_SEP_BF16_X3,
    "sep_f16_x3": GRF_SEP_F16_X3, "direct_f32_binned": GRF_DIRECT_F32_BINNED, "direct_f32_pointwise": GRF_DIRECT_F32_POINTWISE,
}

# Every symbol include/grf.h declares.
EXPORTS = [
    "grf_version", "grf_last_error", "make_modes", "grf_modes_init", "make_modes_lattice", "snap_periodic", "eval_field_grid_ws_size", "eval_field_grid",
    "eval_field_grid_tile", "grf_sep_tile_count", "grf_sep_tile_shape",
    "eval_pluri_grid_ws_size", "eval_pluri_grid", "eval_pluri_points_ws_size", "eval_pluri_points", "pluri_apply",
    "krige_weights_ws_size", "krige_weights", "krige_apply_ws_size", "krige_apply_grid", "krige_apply_points",
    "eval_field_grid_f64", "eval_field_points_ws_size", "eval_field_points", "epilogue_apply",
    "field_backward_ws_size", "field_backward", "field_backward_grid_ws_size", "field_backward_grid",
    "field_backward_grid_method", "grad_z_from_k",
    "grf_plan_create", "grf_plan_destroy", "eval_field_batch", "grf_plan_info",
    "grf_kernel_timer_enable", "grf_kernel_timer_read", "eval_field_grid_noalloc",
]


class GrfSpec(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("cov", ctypes.c_int32), ("sigma2", ctypes.c_double),
                ("mu", ctypes.c_double), ("ell", ctypes.c_double * 3), ("n_modes", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("len_convention", ctypes.c_int32), ("nu", ctypes.c_double)]


class GrfModes(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad_", ctypes.c_int32), ("n", ctypes.c_int64),
                ("z", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("sigma", ctypes.c_double),
                ("ell", ctypes.c_double * 3), ("rotated", ctypes.c_int32), ("pad2_", ctypes.c_int32),
                ("rot", ctypes.c_double * 9), ("w", ctypes.c_void_p)]


class GrfGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 3), ("origin", ctypes.c_double * 3), ("h", ctypes.c_double * 3)]


class GrfEpi(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_float), ("n_thresholds", ctypes.c_int32),
                ("thresholds", ctypes.c_float * GRF_MAX_THRESHOLDS)]


class GrfTrunc2(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int32), ("t", ctypes.c_float * GRF_MAX_THRESHOLDS),
                ("n_s", ctypes.c_int32), ("s", ctypes.c_float * GRF_MAX_THRESHOLDS),
                ("rule", ctypes.c_uint8 * ((GRF_MAX_THRESHOLDS + 1) ** 2)),
                ("n_values", ctypes.c_int32), ("values", ctypes.c_float * GRF_MAX_FACIES)]


class GrfKrige(ctypes.Structure):
    _fields_ = [("cov", ctypes.c_int32), ("pad_", ctypes.c_int32), ("nu", ctypes.c_double),
                ("nugget", ctypes.c_double)]


class GrfBatchItem(ctypes.Structure):
    _fields_ = [("modes", GrfModes), ("grid", GrfGrid), ("epi", GrfEpi), ("y", ctypes.c_void_p),
                ("k", ctypes.c_void_p), ("ind", ctypes.c_void_p)]


_lib = None


class GrfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[grf {code}] {msg}")
        self.code = code


def load():
    """Load libgrf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(str(LIB_PATH))
    P = ctypes.POINTER
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "grf_version": ([], ctypes.c_int),
        "grf_last_error": ([], ctypes.c_char_p),
        "make_modes": ([P(GrfSpec), vp, vp], ctypes.c_int),
        "grf_modes_init": ([P(GrfSpec), vp, vp, P(GrfModes)], ctypes.c_int),
        "snap_periodic": ([ctypes.c_int, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "make_modes_lattice": ([P(GrfSpec), i32, ctypes.c_double, vp, vp, vp], ctypes.c_int),
        "eval_field_grid_ws_size": ([P(GrfModes), P(GrfGrid), ctypes.c_int, P(sz)], ctypes.c_int),
        "eval_field_grid": ([P(GrfModes), P(GrfGrid), ctypes.c_int, P(GrfEpi), vp, vp, vp, vp, sz, vp],
                            ctypes.c_int),
        "eval_field_grid_tile": ([P(GrfModes), P(GrfGrid), ctypes.c_int, ctypes.c_int, P(GrfEpi), vp, vp, vp,
                                  vp, sz, vp], ctypes.c_int),
        "grf_sep_tile_count": ([], ctypes.c_int),
        "grf_sep_tile_shape": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, P(i32), P(i32), P(i32)], ctypes.c_int),
        "eval_pluri_grid_ws_size": ([P(GrfModes), P(GrfModes), P(GrfGrid), ctypes.c_int, P(sz)], ctypes.c_int),
        "eval_pluri_grid": ([P(GrfModes), P(GrfModes), P(GrfGrid), ctypes.c_int, P(GrfTrunc2), vp, vp, vp, vp, vp,
                             sz, vp], ctypes.c_int),
        "eval_pluri_points_ws_size": ([P(GrfModes), P(GrfModes), i64, ctypes.c_int, P(sz)], ctypes.c_int),
        "eval_pluri_points": ([P(GrfModes), P(GrfModes), vp, i64, ctypes.c_int, P(GrfTrunc2), vp, vp, vp, vp, vp,
                               sz, vp], ctypes.c_int),
        "pluri_apply": ([vp, vp, i64, P(GrfTrunc2), vp, vp, vp, sz, vp], ctypes.c_int),
        "krige_weights_ws_size": ([P(GrfModes), i64, P(sz)], ctypes.c_int),
        "krige_weights": ([P(GrfModes), P(GrfKrige), vp, vp, i64, vp, vp, vp, sz, vp], ctypes.c_int),
        "krige_apply_ws_size": ([i64, P(sz)], ctypes.c_int),
        "krige_apply_grid": ([P(GrfModes), P(GrfKrige), vp, vp, i64, P(GrfGrid), vp, vp, sz, vp], ctypes.c_int),
        "krige_apply_points": ([P(GrfModes), P(GrfKrige), vp, vp, i64, vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "eval_field_grid_f64": ([P(GrfModes), P(GrfGrid), ctypes.c_double, vp, vp, vp, sz, vp], ctypes.c_int),
        "eval_field_points_ws_size": ([P(GrfModes), i64, ctypes.c_int, P(sz)], ctypes.c_int),
        "eval_field_points": ([P(GrfModes), vp, i64, ctypes.c_int, P(GrfEpi), vp, vp, vp, vp, sz, vp],
                              ctypes.c_int),
        "epilogue_apply": ([vp, i64, P(GrfEpi), vp, vp, vp], ctypes.c_int),
        "field_backward_ws_size": ([P(GrfModes), i64, P(sz)], ctypes.c_int),
        "field_backward": ([P(GrfModes), vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "field_backward_grid_ws_size": ([P(GrfModes), P(GrfGrid), P(sz)], ctypes.c_int),
        "field_backward_grid": ([P(GrfModes), P(GrfGrid), vp, vp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "field_backward_grid_method": ([P(GrfModes), P(GrfGrid), ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, sz, vp],
                                       ctypes.c_int),
        "grad_z_from_k": ([P(GrfModes), vp, vp, vp], ctypes.c_int),
        "grf_plan_create": ([P(vp), ctypes.c_int, ctypes.c_int, ctypes.c_char_p], ctypes.c_int),
        "grf_plan_destroy": ([vp], ctypes.c_int),
        "eval_field_batch": ([vp, P(GrfBatchItem), i32, vp], ctypes.c_int),
        "grf_plan_info": ([vp, P(i32), P(i32), P(i32), P(i64)], ctypes.c_int),
        "eval_field_grid_noalloc": ([P(GrfModes), P(GrfGrid), ctypes.c_int, P(GrfEpi), vp, vp, vp, vp],
                                    ctypes.c_int),
        "grf_kernel_timer_enable": ([ctypes.c_int], ctypes.c_int),
        "grf_kernel_timer_read": ([P(ctypes.c_double), P(i64)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc: int):
    if rc != GRF_OK:
        raise GrfError(rc, load().grf_last_error().decode(errors="replace"))
    return rc
