"""ctypes binding of libhaar.so: one Python function per C entry point, same names.

Argument marshalling only -- every transform runs in the HIP kernels of the
library.  Pointers are passed as integers (device addresses), streams as
integers (``hipStream_t`` values, 0 = null stream).  Loading fails loudly if
the library has not been built (``python -m paper_1002_2184_amd.build``);
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhaar.so")

STATUS = {
    0: "HAAR_OK", 1: "HAAR_ERR_NULL", 2: "HAAR_ERR_DTYPE", 3: "HAAR_ERR_SHAPE",
    4: "HAAR_ERR_LEVELS", 5: "HAAR_ERR_ALIAS", 6: "HAAR_ERR_WORKSPACE", 7: "HAAR_ERR_HIP",
    8: "HAAR_ERR_PLAN", 9: "HAAR_ERR_UNSUPPORTED", 10: "HAAR_ERR_ARG",
}


class HaarError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Item1D(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("length", ctypes.c_int64),
                ("levels", ctypes.c_int32)]


class Item2D(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("height", ctypes.c_int64),
                ("width", ctypes.c_int64), ("levels", ctypes.c_int32)]


_lib = None

_VP, _I64, _I32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_FP = ctypes.POINTER(ctypes.c_float)
_SIGS = {
    "haar_fwd_1d": ([_VP, _VP, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_inv_1d": ([_VP, _VP, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_fwd_2d": ([_VP, _VP, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_inv_2d": ([_VP, _VP, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_l1_grad_2d": ([_VP, _VP, _VP, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_l1_grad_2d_noalloc": ([_VP, _VP, _VP, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_fwd_3d": ([_VP, _VP, _I64, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_inv_3d": ([_VP, _VP, _I64, _I64, _I64, _I32, _I64, _I32, _VP], ctypes.c_int),
    "haar_shrink_1d": ([_VP, _VP, _I64, _I32, _I64, _I32, _I32, _FP, _VP], ctypes.c_int),
    "haar_shrink_2d": ([_VP, _VP, _I64, _I64, _I32, _I64, _I32, _I32, _FP, _VP], ctypes.c_int),
    "haar_direct_workspace_size": ([_I64, _I64], ctypes.c_size_t),
    "haar_direct_1d": ([_VP, _VP, _I64, _I32, _I64, _I32, _I32, _VP, _SZ, _VP], ctypes.c_int),
    "haar_max_levels_1d": ([_I64], ctypes.c_int),
    "haar_max_levels_2d": ([_I64, _I64], ctypes.c_int),
    "haar_max_levels_3d": ([_I64, _I64, _I64], ctypes.c_int),
    "haar_plan_create_1d": ([ctypes.POINTER(Item1D), _I64, _I32, _I32, ctypes.POINTER(_VP)], ctypes.c_int),
    "haar_plan_create_2d": ([ctypes.POINTER(Item2D), _I64, _I32, _I32, ctypes.POINTER(_VP)], ctypes.c_int),
    "haar_plan_workspace_size": ([_VP, ctypes.POINTER(_SZ)], ctypes.c_int),
    "haar_plan_upload": ([_VP, _VP, _VP], ctypes.c_int),
    "haar_plan_execute": ([_VP, _VP, _VP], ctypes.c_int),
    "haar_plan_info": ([_VP, ctypes.POINTER(_I64), ctypes.POINTER(_I32)], ctypes.c_int),
    "haar_plan_set_config": ([_VP, _I32], ctypes.c_int),
    "haar_plan_tune": ([_VP, _VP, _VP, ctypes.POINTER(_I32)], ctypes.c_int),
    "haar_plan_destroy": ([_VP], ctypes.c_int),
    "haar_tune_2d": ([_I32, _I32, _I64, _I64, _I32, _I64, _VP, _SZ, _VP, ctypes.POINTER(_I32)], ctypes.c_int),
    "haar_tune_1d": ([_I32, _I32, _I64, _I32, _I64, _VP, _SZ, _VP, ctypes.POINTER(_I32)], ctypes.c_int),
    "haar_tune_save": ([ctypes.c_char_p], ctypes.c_int),
    "haar_tune_load": ([ctypes.c_char_p], ctypes.c_int),
    "haar_tune_candidates_2d": ([_I32], ctypes.c_int),
    "haar_tune_candidate_name": ([_I32, _I32], ctypes.c_char_p),
    "haar_force_config_2d": ([_I32, _I32], ctypes.c_int),
    "haar_force_config_1d": ([_I32, _I32], ctypes.c_int),
    "haar_tune_candidates_1d": ([], ctypes.c_int),
    "haar_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "haar_last_error": ([], ctypes.c_char_p),
    "haar_version": ([], ctypes.c_char_p),
}


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1002_2184_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def check(status: int) -> None:
    """Raise HaarError for a non-OK status."""
    if status != 0:
        raise HaarError(status, lib().haar_last_error().decode(errors="replace"))


# --- one wrapper per entry point (same names, integer pointers) -------------
def haar_fwd_1d(x, y, length, levels, batch, dtype, stream=0):
    return lib().haar_fwd_1d(x, y, length, levels, batch, dtype, stream)


def haar_inv_1d(y, x, length, levels, batch, dtype, stream=0):
    return lib().haar_inv_1d(y, x, length, levels, batch, dtype, stream)


def haar_fwd_2d(x, y, height, width, levels, batch, dtype, stream=0):
    return lib().haar_fwd_2d(x, y, height, width, levels, batch, dtype, stream)


def haar_inv_2d(y, x, height, width, levels, batch, dtype, stream=0):
    return lib().haar_inv_2d(y, x, height, width, levels, batch, dtype, stream)


def haar_l1_grad_2d(x, grad_x, loss, height, width, levels, batch, dtype, stream=0):
    return lib().haar_l1_grad_2d(x, grad_x, loss, height, width, levels, batch, dtype, stream)


def haar_l1_grad_2d_noalloc(x, grad_x, loss, height, width, levels, batch, dtype, stream=0):
    return lib().haar_l1_grad_2d_noalloc(x, grad_x, loss, height, width, levels, batch, dtype, stream)


def haar_fwd_3d(x, y, depth, height, width, levels, batch, dtype, stream=0):
    return lib().haar_fwd_3d(x, y, depth, height, width, levels, batch, dtype, stream)


def haar_inv_3d(y, x, depth, height, width, levels, batch, dtype, stream=0):
    return lib().haar_inv_3d(y, x, depth, height, width, levels, batch, dtype, stream)


def haar_shrink_1d(x, y, length, levels, batch, dtype, mode, thresholds, stream=0):
    """thresholds: a sequence of `levels` floats (copied into a host array)."""
    return lib().haar_shrink_1d(x, y, length, levels, batch, dtype, mode, _floats(thresholds), stream)


def haar_shrink_2d(x, y, height, width, levels, batch, dtype, mode, thresholds, stream=0):
    return lib().haar_shrink_2d(x, y, height, width, levels, batch, dtype, mode, _floats(thresholds),
                                stream)


def haar_direct_workspace_size(length, batch):
    return lib().haar_direct_workspace_size(length, batch)


def haar_direct_1d(x, y, length, levels, batch, dtype, inverse, workspace, workspace_bytes, stream=0):
    return lib().haar_direct_1d(x, y, length, levels, batch, dtype, inverse, workspace, workspace_bytes,
                                stream)


def _floats(values):
    if values is None:
        return None
    vals = [float(v) for v in values]
    return (ctypes.c_float * max(1, len(vals)))(*vals)


def haar_max_levels_1d(length):
    return lib().haar_max_levels_1d(length)


def haar_max_levels_2d(height, width):
    return lib().haar_max_levels_2d(height, width)


def haar_max_levels_3d(depth, height, width):
    return lib().haar_max_levels_3d(depth, height, width)


def haar_plan_create_1d(items, count, dtype, inverse, out_ptr):
    return lib().haar_plan_create_1d(items, count, dtype, inverse, out_ptr)


def haar_plan_create_2d(items, count, dtype, inverse, out_ptr):
    return lib().haar_plan_create_2d(items, count, dtype, inverse, out_ptr)


def haar_plan_workspace_size(plan, out_bytes):
    return lib().haar_plan_workspace_size(plan, out_bytes)


def haar_plan_upload(plan, workspace, stream=0):
    return lib().haar_plan_upload(plan, workspace, stream)


def haar_plan_execute(plan, workspace, stream=0):
    return lib().haar_plan_execute(plan, workspace, stream)


def haar_plan_info(plan, tiles, grid):
    return lib().haar_plan_info(plan, tiles, grid)


def haar_plan_set_config(plan, config):
    return lib().haar_plan_set_config(plan, config)


def haar_plan_tune(plan, workspace, stream, choice):
    return lib().haar_plan_tune(plan, workspace, stream, choice)


def haar_plan_destroy(plan):
    return lib().haar_plan_destroy(plan)


def haar_tune_2d(dtype, inverse, height, width, levels, batch, scratch, scratch_bytes, stream, choice):
    return lib().haar_tune_2d(dtype, inverse, height, width, levels, batch, scratch, scratch_bytes,
                              stream, choice)


def haar_tune_1d(dtype, inverse, length, levels, batch, scratch, scratch_bytes, stream, choice):
    return lib().haar_tune_1d(dtype, inverse, length, levels, batch, scratch, scratch_bytes, stream,
                              choice)


def haar_tune_save(path):
    return lib().haar_tune_save(path.encode() if isinstance(path, str) else path)


def haar_tune_load(path):
    return lib().haar_tune_load(path.encode() if isinstance(path, str) else path)


def haar_tune_candidates_2d(dtype):
    return lib().haar_tune_candidates_2d(dtype)


def haar_tune_candidate_name(dtype, index):
    return lib().haar_tune_candidate_name(dtype, index).decode()


def haar_force_config_2d(dtype, index):
    return lib().haar_force_config_2d(dtype, index)


def haar_force_config_1d(dtype, index):
    return lib().haar_force_config_1d(dtype, index)


def haar_tune_candidates_1d():
    return lib().haar_tune_candidates_1d()


def haar_status_string(status):
    return lib().haar_status_string(status).decode()


def haar_last_error():
    return lib().haar_last_error().decode(errors="replace")


def haar_version():
    return lib().haar_version().decode()
