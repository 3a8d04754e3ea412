"""ctypes view of the C ABI in ``include/dwt_fuse.h`` (libdwtfuse.so).

Marshalling only.  PyTorch's HIP runtime must be loaded before the library
(importing torch first makes the library bind to that runtime, so torch's
stream handles and device pointers are valid inside it); ``load()`` does
this.  There is no fallback: if the library is missing, every entry point
raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdwtfuse.so")

# Every symbol the header declares.
EXPORTS = (
    "dwt_fuse_create", "dwt_fuse_destroy", "dwt_fuse_set_stream", "dwt_fuse_run",
    "dwt_fuse_run_batched", "dwt_fuse_backward", "dwt_fuse_check_run", "dwt_fuse_check_batched",
    "dwt_fuse_check_backward", "dwt_fuse_status_str", "dwt_fuse_last_error", "dwt_fuse_set_tuning",
    "dwt_fuse_tune_save", "dwt_fuse_tune_load", "dwt_fuse_force_tile", "dwt_fuse_run_multipass",
    "dwt_fuse_run_ex", "dwt_fuse_check_run_ex", "dwt_fuse_quality", "dwt_fuse_check_quality",
    "dwt_fuse_force_band_split", "dwt_fuse_backward_batched", "dwt_fuse_check_backward_batched",
    "dwt_fuse_backward_noalloc", "dwt_fuse_force_order", "dwt_fuse_quality_scores",
)

HAAR = 0
D4 = 1
WAVELETS = {"haar": HAAR, "d4": D4}

OK, E_NULL, E_SHAPE, E_WAVELET, E_STRIDE, E_ALIAS, E_NOMEM, E_DEVICE, E_STATE, E_FORMAT = range(10)
STATUS_NAMES = {0: "OK", 1: "E_NULL", 2: "E_SHAPE", 3: "E_WAVELET", 4: "E_STRIDE", 5: "E_ALIAS",
                6: "E_NOMEM", 7: "E_DEVICE", 8: "E_STATE", 9: "E_FORMAT"}
GRAPH = 1
F32 = 0
U8 = 1


class Opts(ctypes.Structure):
    """dwt_fuse_opts."""

    _fields_ = [("in_format", ctypes.c_int32), ("out_format", ctypes.c_int32), ("kappa", ctypes.c_float)]


class Item(ctypes.Structure):
    """dwt_fuse_item."""

    _fields_ = [
        ("wavelet", ctypes.c_int32), ("B", ctypes.c_int32),
        ("H", ctypes.c_int64), ("W", ctypes.c_int64),
        ("pan", ctypes.c_void_p), ("ms", ctypes.c_void_p), ("gain", ctypes.c_void_p), ("out", ctypes.c_void_p),
        ("pan_ld", ctypes.c_int64), ("ms_ld", ctypes.c_int64), ("ms_band_stride", ctypes.c_int64),
        ("out_ld", ctypes.c_int64), ("out_band_stride", ctypes.c_int64),
    ]


class BwdItem(ctypes.Structure):
    """dwt_fuse_bwd_item."""

    _fields_ = [
        ("wavelet", ctypes.c_int32), ("B", ctypes.c_int32),
        ("H", ctypes.c_int64), ("W", ctypes.c_int64),
        ("pan", ctypes.c_void_p), ("gain", ctypes.c_void_p), ("grad_out", ctypes.c_void_p),
        ("grad_pan", ctypes.c_void_p), ("grad_ms", ctypes.c_void_p), ("grad_gain", ctypes.c_void_p),
        ("pan_ld", ctypes.c_int64), ("go_ld", ctypes.c_int64), ("go_band_stride", ctypes.c_int64),
    ]


class DwtFuseError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = STATUS_NAMES.get(status, str(status))
        super().__init__("%s failed: %s%s" % (where, name, (" (" + detail + ")") if detail else ""))


_lock = threading.Lock()
_lib = None


def load(require_torch: bool = True):
    """Load libdwtfuse.so (after torch, so both share one HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdwtfuse.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_1803_00737_amd.build" % LIB_PATH)
        if require_torch:
            import torch  # noqa: F401  (loads torch's HIP runtime first)
        lib = ctypes.CDLL(LIB_PATH)
        i64, i32, vp, st = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int
        lib.dwt_fuse_create.argtypes = [ctypes.POINTER(vp), i32, vp]
        lib.dwt_fuse_create.restype = st
        lib.dwt_fuse_destroy.argtypes = [vp]
        lib.dwt_fuse_destroy.restype = None
        lib.dwt_fuse_set_stream.argtypes = [vp, vp]
        lib.dwt_fuse_set_stream.restype = st
        run_args = [i32, i64, i64, i64, vp, i64, vp, i64, i64, vp, vp, i64, i64]
        lib.dwt_fuse_run.argtypes = [vp] + run_args
        lib.dwt_fuse_run.restype = st
        lib.dwt_fuse_check_run.argtypes = run_args
        lib.dwt_fuse_check_run.restype = st
        lib.dwt_fuse_run_batched.argtypes = [vp, ctypes.POINTER(Item), i64, ctypes.c_uint32]
        lib.dwt_fuse_run_batched.restype = st
        lib.dwt_fuse_check_batched.argtypes = [ctypes.POINTER(Item), i64]
        lib.dwt_fuse_check_batched.restype = st
        bwd_args = [i32, i64, i64, i64, vp, i64, vp, vp, i64, i64, vp, vp, vp]
        lib.dwt_fuse_backward.argtypes = [vp] + bwd_args
        lib.dwt_fuse_backward.restype = st
        lib.dwt_fuse_backward_noalloc.argtypes = [vp] + bwd_args
        lib.dwt_fuse_backward_noalloc.restype = st
        lib.dwt_fuse_check_backward.argtypes = bwd_args
        lib.dwt_fuse_check_backward.restype = st
        lib.dwt_fuse_backward_batched.argtypes = [vp, ctypes.POINTER(BwdItem), i64]
        lib.dwt_fuse_backward_batched.restype = st
        lib.dwt_fuse_check_backward_batched.argtypes = [ctypes.POINTER(BwdItem), i64]
        lib.dwt_fuse_check_backward_batched.restype = st
        lib.dwt_fuse_status_str.argtypes = [st]
        lib.dwt_fuse_status_str.restype = ctypes.c_char_p
        lib.dwt_fuse_last_error.argtypes = [vp]
        lib.dwt_fuse_last_error.restype = ctypes.c_char_p
        lib.dwt_fuse_set_tuning.argtypes = [vp, i32]
        lib.dwt_fuse_set_tuning.restype = st
        lib.dwt_fuse_tune_save.argtypes = [vp, ctypes.c_char_p]
        lib.dwt_fuse_tune_save.restype = st
        lib.dwt_fuse_tune_load.argtypes = [vp, ctypes.c_char_p]
        lib.dwt_fuse_tune_load.restype = st
        lib.dwt_fuse_force_tile.argtypes = [vp, i32, i32, i32, i32]
        lib.dwt_fuse_force_tile.restype = st
        lib.dwt_fuse_force_band_split.argtypes = [vp, i32]
        lib.dwt_fuse_force_band_split.restype = st
        lib.dwt_fuse_force_order.argtypes = [vp, i32]
        lib.dwt_fuse_force_order.restype = st
        lib.dwt_fuse_run_multipass.argtypes = [vp, i32, i64, i64, i64, vp, i64, vp, i64, i64, vp, i64, i64]
        lib.dwt_fuse_run_multipass.restype = st
        ex_args = run_args + [ctypes.POINTER(Opts)]
        lib.dwt_fuse_run_ex.argtypes = [vp] + ex_args
        lib.dwt_fuse_run_ex.restype = st
        lib.dwt_fuse_check_run_ex.argtypes = ex_args
        lib.dwt_fuse_check_run_ex.restype = st
        q_args = [i64, i64, i64, vp, i64, i64, vp, i64, i64, vp]
        lib.dwt_fuse_quality.argtypes = [vp] + q_args
        lib.dwt_fuse_quality.restype = st
        lib.dwt_fuse_quality_scores.argtypes = [vp] + q_args
        lib.dwt_fuse_quality_scores.restype = st
        lib.dwt_fuse_check_quality.argtypes = q_args
        lib.dwt_fuse_check_quality.restype = st
        _lib = lib
        return lib


def wavelet_id(w) -> int:
    if isinstance(w, int) and w in (HAAR, D4):
        return w
    try:
        return WAVELETS[str(w).lower()]
    except KeyError:
        raise ValueError("wavelet must be 'haar' or 'd4', got %r" % (w,))
