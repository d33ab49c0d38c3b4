"""ctypes declarations of libscrooge_hip.so (the C ABI in include/scrooge.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built (``python -m paper_2208_09985_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscrooge_hip.so")

OK, EINVAL, EALPHABET, ERANGE, ENOMEM, EDEVICE, ENOMODEL, EINTERNAL, ELIMIT = 0, -1, -2, -3, -4, -5, -6, -7, -8
NOALLOC_MAX_PAIRS, NOALLOC_MAX_BASES = 65536, 67108864
PAIR_OK, PAIR_NOT_ALIGNED, PAIR_BAD_INPUT, PAIR_ERROR = 0, 1, 2, 3
MODE_PLAIN, MODE_LEARNED, MODE_FIXED = 0, 1, 2
ORDER_INPUT, ORDER_LONGEST_FIRST, ORDER_AUTO = 0, 1, 2
WHERE_HOST, WHERE_DEVICE = 0, 1
INPUT_ASCII, INPUT_PACKED2 = 0, 1
FLAG_GRAPH = 1
FLAG_NO_EARLY_TERMINATION = 2
FLAG_STORE_ALL_COLUMNS = 4
FLAG_ROWS_LDS = 8
FLAG_STORE_EDGES = 16
FLAG_ROW_RING = 32
KERNEL_AUTO, KERNEL_ROWS, KERNEL_COLUMNS, KERNEL_LANES = 0, 1, 2, 3
NFEATURES = 16

EXPORTED = [
    "scg_strerror", "scg_last_hip_error", "scg_params_default", "scg_create", "scg_destroy", "scg_device_cus", "scg_set_model",
    "scg_batch_create", "scg_batch_destroy", "scg_batch_runs_capacity", "scg_batch_runs_offsets",
    "scg_batch_launch_shape",
    "scg_batch_run", "scg_batch_stats", "scg_align", "scg_align_batch", "scg_last_stats", "scg_last_stats_all",
    "scg_runs_to_cigar", "scg_ops_to_cigar",
    "scg_features",
    "scg_mlp_forward", "scg_mlp_backward", "scg_mlp_backward_workspace", "scg_adam_step",
    "scg_align_batch_noalloc",
]


class Params(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("O", ctypes.c_int32), ("k", ctypes.c_int32),
        ("mode", ctypes.c_int32), ("slots", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
        ("order", ctypes.c_int32), ("fixed_rows", ctypes.c_int32), ("tau", ctypes.c_float),
        ("flags", ctypes.c_int32), ("yield_chars", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("one_per_simd", ctypes.c_int32),
        ("offtrack_helpers", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("kernel_ms", ctypes.c_double), ("pack_ms", ctypes.c_double),
        ("kernel_ms_avg", ctypes.c_double), ("pack_ms_avg", ctypes.c_double), ("timed_runs", ctypes.c_int64),
        ("windows", ctypes.c_int64), ("ops_alg", ctypes.c_int64), ("fallback_windows", ctypes.c_int64),
        ("lane_steps", ctypes.c_int64), ("rounds", ctypes.c_int64), ("rows_budgeted", ctypes.c_int64),
        ("yields", ctypes.c_int64),
    ]


class ScgError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        detail = ""
        if code in (EDEVICE, ENOMEM) and _lib is not None:
            detail = " [" + _lib.scg_last_hip_error().decode(errors="replace") + "]"
        super().__init__(f"{what}: {strerror(code)} ({code}){detail}")


_lib = None


def load():
    """Load the in-tree shared library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2208_09985_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "scg_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "scg_last_hip_error": ([], ctypes.c_char_p),
        "scg_params_default": ([ctypes.POINTER(Params)], None),
        "scg_create": ([pp, ctypes.c_int, ctypes.c_char_p], ctypes.c_int),
        "scg_destroy": ([P], None),
        "scg_device_cus": ([P], ctypes.c_int),
        "scg_set_model": ([P, i32, i32, i32, P, P, P, P, P], ctypes.c_int),
        "scg_batch_create": ([P, ctypes.POINTER(Params), i32, P, P, P, P, i32, i32, P, pp], ctypes.c_int),
        "scg_batch_destroy": ([P], None),
        "scg_batch_runs_capacity": ([P], i64),
        "scg_batch_runs_offsets": ([P, P], ctypes.c_int),
        "scg_batch_launch_shape": ([P, P], ctypes.c_int),
        "scg_batch_run": ([P, P, P, P, P, P, P], ctypes.c_int),
        "scg_batch_stats": ([P, ctypes.POINTER(Stats)], ctypes.c_int),
        "scg_align_batch": ([P, ctypes.POINTER(Params), i32, P, P, P, P, i32, i32, P, P, P, P, P, P, P], ctypes.c_int),
        "scg_last_stats": ([P, P, P, P], ctypes.c_int),
        "scg_last_stats_all": ([P, ctypes.POINTER(Stats)], ctypes.c_int),
        "scg_ops_to_cigar": ([P, i32, ctypes.c_char_p, i32, P], ctypes.c_int),
        "scg_align_batch_noalloc": ([P, ctypes.POINTER(Params), i32, P, P, i64, P, P, i64, P, P, P, P, P, P],
                                    ctypes.c_int),
        "scg_align": ([P, ctypes.c_char_p, i32, ctypes.c_char_p, i32, i32, i32, i32, P, P, ctypes.c_char_p, i32, P],
                      ctypes.c_int),
        "scg_runs_to_cigar": ([P, i32, ctypes.c_char_p, i32, P], ctypes.c_int),
        "scg_features": ([P, i32, P, P, P], ctypes.c_int),
        "scg_mlp_forward": ([i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
        "scg_mlp_backward": ([i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, i64, P], ctypes.c_int),
        "scg_mlp_backward_workspace": ([i32, i32, i32], i64),
        "scg_adam_step": ([i32, P, P, P, P, P, f32, f32, f32, f32, i32, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return load().scg_strerror(code).decode()
    except ImportError:
        return f"status {code}"


def check(code: int, what: str) -> None:
    if code != OK:
        raise ScgError(code, what)
