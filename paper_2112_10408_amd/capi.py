"""ctypes declarations of the C ABI in include/tnn.h (libtnn.so).

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnn.so")

TNN_OK = 0
TNN_E_ARG = -1
TNN_E_UNSORTED = -2
TNN_E_NONFINITE = -3
TNN_E_WORKSPACE = -4
TNN_E_HIP = -5
TNN_E_UNSUPPORTED = -6
TNN_E_FORMAT = -7

TNN_PLAIN = 0
TNN_BRUTE = 1
TNN_MIXED_BF16 = 2
TNN_LEARNED = 4
TNN_LEARNED_SEED = 16

STAT_NAMES = ["queries", "blocks", "segments", "points", "merges", "rounds", "fallbacks",
              "rescored", "max_err_bits"]
TNN_STAT_COUNT = 16
NOALLOC_SCRATCH_BYTES = 16 << 20  # TNN_NOALLOC_SCRATCH_BYTES

# Radius model (layout of the device blob, see tnn.h)
RADIUS_HIDDEN = 64
RADIUS_INPUTS = 6
RADIUS_GRID = 32
RADIUS_START_XY = 128
RADIUS_START_T = 512
RADIUS_NPARAMS = RADIUS_HIDDEN * RADIUS_INPUTS + RADIUS_HIDDEN + RADIUS_HIDDEN * RADIUS_HIDDEN \
    + RADIUS_HIDDEN + RADIUS_HIDDEN + 1

P = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
f32 = ctypes.c_float
f64 = ctypes.c_double
sz = ctypes.c_size_t


class TnnPoints(ctypes.Structure):
    _fields_ = [("x", P), ("y", P), ("z", P), ("t", P), ("n", i64)]


class TnnIndex(ctypes.Structure):
    _fields_ = [("opaque", u64 * 48)]


class TnnQueryParams(ctypes.Structure):
    _fields_ = [("scale", f64 * 4), ("t_window", f64), ("k", i32), ("flags", u32),
                ("seed_segments", i32), ("waves_per_block", i32), ("d_radius2", P),
                ("d_stats", P), ("d_query_scale", P), ("d_gka_values", P), ("d_gka_out", P),
                ("gka_comp", i32), ("radius_alpha", f32), ("radius_model", P)]


class TnnBatchItem(ctypes.Structure):
    _fields_ = [("index", ctypes.POINTER(TnnIndex)), ("queries", TnnPoints),
                ("params", TnnQueryParams), ("d_out_idx", P), ("d_out_dist", P)]


class TnnBatchConfig(ctypes.Structure):
    _fields_ = [("chunk", i32), ("waves_per_block", i32), ("blocks_per_cu", i32), ("reserved", i32)]


class TnnBatchPlan(ctypes.Structure):
    _fields_ = [("opaque", u64 * 16)]


_SIGS = {
    "tnn_status_string": (ctypes.c_char_p, [i32]),
    "tnn_build_segments_workspace": (i32, [P, i64, i32, ctypes.POINTER(sz)]),
    "tnn_build_segments": (i32, [TnnPoints, P, i64, i32, P, P, sz, P, ctypes.POINTER(TnnIndex)]),
    "tnn_index_info": (i32, [ctypes.POINTER(TnnIndex), ctypes.POINTER(i64), ctypes.POINTER(i64),
                             ctypes.POINTER(i64), ctypes.POINTER(i32)]),
    "tnn_query_workspace": (i32, [ctypes.POINTER(TnnIndex), i64, ctypes.POINTER(TnnQueryParams),
                                  ctypes.POINTER(sz)]),
    "tnn_query": (i32, [ctypes.POINTER(TnnIndex), TnnPoints, ctypes.POINTER(TnnQueryParams), P, P,
                        P, sz, P]),
    "tnn_query_noalloc": (i32, [ctypes.POINTER(TnnIndex), TnnPoints, ctypes.POINTER(TnnQueryParams),
                                P, P, P]),
    "tnn_debug_export_index": (i32, [ctypes.POINTER(TnnIndex), P, P, P, P, P]),
    "tnn_debug_lower_bounds": (i32, [ctypes.POINTER(TnnIndex), TnnPoints, P, f64, P, P, P, P, sz,
                                     P]),
    "tnn_radius_model_bytes": (i32, [ctypes.POINTER(sz)]),
    "tnn_radius_model_init": (i32, [ctypes.POINTER(TnnIndex), P, u64, P]),
    "tnn_radius_train_workspace": (i32, [i64, ctypes.POINTER(sz)]),
    "tnn_radius_shuffle": (i32, [i64, u64, P, P]),
    "tnn_radius_grad": (i32, [P, TnnPoints, P, P, i32, i64, i64, P, P, P, sz, P]),
    "tnn_radius_train_step": (i32, [P, P, TnnPoints, P, P, i32, i64, i64, i32, f32, P, P, sz, P]),
    "tnn_radius_calibrate_workspace": (i32, [i64, ctypes.POINTER(sz)]),
    "tnn_radius_calibrate": (i32, [P, TnnPoints, P, i32, f64, P, P, sz, P]),
    "tnn_radius_checkpoint_bytes": (i32, [ctypes.POINTER(sz)]),
    "tnn_radius_model_save": (i32, [P, P, sz, P]),
    "tnn_radius_model_load": (i32, [P, sz, P, P]),
    "tnn_radius_features": (i32, [P, TnnPoints, P, P]),
    "tnn_radius_infer": (i32, [P, TnnPoints, f32, P, P, P]),
    "tnn_gka_average": (i32, [P, P, i64, i32, P, i32, i64, P, P]),
    "tnn_batch_workspace": (i32, [ctypes.POINTER(TnnBatchItem), i32, ctypes.POINTER(sz)]),
    "tnn_batch_prepare": (i32, [ctypes.POINTER(TnnBatchItem), i32, ctypes.POINTER(TnnBatchConfig),
                                P, sz, P, ctypes.POINTER(TnnBatchPlan)]),
    "tnn_query_batched": (i32, [ctypes.POINTER(TnnBatchPlan), P]),
    "tnn_batch_ticks": (i32, [ctypes.POINTER(TnnBatchPlan), ctypes.POINTER(ctypes.c_void_p)]),
    "tnn_wall_clock_rate_khz": (i32, [ctypes.POINTER(i64)]),
    "tnn_autotune_batched": (i32, [ctypes.POINTER(TnnBatchItem), i32, P, sz, P, ctypes.c_char_p,
                                   ctypes.POINTER(TnnBatchConfig)]),
}

_lib = None


def lib():
    """The loaded libtnn.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_2112_10408_amd.build_lib.build() (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


class TnnError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {lib().tnn_status_string(code).decode()} ({code})")
        self.code = code


def check(code, where):
    if code != TNN_OK:
        raise TnnError(code, where)
