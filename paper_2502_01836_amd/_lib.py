"""ctypes binding of libleafi (include/leafi.h).

Argument marshalling only: tensors become device pointers, the current torch
stream becomes the hipStream_t, and C structs are filled from keyword
arguments.  Every computation runs in the HIP library; if the library is not
built this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleafi.so")

LEAFI_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "ESTATE", -4: "EHIP", -5: "EAGAIN", -6: "EINTERNAL"}

LEAFI_SCAN_BF16 = 0
LEAFI_SCAN_FP32 = 1
LEAFI_SEARCH_NO_GRAPH = 1
LEAFI_SEARCH_HOST_ROUNDS = 2
LEAFI_SEARCH_FILTER_TILE_SMALL = 4
LEAFI_SEARCH_FILTER_TILE_LARGE = 8
LEAFI_CALIB_STEP = 0
LEAFI_CALIB_STEFFEN = 1
LEAFI_CALIB_NO_CORRECTION = 2
LEAFI_SELECT_SIZE = 0
LEAFI_SELECT_KNAPSACK = 1
LEAFI_FILTER_MLP = 0
LEAFI_FILTER_CNN = 1


class LeafiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"leafi {ERRORS.get(code, code)}: {msg}")
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_capacity", ctypes.c_int32), ("n_segments", ctypes.c_int32),
                ("split_rule", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_series", ctypes.c_int64), ("m", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("n_segments", ctypes.c_int32), ("n_filters", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("n_calibrated", ctypes.c_int32), ("padded_rows", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("filter_arch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("n_global", ctypes.c_int32), ("n_local", ctypes.c_int32), ("noise_lo", ctypes.c_float),
                ("noise_hi", ctypes.c_float), ("a", ctypes.c_float), ("val_fraction", ctypes.c_float),
                ("th_override", ctypes.c_double), ("mem_budget", ctypes.c_int64), ("hidden", ctypes.c_int32),
                ("max_epochs", ctypes.c_int32), ("lr0", ctypes.c_float), ("lr_min", ctypes.c_float),
                ("batch", ctypes.c_int32), ("patience", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("keep_examples", ctypes.c_int32), ("selection", ctypes.c_int32), ("arch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("t_filter_s", ctypes.c_double), ("t_series_s", ctypes.c_double), ("th", ctypes.c_double),
                ("n_filters", ctypes.c_int32), ("epochs_max_run", ctypes.c_int32), ("ms_collect", ctypes.c_double),
                ("ms_train", ctypes.c_double), ("mean_val_mse", ctypes.c_double)]


class SearchOpts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("scan", ctypes.c_int32), ("use_filters", ctypes.c_int32),
                ("n_schedule", ctypes.c_int32), ("schedule", ctypes.c_int32 * 8), ("kprime", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class SearchStats(ctypes.Structure):
    _fields_ = [("leaves_scanned", ctypes.c_int64), ("leaves_lb_pruned", ctypes.c_int64),
                ("leaves_filter_pruned", ctypes.c_int64), ("series_scanned", ctypes.c_int64),
                ("fallback_items", ctypes.c_int64), ("rounds", ctypes.c_int32), ("path", ctypes.c_int32),
                ("ms_total", ctypes.c_double), ("ms_scan", ctypes.c_double), ("scan_bytes", ctypes.c_double),
                ("filter_evals", ctypes.c_int64)]


LEAFI_TUNE_MAX = 16


class TuneReport(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int32 * LEAFI_TUNE_MAX), ("queries_per_tile", ctypes.c_int32 * LEAFI_TUNE_MAX),
                ("ms", ctypes.c_double * LEAFI_TUNE_MAX)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("k_max", ctypes.c_int32), ("scan", ctypes.c_int32),
                ("use_filters", ctypes.c_int32), ("n_schedule", ctypes.c_int32), ("schedule", ctypes.c_int32 * 8),
                ("queue_capacity", ctypes.c_int32), ("mem_budget", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4)]


class ServerReport(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("rounds", ctypes.c_int64), ("wall_s", ctypes.c_double),
                ("mean_active", ctypes.c_double), ("max_active", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        if name == "reserved":
            continue
        v = getattr(s, name)
        out[name] = list(v) if isinstance(v, ctypes.Array) else v
    return out


# caller-supplied device allocator (leafi_alloc_fn / leafi_free_fn)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p))
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# (name, restype, argtypes) of every entry point declared in include/leafi.h
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F32 = ctypes.c_float
SIGNATURES = [
    ("leafi_create", ctypes.c_int, [ALLOC_FN, FREE_FN, P, ctypes.POINTER(P)]),
    ("leafi_destroy", None, [P]),
    ("leafi_last_error", ctypes.c_char_p, []),
    ("leafi_version", ctypes.c_char_p, []),
    ("leafi_build_index", ctypes.c_int, [P, P, I64, I32, ctypes.POINTER(BuildOpts), P]),
    ("leafi_get_info", ctypes.c_int, [P, ctypes.POINTER(Info)]),
    ("leafi_export_leaves", ctypes.c_int, [P, P, P]),
    ("leafi_export_boxes", ctypes.c_int, [P, P]),
    ("leafi_default_train_opts", None, [ctypes.POINTER(TrainOpts)]),
    ("leafi_train_filters", ctypes.c_int, [P, ctypes.POINTER(TrainOpts), ctypes.POINTER(TrainReport), P]),
    ("leafi_set_filters", ctypes.c_int, [P, I32, I32, P, P, P]),
    ("leafi_set_cnn_filters", ctypes.c_int, [P, I32, I32, P, P, P]),
    ("leafi_get_filters", ctypes.c_int, [P, P, P, P]),
    ("leafi_get_train_trace", ctypes.c_int, [P, ctypes.POINTER(I32), P, P]),
    ("leafi_get_examples", ctypes.c_int, [P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32), P, P, P,
                                          P]),
    ("leafi_calibrate", ctypes.c_int, [P, P, I32, P, I32, P, I32, I32, P]),
    ("leafi_get_offsets", ctypes.c_int, [P, P]),
    ("leafi_set_offsets", ctypes.c_int, [P, P, I32, P, I32, P]),
    ("leafi_default_search_opts", None, [ctypes.POINTER(SearchOpts)]),
    ("leafi_search_knn", ctypes.c_int, [P, P, I64, P, P, ctypes.POINTER(SearchOpts), P, P,
                                        ctypes.POINTER(SearchStats), P]),
    ("leafi_search_knn_noalloc", ctypes.c_int, [P, P, I64, P, P, ctypes.POINTER(SearchOpts), P, P, P]),
    ("leafi_autotune", ctypes.c_int, [P, P, I64, P, P, ctypes.POINTER(SearchOpts), I32, ctypes.POINTER(TuneReport), P]),
    ("leafi_set_tiling", ctypes.c_int, [P, I32, I32]),
    ("leafi_set_plan_capacity", ctypes.c_int, [P, I64]),
    ("leafi_graph_note", ctypes.c_char_p, [P]),
    ("leafi_default_server_opts", None, [ctypes.POINTER(ServerOpts)]),
    ("leafi_server_create", ctypes.c_int, [P, ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]),
    ("leafi_server_destroy", None, [P]),
    ("leafi_server_info", ctypes.c_int, [P, ctypes.POINTER(I32)]),
    ("leafi_server_submit", ctypes.c_int, [P, P, I32, F32, ctypes.POINTER(ctypes.c_uint64)]),
    ("leafi_server_poll", ctypes.c_int, [P, ctypes.c_uint64, P, P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(I32)]),
    ("leafi_server_replay", ctypes.c_int, [P, P, I64, P, P, P, P, P, P, ctypes.POINTER(ServerReport)]),
    ("leafi_znorm", ctypes.c_int, [P, I64, I32, P, P]),
    ("leafi_lower_bounds", ctypes.c_int, [P, P, I64, P, P]),
    ("leafi_mlp_infer", ctypes.c_int, [P, I32, I32, I32, P, I64, P, P]),
    ("leafi_mlp_sgd_step", ctypes.c_int, [P, I32, I32, I32, P, P, I32, F32, P, P]),
    ("leafi_cnn_infer", ctypes.c_int, [P, I32, I32, I32, P, I64, P, P]),
    ("leafi_cnn_sgd_step", ctypes.c_int, [P, I32, I32, I32, P, P, I32, F32, P, P]),
    ("leafi_leaf_knn", ctypes.c_int, [P, P, I64, I32, P, P, P]),
    ("leafi_select_knapsack", ctypes.c_int, [P, P, I64, ctypes.c_float, ctypes.c_double, ctypes.c_double, I32, I64,
                                             P, P, P, P, P, P]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libleafi.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2502_01836_amd.build` "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != LEAFI_OK:
        msg = load().leafi_last_error().decode(errors="replace")
        raise LeafiError(rc, msg)
