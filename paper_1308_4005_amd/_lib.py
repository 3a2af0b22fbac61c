"""ctypes binding of ``libmlsdisp.so`` (declarations of include/mlsdisp.h).

Argument marshalling only: every step of the evaluation runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlsdisp.so")

MLS_OK = 0
MLS_ERR_INVALID_ARG = -1
MLS_ERR_UNSUPPORTED = -2
MLS_ERR_HIP = -3
MLS_ERR_OOM = -4
MLS_ERR_NONFINITE = -5
MLS_FP64 = 0
MLS_MIXED = 1
MLS_GEOMETRIC = 0
MLS_LORENTZ_BERTHELOT = 1

MLS_STAGE_PERM = 0
MLS_STAGE_CELL_START = 1
MLS_STAGE_E0 = 2
MLS_STAGE_FLOC = 3
MLS_STAGE_Q = 4
MLS_STAGE_E_LEVEL = 5
MLS_STAGE_E_TOTAL = 6

EXPORTS = [
    "mls_plan_create", "mls_plan_get_info", "mls_evaluate", "mls_evaluate_lb", "mls_plan_copy_stage",
    "mls_plan_status", "mls_plan_destroy", "mls_batch_create", "mls_batch_evaluate",
    "mls_batch_set_graph", "mls_batch_get_tuning", "mls_batch_set_tuning", "mls_batch_box_info",
    "mls_batch_status", "mls_batch_destroy", "mls_status_string", "mls_last_error",
    "mls_plan_set_timing", "mls_plan_read_timing", "mls_evaluate_md", "mls_md_run",
    "mls_md_run_mts", "mls_evaluate_noalloc", "mls_md_run_mts_levels", "mls_batch_evaluate_lb",
]

STAGE_NAMES = ["binning", "pair", "anterpolation", "restriction", "stencil", "coarsest",
               "prolongation", "interpolation"]


class MLSParams(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("cutoff", ctypes.c_double),
        ("h", ctypes.c_double),
        ("order", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("grid", ctypes.c_int * 3),
        ("precision", ctypes.c_int),
        ("continuity", ctypes.c_int),
        ("mixing", ctypes.c_int),
        ("skin", ctypes.c_double),
    ]


class MLSPlanInfo(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("grid", ctypes.c_int * 3),
        ("coarsest", ctypes.c_int * 3),
        ("cells", ctypes.c_int * 3),
        ("h_eff", ctypes.c_double * 3),
        ("taps", ctypes.c_int64),
        ("n_max", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("precision", ctypes.c_int),
        ("order", ctypes.c_int),
        ("cell_width", ctypes.c_double * 3),
        ("continuity", ctypes.c_int),
        ("mixing", ctypes.c_int),
        ("stencil_path", ctypes.c_int),
    ]


STENCIL_PATHS = {0: "none", 1: "tile_f32", 2: "tile_f64", 3: "stream_f64", 4: "taps_f64", 5: "tile_mfma_f32"}


class MLSBatchTuning(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int * 8),
        ("stencil_zc", ctypes.c_int),
        ("tuned_ms", ctypes.c_double),
        ("stage_ms", ctypes.c_double * 8),
    ]


class MLSError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def load():
    """Load the library (importing torch first so the process has a single HIP
    runtime); raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1308_4005_amd.build` (HIP extension required)")
    import torch  # noqa: F401  (shares its HIP runtime with the library)
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    dp = ctypes.c_void_p
    lib.mls_plan_create.argtypes = [ctypes.POINTER(MLSParams), i64, ctypes.POINTER(P)]
    lib.mls_plan_get_info.argtypes = [P, ctypes.POINTER(MLSPlanInfo)]
    lib.mls_evaluate.argtypes = [P, i64, dp, dp, dp, dp, dp, dp, P]
    lib.mls_evaluate_noalloc.argtypes = [ctypes.POINTER(MLSParams), i64, dp, dp, dp, dp, dp, dp, P]
    lib.mls_evaluate_lb.argtypes = [P, i64, dp, dp, dp, dp, dp, P]
    dbl = ctypes.c_double
    lib.mls_evaluate_md.argtypes = [P, i64, dp, dp, dp, dbl, dp, dp, P]
    lib.mls_md_run.argtypes = [P, i64, dp, dp, dp, dp, dbl, dp, dbl, ctypes.c_int, dp, dp, dp, P]
    lib.mls_md_run_mts.argtypes = [P, i64, dp, dp, dp, dp, dbl, dp, dbl, ctypes.c_int, ctypes.c_int, dp, dp, dp, P]
    lib.mls_md_run_mts_levels.argtypes = [P, i64, dp, dp, dp, dp, dbl, dp, dbl, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, dp, dp, dp, P]
    lib.mls_plan_copy_stage.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, i64, P]
    lib.mls_plan_status.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.mls_plan_destroy.argtypes = [P]
    lib.mls_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(MLSParams), ctypes.POINTER(i64),
                                     ctypes.c_int, ctypes.POINTER(P)]
    lib.mls_batch_evaluate.argtypes = [P, dp, dp, dp, dp, dp, P]
    lib.mls_batch_evaluate_lb.argtypes = [P, dp, dp, dp, dp, dp, P]
    lib.mls_batch_set_graph.argtypes = [P, ctypes.c_int]
    lib.mls_batch_get_tuning.argtypes = [P, ctypes.POINTER(MLSBatchTuning)]
    lib.mls_batch_set_tuning.argtypes = [P, ctypes.POINTER(MLSBatchTuning)]
    lib.mls_batch_box_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(MLSPlanInfo)]
    lib.mls_batch_status.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.mls_batch_destroy.argtypes = [P]
    lib.mls_plan_set_timing.argtypes = [P, ctypes.c_int]
    lib.mls_plan_read_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    for fn in EXPORTS:
        if fn not in ("mls_status_string", "mls_last_error"):
            getattr(lib, fn).restype = ctypes.c_int
    lib.mls_status_string.argtypes = [ctypes.c_int]
    lib.mls_status_string.restype = ctypes.c_char_p
    lib.mls_last_error.argtypes = []
    lib.mls_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status, where):
    if status != MLS_OK:
        lib = load()
        detail = lib.mls_last_error().decode() or lib.mls_status_string(status).decode()
        raise MLSError(status, where, detail)
