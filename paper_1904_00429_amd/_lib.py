"""ctypes declarations of the C ABI in include/mlmc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlmc.so")

MLMC_MAX_LEVELS = 32
STATUS = {0: "MLMC_OK", 1: "MLMC_EINVAL", 2: "MLMC_EDEVICE", 3: "MLMC_EBUDGET", 4: "MLMC_EWORKSPACE"}
EXPORTED = [
    "mlmc_matmul_workspace_size", "mlmc_inner_product_workspace_size", "mlmc_matmul_estimate",
    "mlmc_inner_product_estimate", "mlmc_philox4x32_10", "mlmc_sample_indices",
    "mlmc_gather_columns", "mlmc_status_string", "mlmc_last_error",
    "mlmc_matmul_adjoint_workspace_size", "mlmc_matmul_adjoint_reparam",
    "mlmc_matmul_batched_workspace_size", "mlmc_matmul_estimate_batched",
    "mlmc_matmul_batched_graph_create", "mlmc_graph_launch", "mlmc_graph_destroy",
    "mlmc_optimal_index_weights", "mlmc_sample_indices_weighted",
    "mlmc_inner_product_noalloc_limit", "mlmc_inner_product_estimate_noalloc",
    "mlmc_inner_product_graph_create", "mlmc_inner_product_graph_report",
]


class Dist(ctypes.Structure):
    _fields_ = [("law", ctypes.c_int32), ("loc", ctypes.c_double), ("scale", ctypes.c_double),
                ("mean", ctypes.c_void_p), ("stdev", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class Levels(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int32), ("c", ctypes.POINTER(ctypes.c_int64)),
                ("n_samples", ctypes.POINTER(ctypes.c_int64)), ("rmse_target", ctypes.c_double),
                ("pilot_samples", ctypes.c_int64), ("max_total_draws", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("prec", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("problem", ctypes.c_uint32), ("func", ctypes.c_int32),
                ("func_param", ctypes.c_double * 2), ("index_weights", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("A", Dist), ("B", Dist), ("problem", ctypes.c_uint32),
                ("out", ctypes.c_void_p), ("level_means", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("target_blocks", ctypes.c_int64),
                ("gather_budget", ctypes.c_int64), ("single_launch", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("n_used", ctypes.c_int64 * MLMC_MAX_LEVELS),
                ("level_var", ctypes.c_double * MLMC_MAX_LEVELS),
                ("rmse_est", ctypes.c_double), ("total_draws", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double * 4), ("kernel_launches", ctypes.c_int64 * 4),
                ("levels_used", ctypes.c_int32), ("bias_test_passed", ctypes.c_int32)]


class MLMCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmlmc.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1904_00429_amd/build.py` (there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    LP, DP, RP = ctypes.POINTER(Levels), ctypes.POINTER(Dist), ctypes.POINTER(Report)
    L.mlmc_matmul_workspace_size.restype = ctypes.c_size_t
    L.mlmc_matmul_workspace_size.argtypes = [i64, i64, i64, LP]
    L.mlmc_inner_product_workspace_size.restype = ctypes.c_size_t
    L.mlmc_inner_product_workspace_size.argtypes = [i64, LP]
    L.mlmc_matmul_estimate.restype = ctypes.c_int
    L.mlmc_matmul_estimate.argtypes = [i64, i64, i64, DP, DP, LP, vp, vp, vp, ctypes.c_size_t, RP, vp]
    L.mlmc_inner_product_estimate.restype = ctypes.c_int
    L.mlmc_inner_product_estimate.argtypes = [i64, DP, DP, LP, vp, vp, vp, ctypes.c_size_t, RP, vp]
    L.mlmc_inner_product_noalloc_limit.restype = ctypes.c_size_t
    L.mlmc_inner_product_noalloc_limit.argtypes = []
    L.mlmc_inner_product_estimate_noalloc.restype = ctypes.c_int
    L.mlmc_inner_product_estimate_noalloc.argtypes = [i64, DP, DP, LP, vp, vp, RP, vp]
    L.mlmc_philox4x32_10.restype = ctypes.c_int
    L.mlmc_philox4x32_10.argtypes = [i64, vp, u64, vp, vp]
    L.mlmc_sample_indices.restype = ctypes.c_int
    L.mlmc_sample_indices.argtypes = [u64, u32, u32, u32, i64, i64, i64, vp, vp]
    L.mlmc_gather_columns.restype = ctypes.c_int
    L.mlmc_gather_columns.argtypes = [i64, i64, i64, DP, DP, u64, u32, u32, u32, i64, i64, i32, vp, vp, vp]
    L.mlmc_optimal_index_weights.restype = ctypes.c_int
    L.mlmc_optimal_index_weights.argtypes = [i64, i64, i64, DP, DP, vp, vp, vp]
    L.mlmc_sample_indices_weighted.restype = ctypes.c_int
    L.mlmc_sample_indices_weighted.argtypes = [u64, u32, u32, u32, i64, i64, i64, vp, vp, vp, vp]
    L.mlmc_matmul_adjoint_workspace_size.restype = ctypes.c_size_t
    L.mlmc_matmul_adjoint_workspace_size.argtypes = [i64, i64, i64, LP]
    L.mlmc_matmul_adjoint_reparam.restype = ctypes.c_int
    L.mlmc_matmul_adjoint_reparam.argtypes = [i64, i64, i64, DP, DP, LP, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    PP, TP = ctypes.POINTER(Problem), ctypes.POINTER(Tuning)
    L.mlmc_matmul_batched_workspace_size.restype = ctypes.c_size_t
    L.mlmc_matmul_batched_workspace_size.argtypes = [i32, PP, LP, TP]
    L.mlmc_matmul_estimate_batched.restype = ctypes.c_int
    L.mlmc_matmul_estimate_batched.argtypes = [i32, PP, LP, TP, vp, ctypes.c_size_t, vp, vp]
    L.mlmc_matmul_batched_graph_create.restype = ctypes.c_int
    L.mlmc_matmul_batched_graph_create.argtypes = [i32, PP, LP, TP, vp, ctypes.c_size_t, vp,
                                                   ctypes.POINTER(ctypes.c_void_p)]
    L.mlmc_inner_product_graph_create.restype = ctypes.c_int
    L.mlmc_inner_product_graph_create.argtypes = [i64, DP, DP, LP, vp, vp, vp, ctypes.c_size_t, vp,
                                                  ctypes.POINTER(ctypes.c_void_p)]
    L.mlmc_inner_product_graph_report.restype = ctypes.c_int
    L.mlmc_inner_product_graph_report.argtypes = [i64, LP, vp, ctypes.c_size_t, RP, vp]
    L.mlmc_graph_launch.restype = ctypes.c_int
    L.mlmc_graph_launch.argtypes = [vp, vp]
    L.mlmc_graph_destroy.restype = ctypes.c_int
    L.mlmc_graph_destroy.argtypes = [vp]
    L.mlmc_status_string.restype = ctypes.c_char_p
    L.mlmc_status_string.argtypes = [ctypes.c_int]
    L.mlmc_last_error.restype = ctypes.c_char_p
    L.mlmc_last_error.argtypes = []
    _lib = L
    return L


def check(status: int) -> None:
    if status != 0:
        raise MLMCError(status, lib().mlmc_last_error().decode(errors="replace"))
