"""ctypes view of libgcp.so (the C ABI declared in include/gcp.h).

Loading fails loudly: there is no fallback path.  Build the library with
``python -m paper_1906_01687_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcp.so")

GCP_MAX_D = 8
GCP_MAX_RANK = 64

# enums (include/gcp.h)
F32, F64, BF16 = 0, 1, 2
GAUSSIAN, BERNOULLI_ODDS, POISSON, GAMMA, BETA_HALF = 0, 1, 2, 3, 4
UNIFORM, STRATIFIED, SEMI_STRATIFIED, FULL = 0, 1, 2, 3
STRATUM_UNIFORM, STRATUM_NZ, STRATUM_ZERO, STRATUM_NZ_CORR, STRATUM_SEMI_ZERO = 0, 1, 2, 3, 4
DENSE, COO = 0, 1
EPS_INSIDE_SQRT, EPS_OUTSIDE_SQRT = 0, 1

STATUS_NAMES = {0: "GCP_OK", 1: "GCP_ERR_INVALID_ARG", 2: "GCP_ERR_UNSUPPORTED",
                3: "GCP_ERR_HIP", 4: "GCP_ERR_WORKSPACE"}


class GcpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class GcpTensor(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("format", ctypes.c_int32), ("vdtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dims", ctypes.c_int64 * GCP_MAX_D),
                ("values", ctypes.c_void_p), ("coo_idx", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("nz_table", ctypes.c_void_p), ("nz_slots", ctypes.c_int64), ("nz_bitmap", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("w_zero", ctypes.c_double)]


class GcpFactors(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32), ("rank", ctypes.c_int64),
                ("A", ctypes.c_void_p * GCP_MAX_D)]


class GcpSampling(ctypes.Structure):
    _fields_ = [("sampler", ctypes.c_int32), ("reserved", ctypes.c_int32), ("s", ctypes.c_int64),
                ("p", ctypes.c_int64), ("q", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("problem_id", ctypes.c_uint64), ("iteration", ctypes.c_uint64), ("rho", ctypes.c_double),
                ("iteration_counter", ctypes.c_void_p)]


class GcpProblem(ctypes.Structure):
    _fields_ = [("X", GcpTensor), ("M", GcpFactors), ("cfg", GcpSampling), ("loss", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eps", ctypes.c_double), ("lower", ctypes.c_double),
                ("A", ctypes.c_void_p), ("A_master", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("G", ctypes.c_void_p)]


class GcpBatchTuning(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("unit_items", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("cols_per_lane", ctypes.c_int32)]


BATCH_CONTIGUOUS, BATCH_LPT = 0, 1


class GcpFitOptions(ctypes.Structure):
    _fields_ = [("grad", GcpSampling), ("est", GcpSampling), ("alpha", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("adam_eps", ctypes.c_double),
                ("lower", ctypes.c_double), ("nu", ctypes.c_double), ("eps_mode", ctypes.c_int32),
                ("tau", ctypes.c_int32), ("kappa", ctypes.c_int32), ("max_epochs", ctypes.c_int32)]


EXPORTS = [
    "gcp_last_error", "gcp_abi_version", "gcp_set_cols_per_lane", "gcp_nz_table_slots", "gcp_nz_table_bytes",
    "gcp_nz_index_build", "gcp_nz_bitmap_bytes", "gcp_nz_bitmap_build", "gcp_sample_workspace_bytes", "gcp_sample", "gcp_loss_grad",
    "gcp_mttkrp_workspace_bytes", "gcp_mttkrp", "gcp_mttkrp_scaled", "gcp_bf16_round", "gcp_rejection_status_offset", "gcp_sampled_grad_workspace_bytes",
    "gcp_sampled_grad", "gcp_sampled_grad_noalloc", "gcp_sampled_adam_step", "gcp_adam_step", "gcp_timing_start",
    "gcp_timing_stop", "gcp_batched_create", "gcp_batched_workspace_bytes", "gcp_batched_prepare", "gcp_batched_plan", "gcp_adam_fit_workspace_bytes", "gcp_adam_fit",
    "gcp_batched_grad", "gcp_batched_adam_step", "gcp_batched_destroy", "gcp_batched_graph_capture",
    "gcp_batched_graph_launch", "gcp_batched_graph_destroy",
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1906_01687_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, u64, sz, dbl, st = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t,
                                ctypes.c_double, ctypes.c_int)
    T, M, S = ctypes.POINTER(GcpTensor), ctypes.POINTER(GcpFactors), ctypes.POINTER(GcpSampling)
    sig = {
        "gcp_last_error": (ctypes.c_char_p, []),
        "gcp_abi_version": (ctypes.c_int, []),
        "gcp_set_cols_per_lane": (st, [ctypes.c_int32]),
        "gcp_nz_table_slots": (i64, [i64]),
        "gcp_nz_table_bytes": (sz, [i64]),
        "gcp_nz_index_build": (st, [T, P, i64, P]),
        "gcp_nz_bitmap_bytes": (sz, [T]),
        "gcp_nz_bitmap_build": (st, [T, P, sz, P]),
        "gcp_sample_workspace_bytes": (sz, [T, S]),
        "gcp_sample": (st, [T, S, P, P, P, P, sz, P]),
        "gcp_loss_grad": (st, [ctypes.c_int, T, S, M, P, P, P, i64, dbl, P, P, P]),
        "gcp_mttkrp_workspace_bytes": (sz, [T, M, i64]),
        "gcp_mttkrp": (st, [T, M, P, P, i64, P, ctypes.c_int, P, sz, P]),
        "gcp_mttkrp_scaled": (st, [T, M, P, P, i64, P, ctypes.c_int, P, P, sz, P]),
        "gcp_bf16_round": (st, [i64, P, P, P]),
        "gcp_rejection_status_offset": (i64, [T, M, S]),
        "gcp_sampled_grad_workspace_bytes": (sz, [T, M, S]),
        "gcp_sampled_grad": (st, [ctypes.c_int, T, M, S, dbl, P, P, P, sz, P]),
        "gcp_sampled_grad_noalloc": (st, [ctypes.c_int, T, M, S, dbl, P, P, P]),
        "gcp_sampled_adam_step": (st, [ctypes.c_int, T, M, S, dbl, P, P, P, P, P, dbl, dbl, dbl, dbl, dbl,
                                       ctypes.c_int, P, P, P, sz, P]),
        "gcp_adam_step": (st, [i64, ctypes.c_int, P, P, P, P, P, P, dbl, dbl, dbl, dbl, dbl,
                               ctypes.c_int, P]),
        "gcp_batched_create": (st, [ctypes.POINTER(GcpProblem), ctypes.c_int32, ctypes.POINTER(GcpBatchTuning),
                                    ctypes.POINTER(ctypes.c_void_p)]),
        "gcp_batched_workspace_bytes": (sz, [P]),
        "gcp_batched_prepare": (st, [P, P, sz, P]),
        "gcp_batched_grad": (st, [P, P, P]),
        "gcp_batched_adam_step": (st, [P, P, P, dbl, dbl, dbl, dbl, ctypes.c_int, P]),
        "gcp_batched_plan": (st, [P, P, P, P, P, P]),
        "gcp_adam_fit_workspace_bytes": (sz, [P, P, ctypes.POINTER(GcpFitOptions)]),
        "gcp_adam_fit": (st, [ctypes.c_int, P, P, ctypes.POINTER(GcpFitOptions), dbl, P, P, P, P, P, P, P, P,
                              P, P, sz, P]),
        "gcp_batched_destroy": (None, [P]),
        "gcp_batched_graph_capture": (st, [P, ctypes.c_int32, P, P, dbl, dbl, dbl, dbl, ctypes.c_int]),
        "gcp_batched_graph_launch": (st, [P, P]),
        "gcp_batched_graph_destroy": (None, [P]),
        "gcp_timing_start": (st, [i64]),
        "gcp_timing_stop": (st, [ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int) -> None:
    if status != 0:
        raise GcpError(status, lib().gcp_last_error().decode())
