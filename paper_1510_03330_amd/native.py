"""ctypes binding of libparquet (the C ABI declared in include/parquet.h).

Argument marshalling only: every step of the parquet iteration runs in the HIP
library. PyTorch provides device memory (tensors) and streams. There is no CPU
fallback: if the library is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libparquet.so")

# ---------------------------------------------------------------- constants
PQ_OK, PQ_ERR_ARG, PQ_ERR_HIP, PQ_ERR_NOMEM, PQ_ERR_SINGULAR = 0, 1, 2, 3, 4
PQ_ERR_NOT_CONVERGED, PQ_ERR_NONFINITE = 5, 6
PQ_STORE_C128, PQ_STORE_C64 = 0, 1
PQ_PREC_FP64, PQ_PREC_FP32, PQ_PREC_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": PQ_PREC_FP64, "fp32": PQ_PREC_FP32, "bf16x3": PQ_PREC_BF16X3}
FIELDS = {"sigma": 0, "g": 1, "phi": 2, "gamma": 3, "k1": 4, "k2": 5, "mu": 6, "xph": 7, "xpp": 8,
          "lambda": 9, "f": 10}
# pq_bse_block_stats.flags bits
BSE_FLAGGED, BSE_NONFINITE, BSE_RESOLVED, BSE_UNRESOLVED, BSE_ESTIMATE = 1, 2, 4, 8, 16

STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_HIP", 3: "ERR_NOMEM", 4: "ERR_SINGULAR",
                5: "ERR_NOT_CONVERGED", 6: "ERR_NONFINITE"}

# Every entry point the header declares (checked by the CPU test suite).
EXPORTS = [
    "pq_dims_from_params", "parquet_last_error", "dyson_update", "bubble_build", "kernel_extract",
    "channel_remap", "sigma_sde_workspace", "sigma_sde", "bse_workspace", "bse_solve", "sigma_mix",
    "parquet_query_workspace", "parquet_init", "parquet_iterate", "parquet_get", "parquet_set",
    "parquet_field_bytes", "parquet_copy_state", "parquet_iterate_batch", "parquet_destroy",
    "phi_from_kernels", "mlp_param_count", "mlp_forward", "mlp_backward", "mlp_adam", "mlp_to_bf16",
    "mlp_basis_workspace", "mlp_basis", "mlp_expand", "parquet_warm_start",
    "parquet_batch_query_workspace", "parquet_batch_init", "parquet_batch_iterate", "parquet_batch_status",
    "parquet_batch_get", "parquet_batch_tile", "parquet_batch_destroy", "hbm_stream",
    "sigma_sde_no_alloc",
]


class PqParams(ctypes.Structure):
    _fields_ = [
        ("Lx", c_int32), ("Ly", c_int32), ("Nv", c_int32), ("f_ext", c_int32),
        ("kernel_level", c_int32), ("edge_rule", c_int32), ("mu_mode", c_int32),
        ("storage", c_int32), ("precision", c_int32), ("resolve_slots", c_int32),
        ("regulation", c_int32), ("bse_tile", c_int32), ("U", c_double), ("beta", c_double), ("t", c_double), ("tp", c_double),
        ("filling", c_double), ("D", c_double), ("mu_fixed", c_double), ("alpha", c_double),
        ("bse_tol", c_double),
    ]


class PqDims(ctypes.Structure):
    _fields_ = [
        ("Lx", c_int32), ("Ly", c_int32), ("Nk", c_int32), ("Nv", c_int32), ("NW", c_int32),
        ("f_ext", c_int32), ("Nve", c_int32), ("NWe", c_int32), ("NG", c_int32), ("n", c_int32),
        ("Nq", c_int32), ("ntau", c_int32), ("vertex_elems", c_int64),
    ]


class PqIterStats(ctypes.Structure):
    _fields_ = [
        ("iteration", c_int32), ("flagged_blocks", c_int32), ("dsigma", c_double), ("mu", c_double),
        ("ms_total", c_double), ("ms_stage", c_double * 8), ("ms_bse_kernel", c_double * 6),
        ("n_bse_launch", c_int32 * 6), ("resolved_blocks", c_int32), ("unresolved_blocks", c_int32),
        ("update_flops", c_double), ("max_err_est", c_double),
    ]


class PqBseBlockStats(ctypes.Structure):
    _fields_ = [("min_pivot", ctypes.c_float), ("growth", ctypes.c_float), ("flags", c_int32),
                ("err_est", ctypes.c_float)]


class ParquetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def library_path() -> str:
    return LIB_PATH


def load() -> ctypes.CDLL:
    """Load libparquet.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1510_03330_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER(PqParams)
    sig = {
        "pq_dims_from_params": [P, POINTER(PqDims)],
        "dyson_update": [P, c_void_p, c_void_p, c_void_p, c_void_p],
        "bubble_build": [P, c_void_p, c_void_p, c_void_p, c_void_p],
        "kernel_extract": [P, c_void_p, c_void_p, c_void_p, c_void_p],
        "channel_remap": [P, POINTER(c_double), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                          c_void_p],
        "sigma_sde_workspace": [P, POINTER(c_size_t)],
        "sigma_sde": [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                      c_size_t, c_void_p],
        "sigma_sde_no_alloc": [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p],
        "bse_workspace": [P, POINTER(c_size_t)],
        "bse_solve": [P, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                      c_void_p, c_size_t, c_void_p],
        "sigma_mix": [P, c_void_p, c_void_p, c_double, c_void_p, c_void_p],
        "parquet_query_workspace": [P, POINTER(c_size_t)],
        "parquet_init": [P, c_void_p, c_size_t, c_void_p, POINTER(c_void_p)],
        "parquet_iterate": [c_void_p, c_int32, c_double, POINTER(PqIterStats), POINTER(c_int32),
                            POINTER(c_int32)],
        "parquet_get": [c_void_p, c_int32, c_void_p, c_size_t],
        "parquet_set": [c_void_p, c_int32, c_void_p, c_size_t],
        "parquet_field_bytes": [c_void_p, c_int32, POINTER(c_size_t)],
        "parquet_copy_state": [c_void_p, c_void_p],
        "parquet_iterate_batch": [POINTER(c_void_p), c_int32, c_int32, c_double, POINTER(c_int32),
                                  POINTER(c_int32)],
        "phi_from_kernels": [P, c_void_p, c_void_p, c_void_p, c_void_p],
        "mlp_param_count": [POINTER(c_int32), c_int32, POINTER(c_size_t)],
        "mlp_forward": [POINTER(c_int32), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p],
        "mlp_backward": [POINTER(c_int32), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                         c_void_p, c_int32, c_void_p],
        "mlp_adam": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, ctypes.c_float, ctypes.c_float,
                     ctypes.c_float, ctypes.c_float, c_int32, c_void_p],
        "mlp_to_bf16": [c_void_p, c_void_p, c_size_t, c_void_p],
        "mlp_basis_workspace": [c_int32, POINTER(c_size_t)],
        "parquet_warm_start": [c_void_p, c_void_p, c_void_p, c_void_p],
        "mlp_basis": [c_void_p, c_int32, c_size_t, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p],
        "mlp_expand": [c_void_p, c_int32, c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
        "parquet_destroy": [c_void_p],
        "parquet_batch_query_workspace": [P, c_int32, POINTER(c_size_t)],
        "parquet_batch_init": [P, c_int32, c_void_p, c_size_t, c_void_p, c_int32, POINTER(c_void_p)],
        "parquet_batch_iterate": [c_void_p, c_int32, c_double, c_double, POINTER(c_int32)],
        "parquet_batch_status": [c_void_p, c_void_p, c_void_p, c_void_p],
        "parquet_batch_get": [c_void_p, c_int32, c_int32, c_void_p, c_size_t],
        "parquet_batch_tile": [c_void_p, POINTER(c_int32), c_void_p],
        "parquet_batch_destroy": [c_void_p],
        "hbm_stream": [c_int32, c_void_p, c_void_p, c_size_t, c_void_p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.parquet_last_error.argtypes = []
    lib.parquet_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


BATCH_STATES = {0: "running", 1: "converged", 2: "diverged", 3: "nonfinite", 4: "singular"}


def check(status: int):
    if status != PQ_OK:
        msg = load().parquet_last_error().decode(errors="replace")
        raise ParquetError(status, msg)


def make_params(p, precision: str = "fp64", resolve_slots: int = 0, bse_tol: float = 0.0,
                bse_tile: int = 0) -> PqParams:
    """pq_params from any object with the ModelParams attributes (resolve_slots
    and bse_tol: 0 selects the library defaults; bse_tile: the FP32 update tile)."""
    if precision not in PRECISIONS:
        raise ValueError(f"precision {precision!r} not available ({', '.join(PRECISIONS)})")
    out = PqParams()
    out.Lx, out.Ly, out.Nv = int(p.Lx), int(p.Ly), int(p.Nv)
    out.f_ext = int(p.f_ext)
    out.kernel_level = int(p.kernel_level)
    out.edge_rule = int(p.edge_rule)
    out.mu_mode = int(p.mu_mode)
    out.storage = PQ_STORE_C128 if precision == "fp64" else PQ_STORE_C64
    out.precision = PRECISIONS[precision]
    out.U, out.beta, out.t, out.tp = float(p.U), float(p.beta), float(p.t), float(p.tp)
    out.filling, out.D, out.mu_fixed, out.alpha = float(p.filling), float(p.D), float(p.mu_fixed), float(p.alpha)
    out.resolve_slots = int(resolve_slots)
    out.regulation = int(getattr(p, "regulation", 1))
    out.bse_tol = float(bse_tol)
    out.bse_tile = int(bse_tile)
    return out


def dims(pp: PqParams) -> PqDims:
    d = PqDims()
    check(load().pq_dims_from_params(ctypes.byref(pp), ctypes.byref(d)))
    return d
