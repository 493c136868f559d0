"""ctypes declarations of the C ABI in include/itsolve.h.

Loading fails loudly: there is no fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libitsolve.so")

ITS_OK, ITS_NOT_CONVERGED, ITS_BREAKDOWN = 0, 1, 2
ITS_E_INVALID, ITS_E_HIP, ITS_E_WORKSPACE, ITS_E_UNSUPPORTED = -1, -2, -3, -4
ITS_JACOBI, ITS_SGS, ITS_CG, ITS_BICGSTAB, ITS_CG_NB = 0, 1, 2, 3, 4
ITS_F64, ITS_F32, ITS_F16 = 0, 1, 2
ITS_RESTART_COSINE, ITS_RESTART_PAPER = 0, 1
MAX_KERNEL_CLASSES = 8
NOALLOC_SCRATCH_BYTES = 64 << 20  # ITS_NOALLOC_SCRATCH_BYTES

# every symbol include/itsolve.h declares
EXPORTS = (
    "its_default_options", "its_csr_create", "its_csr_create64", "its_csr_validate", "its_csr_set_lowp",
    "its_csr_set_colors", "its_stencil_create", "its_matrix_destroy", "its_matrix_rows",
    "its_spmv", "its_dot_workspace_size", "its_dot", "its_workspace_size", "its_solve",
    "its_cast_values", "its_stream_copy", "its_status_string", "its_last_error",
    "its_csr_pack", "its_csr_packed_slots", "its_csr_packed_column_slots", "its_varcoef_create", "its_varcoef_grad",
    "its_batch_create", "its_batch_destroy", "its_batch_cells", "its_batch_workspace_size",
    "its_batch_solve", "its_batch_set_schedule", "its_csr_transpose", "its_csr_value_grad",
    "its_stencil_plan", "its_solve_noalloc",
)


class Options(C.Structure):
    _fields_ = [("method", C.c_int32), ("restart_mode", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int64), ("restart_tol", C.c_double),
                ("check_every", C.c_int32), ("inner_dtype", C.c_int32),
                ("inner_rtol", C.c_double), ("max_outer", C.c_int64),
                ("profile", C.c_int32), ("transpose", C.c_int32),
                ("graph", C.c_int32), ("persistent", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iters", C.c_int64),
                ("inner_iters", C.c_int64), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double),
                ("kernel_ms", C.c_double * MAX_KERNEL_CLASSES),
                ("kernel_launches", C.c_int64 * MAX_KERNEL_CLASSES)]


class BatchResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("tiles_per_item", C.c_int32),
                ("graph_iters", C.c_int32), ("planes_per_brick", C.c_int32), ("max_iters", C.c_int64),
                ("replays", C.c_int64), ("tune_ms", C.c_double), ("solve_ms", C.c_double)]


class ItsError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {status_string(status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    L = C.CDLL(path)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    st = C.c_int
    sig = {
        "its_default_options": (None, [P]),
        "its_csr_create": (st, [I64, I64, P, P, P, P]),
        "its_csr_create64": (st, [I64, I64, P, P, P, P, P]),
        "its_csr_validate": (st, [P, I32, P]),
        "its_csr_set_lowp": (st, [P, P, I32]),
        "its_csr_pack": (st, [P, C.c_double, P]),
        "its_varcoef_create": (st, [I32, I32, I32, P, P]),
        "its_varcoef_grad": (st, [P, P, P, P, P]),
        "its_batch_create": (st, [I32, P, P, I32, P, P]),
        "its_batch_destroy": (st, [P]),
        "its_batch_cells": (I64, [P]),
        "its_batch_workspace_size": (SZ, [P]),
        "its_batch_solve": (st, [P, P, P, P, P, SZ, P, P, P, P]),
        "its_batch_set_schedule": (st, [P, I32, I32]),
        "its_csr_transpose": (st, [P, P]),
        "its_csr_value_grad": (st, [P, P, P, P, P]),
        "its_csr_packed_slots": (C.c_int64, [P]),
        "its_csr_packed_column_slots": (C.c_int64, [P]),
        "its_csr_set_colors": (st, [P, P, I32, P]),
        "its_stencil_create": (st, [I32, I32, I32, I32, P, P]),
        "its_matrix_destroy": (st, [P]),
        "its_matrix_rows": (I64, [P]),
        "its_stencil_plan": (st, [P, P]),
        "its_spmv": (st, [P, P, P, P]),
        "its_dot_workspace_size": (SZ, [I64]),
        "its_dot": (st, [I64, P, P, P, P, SZ, P]),
        "its_workspace_size": (st, [P, P, P]),
        "its_solve": (st, [P, P, P, P, P, SZ, P, P]),
        "its_solve_noalloc": (st, [P, P, P, P, P, P]),
        "its_cast_values": (st, [P, P, I32, I64, P]),
        "its_stream_copy": (st, [P, P, I64, P]),
        "its_status_string": (C.c_char_p, [I32]),
        "its_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
        _lib = load(LIB_PATH)
    return _lib


def status_string(s: int) -> str:
    return lib().its_status_string(int(s)).decode()


def check(status: int, where: str) -> int:
    """Raise on negative (error) codes; return solver outcomes unchanged."""
    if status < 0:
        raise ItsError(status, where, lib().its_last_error().decode())
    return status
