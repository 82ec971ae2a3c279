"""ctypes declarations of the C ABI in include/mlspgemm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlspgemm.so")

c_int32, c_int64, c_size_t, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
P = c_void_p


class CsrT(ctypes.Structure):
    _fields_ = [("nrows", c_int32), ("ncols", c_int32), ("nnz", c_int64),
                ("row_ptr", c_void_p), ("col_idx", c_void_p), ("values", c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("algo", c_int32), ("branch", c_int32), ("n_ac_parts", c_int32), ("n_b_parts", c_int32),
                ("nbuf_inner", c_int32), ("n_steps", c_int32), ("fast_bytes", c_int64),
                ("h2d_bytes", c_int64), ("d2h_bytes", c_int64), ("cost_chunk1", c_int64),
                ("cost_chunk2", c_int64), ("chunk_bytes", c_int64), ("ws_bytes", c_int64),
                ("issued_h2d", c_int64), ("issued_d2h", c_int64), ("zero_copy_bytes", c_int64)]


class PlanStep(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("matrix", c_int32), ("part", c_int32), ("row_begin", c_int32),
                ("row_end", c_int32), ("slot", c_int32), ("bytes", c_int64)]


class TraceEntry(ctypes.Structure):
    _fields_ = [("op", c_int32), ("kind", c_int32), ("stream", c_int32), ("event", c_int32), ("space", c_int32),
                ("write", c_int32), ("lo", c_int64), ("hi", c_int64)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("calls", c_int64), ("total_ms", ctypes.c_double)]


CSRP = ctypes.POINTER(CsrT)
I64P = ctypes.POINTER(c_int64)
SZP = ctypes.POINTER(c_size_t)

# name -> (restype, argtypes)
SIGNATURES = {
    "spgemm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "spgemm_last_hip_error": (ctypes.c_int, []),
    "spgemm_version": (ctypes.c_int, []),
    "spgemm_set_option": (ctypes.c_int, [ctypes.c_int, c_int64]),
    "spgemm_get_option": (c_int64, [ctypes.c_int]),
    "spgemm_validate_host": (ctypes.c_int, [CSRP]),
    "spgemm_profile_read": (c_int32, [ctypes.POINTER(ProfileEntry), c_int32]),
    "spgemm_profile_reset": (None, []),
    "spgemm_workspace_size": (ctypes.c_int, [CSRP, CSRP, SZP]),
    "spgemm_row_work": (ctypes.c_int, [CSRP, CSRP, P, I64P, P, c_size_t, P]),
    "spgemm_compress": (ctypes.c_int, [CSRP, P, P, P, c_size_t, P]),
    "spgemm_symbolic": (ctypes.c_int, [CSRP, CSRP, P, P, I64P, P, c_size_t, P]),
    "spgemm_numeric": (ctypes.c_int, [CSRP, CSRP, CSRP, P, c_size_t, P]),
    "spgemm_symbolic_chunked": (ctypes.c_int, [CSRP, CSRP, P, P, I64P, P, c_size_t, P]),
    "spgemm_check_errors": (ctypes.c_int, [P, c_size_t, P]),
    "spgemm_numeric_noalloc": (ctypes.c_int, [CSRP, CSRP, CSRP, P]),
    "spgemm_numeric_placed": (ctypes.c_int, [CSRP, CSRP, CSRP, ctypes.POINTER(ctypes.c_uint32), P, c_size_t, P]),
    "spgemm_chunked_plan": (ctypes.c_int, [CSRP, CSRP, P, c_size_t, c_int32, c_int32, ctypes.POINTER(P)]),
    "spgemm_chunked_plan_knl": (ctypes.c_int, [CSRP, CSRP, P, c_size_t, c_int32, c_int32, ctypes.POINTER(P)]),
    "spgemm_plan_info_get": (ctypes.c_int, [P, ctypes.POINTER(PlanInfo)]),
    "spgemm_plan_parts": (ctypes.c_int, [P, c_int32, P, c_int32]),
    "spgemm_plan_steps": (ctypes.c_int, [P, ctypes.POINTER(PlanStep), c_int32]),
    "spgemm_plan_destroy": (None, [P]),
    "spgemm_numeric_chunked": (ctypes.c_int, [CSRP, CSRP, CSRP, P, P, c_size_t, P, P, P]),
    "spgemm_numeric_chunked_trace": (ctypes.c_int, [CSRP, CSRP, CSRP, P, ctypes.POINTER(TraceEntry), c_int64, I64P]),
    "spgemm_tc_lower": (ctypes.c_int, [CSRP, P, P, P, I64P]),
    "spgemm_tc_workspace_size": (ctypes.c_int, [CSRP, SZP]),
    "spgemm_tc": (ctypes.c_int, [CSRP, P, I64P, P, c_size_t, P]),
    "spgemm_batch_workspace_size": (ctypes.c_int, [c_int32, CSRP, CSRP, SZP]),
    "spgemm_batch_symbolic": (ctypes.c_int, [c_int32, CSRP, CSRP, CSRP, c_int32, I64P, P, c_size_t, P]),
    "spgemm_batch_numeric": (ctypes.c_int, [c_int32, CSRP, CSRP, CSRP, P, c_size_t, P]),
    "spgemm_batch_plan_create": (ctypes.c_int, [c_int32, CSRP, CSRP, CSRP, c_int32, c_int32, ctypes.c_char_p, P,
                                                c_size_t, P, ctypes.POINTER(P)]),
    "spgemm_batch_plan_schedule": (ctypes.c_int, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                                  ctypes.POINTER(c_int32)]),
    "spgemm_batch_plan_run": (ctypes.c_int, [P, P]),
    "spgemm_batch_plan_group_size": (c_int32, [P]),
    "spgemm_batch_plan_destroy": (None, [P]),
    "spgemm_backward_workspace_size": (ctypes.c_int, [CSRP, CSRP, CSRP, c_int32, SZP]),
    "spgemm_backward": (ctypes.c_int, [CSRP, CSRP, CSRP, P, P, c_int32, P, c_size_t, P]),
    "spgemm_transpose_workspace_size": (ctypes.c_int, [CSRP, SZP]),
    "spgemm_transpose": (ctypes.c_int, [CSRP, CSRP, P, c_size_t, P]),
    "spgemm_mask_gather": (ctypes.c_int, [CSRP, CSRP, P, P]),
}

OPT_VALIDATE, OPT_FORCE_SPILL, OPT_GROUP_SIZE, OPT_FORCE_CLASS, OPT_PROFILE, OPT_WIDE_TABLE = 0, 1, 2, 3, 4, 5
STATUS_NAMES = ["OK", "INVALID_ARG", "BAD_CSR", "DIM_MISMATCH", "INDEX_OVERFLOW", "WORKSPACE_TOO_SMALL",
                "BUDGET", "HIP", "UNSUPPORTED", "STRUCTURE"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libmlspgemm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1804_00695_amd.build` "
                          "(the HIP library has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SpgemmError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        msg = f"{where}: SPGEMM_ERR_{name}"
        if status == 7 and _lib is not None:
            msg += f" (hip error {_lib.spgemm_last_hip_error()})"
        super().__init__(msg)


def check(status: int, where: str = ""):
    if status != 0:
        raise SpgemmError(status, where)
