"""ctypes declarations of the libgep C ABI (include/gep.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libgep.so"

JOB_VALUES = 0
JOB_VECTORS = 1
PREC_FP64 = 0
PREC_MIXED = 1

GEP_OK = 0
GEP_ERR_ARG = -1
GEP_ERR_WORKSPACE = -2
GEP_ERR_HIP = -3

# device info codes besides LAPACK's (include/gep.h)
INFO_WAIT_TIMEOUT = -1
INFO_REFINE_FAILED = -2


class GEPError(RuntimeError):
    def __init__(self, status: int, where: str, bad_arg: int = 0):
        msg = f"{where}: {status_string(status)} (status {status})"
        if status == GEP_ERR_ARG:
            msg += f", argument {bad_arg}"
        super().__init__(msg)
        self.status = status
        self.bad_arg = bad_arg


def lib_path() -> str:
    return os.path.join(HERE, _LIB_NAME)


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
INT = ctypes.c_int
SZ = ctypes.c_size_t
DBL = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "gep_status_string": (ctypes.c_char_p, [INT]),
    "gep_last_bad_arg": (INT, []),
    "gep_version": (ctypes.c_char_p, []),
    "gep_workspace_size": (SZ, [I64, INT, INT]),
    "gep_solve": (INT, [I64, P, I64, P, I64, P, P, I64, INT, INT, P, SZ, P, P]),
    "gep_solve_noalloc": (INT, [I64, P, I64, P, I64, P, P, I64, INT, INT, P, P]),
    "gep_noalloc_max_bytes": (SZ, []),
    "gep_workspace_size_lowest": (SZ, [I64, I64]),
    "gep_solve_lowest": (INT, [I64, P, I64, P, I64, I64, P, P, I64, P, SZ, P, P]),
    "gep_workspace_size_cholfree": (SZ, [I64]),
    "gep_solve_cholfree": (INT, [I64, P, I64, P, I64, P, P, I64, P, SZ, P, P]),
    "gep_workspace_size_explicit_inverse": (SZ, [I64]),
    "gep_solve_explicit_inverse": (INT, [I64, P, I64, P, I64, P, P, I64, P, SZ, P, P]),
    "gep_workspace_size_jacobi": (SZ, [I64]),
    "gep_solve_jacobi": (INT, [I64, P, I64, P, I64, P, P, I64, P, SZ, P, P]),
    "gep_last_jacobi_sweeps": (INT, []),
    "gep_workspace_size_batched": (SZ, [INT, P, INT, INT]),
    "gep_solve_batched": (INT, [INT, P, P, P, P, P, P, P, P, INT, INT, P, SZ, P, P]),
    "gep_batched_threads": (INT, [INT]),
    "gep_reduce_workspace_size": (SZ, [I64]),
    "gep_reduce": (INT, [I64, P, I64, P, I64, P, I64, P, I64, P, SZ, P, P]),
    "gep_band_reduce_workspace_size": (SZ, [I64, INT]),
    "gep_band_reduce": (INT, [I64, P, I64, INT, P, I64, P, SZ, P]),
    "gep_tridiagonalize_workspace_size": (SZ, [I64, INT]),
    "gep_tridiagonalize": (INT, [I64, P, I64, INT, P, P, P, SZ, P]),
    "gep_tridiag_eig_workspace_size": (SZ, [I64, INT]),
    "gep_tridiag_eig": (INT, [I64, P, P, P, P, I64, INT, P, SZ, P, P]),
    "gep_backward_workspace_size": (SZ, [I64]),
    "gep_backward": (INT, [I64, P, P, I64, P, P, I64, DBL, DBL, P, I64, P, I64, P, SZ, P]),
    "gep_dgemm": (INT, [INT, INT, INT, I64, I64, I64, DBL, P, I64, P, I64, DBL, P, I64, INT, P]),
    "gep_profile_enable": (INT, [INT]),
    "gep_profile_read": (INT, [P, INT]),
    "gep_profile_dc_flops": (DBL, []),
    "gep_probe_enable": (INT, [INT]),
    "gep_probe_read": (INT, [INT, P, P, P]),
    "gep_probe_name": (ctypes.c_char_p, [INT]),
    "gep_tune_load": (INT, [ctypes.c_char_p]),
    "gep_tune_set": (INT, [ctypes.c_char_p, I64, I64, I64]),
    "gep_tune_reset_overrides": (INT, []),
    "gep_tune_clear": (INT, []),
    "gep_tune_get": (I64, [ctypes.c_char_p, I64]),
    "gep_debug_force_wait_timeout": (INT, [INT]),
    "gep_debug_force_eig_failure": (INT, [INT]),
}


def lib():
    """Load libgep.so (built in place by paper_1504_06443_amd/build.py)."""
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               f"`python -m paper_1504_06443_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().gep_status_string(status).decode()
    except Exception:
        return "unknown"


def check(status: int, where: str) -> None:
    if status != GEP_OK:
        raise GEPError(status, where, lib().gep_last_bad_arg())


def workspace_size(M: int, job: int = JOB_VECTORS, prec: int = PREC_FP64) -> int:
    return int(lib().gep_workspace_size(M, job, prec))
