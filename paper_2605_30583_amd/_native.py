"""ctypes declarations of the C ABI in include/caspar_ba.h."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcaspar_ba.so")

FP64 = 0
FP32_MIXED = 1
ADJ_GAUGE_PROJECT = 1
RECOMPUTE_JACOBIAN = 0x10
LOSS_TRIVIAL, LOSS_HUBER, LOSS_CAUCHY = 0, 1, 2
STATUS = {0: "CASPAR_OK", -1: "CASPAR_EINVAL", -2: "CASPAR_EHIP", -3: "CASPAR_ENOMEM", -4: "CASPAR_ENUMERIC",
          -5: "CASPAR_EIO"}


class SolveOpts(C.Structure):
    _fields_ = [("lambda0", C.c_double), ("pcg_tol", C.c_double), ("max_lm_iters", C.c_int32),
                ("max_pcg_iters", C.c_int32), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("grad_tol", C.c_double), ("min_cost", C.c_double), ("pcg_check_every", C.c_int32),
                ("flags", C.c_int32), ("pred_tol", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("lm_iters", C.c_int32), ("accepted", C.c_int32), ("pcg_iters_total", C.c_int32),
                ("stop_reason", C.c_int32), ("initial_cost", C.c_double), ("final_cost", C.c_double),
                ("final_lambda", C.c_double), ("seconds", C.c_double)]


class IterRecord(C.Structure):
    _fields_ = [("cost", C.c_double), ("trial_cost", C.c_double), ("lam", C.c_double), ("rho", C.c_double),
                ("pred", C.c_double), ("pcg_rel_resid", C.c_double), ("accepted", C.c_int32),
                ("pcg_iters", C.c_int32), ("seconds", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("matvec_launches", C.c_int64), ("matvec_ms", C.c_double), ("matvec_bytes", C.c_double)]


# (name, restype, argtypes) for every exported function
_P = C.c_void_p
_D = C.POINTER(C.c_double)
SIGNATURES = [
    ("caspar_default_solve_opts", None, [C.POINTER(SolveOpts)]),
    ("caspar_ba_workspace_bytes", C.c_size_t, [C.c_int32, C.c_int32, C.c_int64, C.c_int]),
    ("caspar_ba_create", C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.c_int,
                                   _P, C.c_size_t, _P]),
    ("caspar_ba_create_static", C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P,
                                          C.c_int, _P]),
    ("caspar_ba_solve", C.c_int, [_P, C.POINTER(SolveOpts), C.POINTER(SolveStats), C.POINTER(IterRecord)]),
    ("caspar_ba_get_params", C.c_int, [_P, _P, _P]),
    ("caspar_ba_set_params", C.c_int, [_P, _P, _P]),
    ("caspar_ba_set_observations", C.c_int, [_P, _P]),
    ("caspar_ba_set_loss", C.c_int, [_P, C.c_int32, C.c_double]),
    ("caspar_ba_backward", C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_int32, C.c_int32, _P,
                                     C.POINTER(C.c_int32), _D]),
    ("caspar_ba_linearize", C.c_int, [_P, _D, _P, _P, _P, _P, _P]),
    ("caspar_ba_matvec", C.c_int, [_P, C.c_double, _P, _P, _D]),
    ("caspar_ba_block_jacobi_apply", C.c_int, [_P, C.c_double, _P, _P]),
    ("caspar_ba_pcg", C.c_int, [_P, C.c_double, _P, C.c_double, C.c_int32, _P, C.POINTER(C.c_int32), _D]),
    ("caspar_ba_cost_fp64", C.c_int, [_P, _D]),
    ("caspar_project", C.c_int, [C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P]),
    ("caspar_ba_between_workspace_bytes", C.c_size_t, [C.c_int32, C.c_int32]),
    ("caspar_ba_set_between", C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, C.c_size_t]),
    ("caspar_bal_read_header", C.c_int, [C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64)]),
    ("caspar_bal_read", C.c_int, [C.c_char_p, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P]),
    ("caspar_bal_write", C.c_int, [C.c_char_p, C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P]),
    ("caspar_ba_layout_info", C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int32)]),
    ("caspar_ba_set_timing", C.c_int, [_P, C.c_int]),
    ("caspar_ba_get_timing", C.c_int, [_P, C.POINTER(Timing)]),
    ("caspar_ba_destroy", None, [_P]),
    ("caspar_last_error", C.c_char_p, []),
]

_lib = None


def load(path: str | None = None):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_2605_30583_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class CasparError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != 0:
        raise CasparError(status, load().caspar_last_error().decode())
