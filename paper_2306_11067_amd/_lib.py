"""ctypes declarations of the C-ABI in include/rls.h (argument marshalling
only; every computation happens inside librls.so)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librls.so")

RLS_OK = 0
RLS_E_ARG = -1
RLS_E_HIP = -2
RLS_E_OOM = -3
RLS_E_NOT_SPD = -4
RLS_E_UNSUPPORTED = -5
RLS_E_STATE = -6

RLS_OP_BLUR_SEPARABLE = 1
RLS_OP_CSR = 2
RLS_BC_PERIODIC, RLS_BC_REFLECTIVE, RLS_BC_ZERO = 0, 1, 2
RLS_L_NEUMANN, RLS_L_PERIODIC = 0, 1
RLS_PREC_FP64 = 0
RLS_PREC_MIXED_FP32 = 1
RLS_PREC_MIXED_BF16 = 2
RLS_TOL_RELATIVE, RLS_TOL_ABSOLUTE = 0, 1
RLS_FLAG_CONVERGED, RLS_FLAG_MAXIT = 1, 2
RLS_FLAG_BREAKDOWN, RLS_FLAG_NONFINITE = 4, 8

STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_HIP", -3: "E_OOM",
                -4: "E_NOT_SPD", -5: "E_UNSUPPORTED", -6: "E_STATE"}

# Every symbol include/rls.h declares.
EXPORTS = [
    "rls_setup", "rls_set_weights", "rls_solve_sweep", "rls_destroy",
    "rls_last_error", "rls_level_shape", "rls_apply_normal", "rls_vcycle",
    "rls_get_stencil", "rls_get_gram_band", "rls_gershgorin",
    "rls_apply_forward", "rls_apply_adjoint", "rls_kernel_timer",
    "rls_kernel_timer_read", "rls_solve_batch", "rls_update_weights",
    "rls_get_weights", "rls_lcurve_corner", "rls_trim_window",
    "rls_regularize",
]


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("bc", C.c_int), ("r_v", C.c_int),
                ("r_h", C.c_int), ("taps_v", C.POINTER(C.c_double)),
                ("taps_h", C.POINTER(C.c_double)), ("m", C.c_int64),
                ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_float))]


class GridDesc(C.Structure):
    _fields_ = [("nv", C.c_int), ("nh", C.c_int), ("lbc", C.c_int),
                ("levels", C.c_int), ("nu", C.c_int),
                ("cheb_ratio", C.c_double), ("precision", C.c_int),
                ("nu_coarse", C.c_int), ("cheb_ratio_coarse", C.c_double)]


class SweepOpts(C.Structure):
    _fields_ = [("maxit", C.c_int), ("tol_mode", C.c_int),
                ("poll_every", C.c_int), ("graph", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("flags", C.c_int),
                ("relres", C.c_double), ("relres_true", C.c_double)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)


class OuterInfo(C.Structure):
    _fields_ = [("outer", C.c_int), ("stopped", C.c_int),
                ("chosen_index", C.c_int), ("iters", C.c_longlong)]


class Sweep(C.Structure):
    _fields_ = [("prob", _P), ("b", _P), ("lam", _D), ("nlam", C.c_int),
                ("tol", C.c_double), ("opts", C.POINTER(SweepOpts)),
                ("x0", _P), ("x", _P), ("resnorm", _D), ("seminorm", _D),
                ("info", C.POINTER(SolveInfo)), ("status", C.c_int)]


def _declare(lib):
    lib.rls_setup.argtypes = [C.POINTER(_P), C.POINTER(OpDesc),
                              C.POINTER(GridDesc), _P, _P]
    lib.rls_set_weights.argtypes = [_P, _P, _P]
    lib.rls_solve_sweep.argtypes = [_P, _P, _D, C.c_int, C.c_double,
                                    C.POINTER(SweepOpts), _P, _P, _D, _D,
                                    C.POINTER(SolveInfo), _P]
    lib.rls_destroy.argtypes = [_P]
    lib.rls_destroy.restype = None
    lib.rls_last_error.argtypes = []
    lib.rls_last_error.restype = C.c_char_p
    lib.rls_level_shape.argtypes = [_P, C.c_int, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
    lib.rls_apply_normal.argtypes = [_P, C.c_int, _D, C.c_int, _P, _P, _P]
    lib.rls_vcycle.argtypes = [_P, _D, C.c_int, _P, _P, _P]
    lib.rls_get_stencil.argtypes = [_P, C.c_int, _D]
    lib.rls_get_gram_band.argtypes = [_P, C.c_int, C.c_int,
                                      C.POINTER(C.c_int), _D]
    lib.rls_gershgorin.argtypes = [_P, C.c_int, _D, C.c_int, _D, _P]
    lib.rls_apply_forward.argtypes = [_P, _P, _P, C.c_int, _P]
    lib.rls_apply_adjoint.argtypes = [_P, _P, _P, C.c_int, _P]
    lib.rls_kernel_timer.argtypes = [_P, C.c_int]
    lib.rls_solve_batch.argtypes = [C.POINTER(Sweep), C.c_int, _P]
    lib.rls_kernel_timer_read.argtypes = [_P, C.POINTER(C.c_longlong),
                                          C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
    lib.rls_update_weights.argtypes = [_P, _P, C.c_double, _D, _P]
    lib.rls_get_weights.argtypes = [_P, _P, _P]
    lib.rls_lcurve_corner.argtypes = [_D, _D, _D, C.c_int,
                                      C.POINTER(C.c_int)]
    lib.rls_trim_window.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
    lib.rls_regularize.argtypes = [_P, _P, _D, C.c_int, C.c_double,
                                   C.c_double, C.POINTER(SweepOpts), C.c_int,
                                   C.POINTER(C.c_int), _P,
                                   C.POINTER(OuterInfo), _P]
    for name in EXPORTS:
        if name not in ("rls_destroy", "rls_last_error"):
            getattr(lib, name).restype = C.c_int
    return lib


_lib = None


def load():
    """Load librls.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2306_11067_amd.build` (hipcc, gfx950)")
        # torch ships its own HIP runtime; load it first so that the
        # library's HIP dependency resolves to the runtime torch uses (a
        # second runtime in the process finds no device once torch has
        # opened it)
        import torch  # noqa: F401
        _lib = _declare(C.CDLL(LIB_PATH))
    return _lib
