"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/rls.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2306_11067_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rls.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rls_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_null_arguments_rejected_without_gpu():
    lib = L.load()
    h = C.c_void_p()
    assert lib.rls_setup(C.byref(h), None, None, None, None) == L.RLS_E_ARG
    assert b"null" in lib.rls_last_error()
    assert lib.rls_set_weights(None, None, None) == L.RLS_E_STATE
    assert lib.rls_solve_sweep(None, None, None, 0, 1e-8, None, None, None,
                               None, None, None, None) == L.RLS_E_STATE


@pytest.mark.parametrize("field,value", [
    ("nv", 6),            # not divisible by 2^(levels-1) = 4
    ("levels", 0),
    ("nu", 0),
    ("cheb_ratio", 1.0),
    ("precision", 7),
])
def test_grid_validation_without_gpu(field, value):
    lib = L.load()
    taps = (C.c_double * 3)(0.25, 0.5, 0.25)
    op = L.OpDesc()
    op.kind = L.RLS_OP_BLUR_SEPARABLE
    op.bc = L.RLS_BC_REFLECTIVE
    op.r_v = op.r_h = 1
    op.taps_v = op.taps_h = C.cast(taps, C.POINTER(C.c_double))
    g = L.GridDesc(64, 64, L.RLS_L_NEUMANN, 3, 2, 4.0, L.RLS_PREC_FP64, 0, 0.0)
    setattr(g, field, value)
    h = C.c_void_p()
    st = lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), None, None)
    assert st in (L.RLS_E_ARG, L.RLS_E_UNSUPPORTED)
    assert lib.rls_last_error()


def test_coarsest_size_limit_without_gpu():
    lib = L.load()
    taps = (C.c_double * 3)(0.25, 0.5, 0.25)
    op = L.OpDesc()
    op.kind = L.RLS_OP_BLUR_SEPARABLE
    op.bc = L.RLS_BC_REFLECTIVE
    op.r_v = op.r_h = 1
    op.taps_v = op.taps_h = C.cast(taps, C.POINTER(C.c_double))
    g = L.GridDesc(128, 128, L.RLS_L_NEUMANN, 2, 2, 4.0, L.RLS_PREC_FP64, 0, 0.0)
    h = C.c_void_p()
    assert lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), None,
                         None) == L.RLS_E_ARG
    assert b"1024" in lib.rls_last_error()


def test_unsupported_boundary_pair_without_gpu():
    lib = L.load()
    taps = (C.c_double * 3)(0.25, 0.5, 0.25)
    op = L.OpDesc()
    op.kind = L.RLS_OP_BLUR_SEPARABLE
    op.bc = L.RLS_BC_REFLECTIVE
    op.r_v = op.r_h = 1
    op.taps_v = op.taps_h = C.cast(taps, C.POINTER(C.c_double))
    g = L.GridDesc(64, 64, L.RLS_L_PERIODIC, 3, 2, 4.0, L.RLS_PREC_FP64, 0, 0.0)
    h = C.c_void_p()
    assert lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), None,
                         None) == L.RLS_E_UNSUPPORTED


def test_blur_radius_beyond_lds_tile_rejected_without_gpu():
    lib = L.load()
    r = 40
    taps = (C.c_double * (2 * r + 1))(*([1.0 / (2 * r + 1)] * (2 * r + 1)))
    op = L.OpDesc()
    op.kind = L.RLS_OP_BLUR_SEPARABLE
    op.bc = L.RLS_BC_REFLECTIVE
    op.r_v = op.r_h = r
    op.taps_v = op.taps_h = C.cast(taps, C.POINTER(C.c_double))
    g = L.GridDesc(512, 512, L.RLS_L_NEUMANN, 5, 2, 4.0, L.RLS_PREC_FP64, 0, 0.0)
    h = C.c_void_p()
    assert lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), None,
                         None) == L.RLS_E_UNSUPPORTED
    assert b"LDS" in lib.rls_last_error()


def test_batch_argument_checks_without_gpu():
    lib = L.load()
    assert lib.rls_solve_batch(None, 0, None) == L.RLS_E_ARG
    arr = (L.Sweep * 2)()
    assert lib.rls_solve_batch(arr, 2, None) == L.RLS_E_ARG
    assert b"null handle" in lib.rls_last_error()
    fake = C.c_void_p(0x1000)   # never dereferenced: rejected as a duplicate
    arr[0].prob = fake
    arr[1].prob = fake
    assert lib.rls_solve_batch(arr, 2, None) == L.RLS_E_ARG
    assert b"twice" in lib.rls_last_error()


def test_sparse_operator_rejects_bf16_vcycle_without_gpu():
    """Sparse (tomography) operators run their V-cycle in FP32 only; the
    precision is checked on the host before anything reaches the GPU."""
    lib = L.load()
    rowptr = (C.c_int64 * 3)(0, 1, 2)
    col = (C.c_int32 * 2)(0, 1)
    val = (C.c_float * 2)(1.0, 1.0)
    op = L.OpDesc()
    op.kind = L.RLS_OP_CSR
    op.m, op.nnz = 2, 2
    op.rowptr = C.cast(rowptr, C.POINTER(C.c_int64))
    op.col = C.cast(col, C.POINTER(C.c_int32))
    op.val = C.cast(val, C.POINTER(C.c_float))
    g = L.GridDesc(64, 64, L.RLS_L_NEUMANN, 3, 2, 4.0, L.RLS_PREC_MIXED_BF16,
                   0, 0.0)
    h = C.c_void_p()
    st = lib.rls_setup(C.byref(h), C.byref(op), C.byref(g), None, None)
    assert st == L.RLS_E_UNSUPPORTED
    assert b"FP32" in lib.rls_last_error()
