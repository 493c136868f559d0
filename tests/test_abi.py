"""The C ABI library loads on a machine without a GPU, exports every entry
point the header declares, and rejects bad arguments before touching HIP."""
import ctypes as C
import os
import re

import pytest

from paper_2305_05988_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "itsolve.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2305_05988_amd import build
        build.build()
    return L.load(L.LIB_PATH)


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(its_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(L.EXPORTS) == _declared()


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options(lib):
    o = L.Options()
    lib.its_default_options(C.byref(o))
    assert o.method == L.ITS_CG and o.rtol == 1e-8 and o.max_iter == 10000
    assert o.restart_tol == 1e-5 and o.restart_mode == L.ITS_RESTART_COSINE
    assert o.inner_dtype == L.ITS_F64 and o.profile == 0 and o.graph == 0 and o.transpose == 0


def test_status_strings(lib):
    for code, name in [(0, b"ITS_OK"), (1, b"ITS_NOT_CONVERGED"), (2, b"ITS_BREAKDOWN"),
                       (-1, b"ITS_E_INVALID"), (-2, b"ITS_E_HIP"), (-3, b"ITS_E_WORKSPACE"),
                       (-4, b"ITS_E_UNSUPPORTED")]:
        assert lib.its_status_string(code) == name


def test_host_side_argument_errors(lib):
    h = C.c_void_p()
    P0 = C.c_void_p(0)
    assert lib.its_csr_create(4, 4, P0, P0, P0, C.byref(h)) == L.ITS_E_INVALID
    assert b"null" in lib.its_last_error()
    assert lib.its_csr_create(-1, 0, P0, P0, P0, C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_csr_create(1 << 31, 1, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                              C.byref(h)) == L.ITS_E_UNSUPPORTED
    assert lib.its_csr_create64(4, 4, P0, P0, P0, P0, C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_csr_create64(4, -1, C.c_void_p(8), C.c_void_p(16), C.c_void_p(16), P0,
                                C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_csr_create64(8, 1 << 31, C.c_void_p(8), C.c_void_p(16), C.c_void_p(16), P0,
                                C.byref(h)) == L.ITS_E_UNSUPPORTED
    assert lib.its_csr_create64(4, 4, C.c_void_p(8), C.c_void_p(8), C.c_void_p(16), P0,
                                C.byref(h)) == L.ITS_E_INVALID  # col not 16-byte aligned
    assert lib.its_csr_create64(4, 4, C.c_void_p(8), C.c_void_p(16), C.c_void_p(16), P0,
                                P0) == L.ITS_E_INVALID
    coef = (C.c_double * 7)(*([1.0] * 7))
    assert lib.its_stencil_create(4, 4, 4, 5, coef, C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_stencil_create(2048, 2048, 1024, 7, coef, C.byref(h)) == L.ITS_E_UNSUPPORTED
    bad = (C.c_double * 7)(*([float("nan")] * 7))
    assert lib.its_stencil_create(4, 4, 4, 7, bad, C.byref(h)) == L.ITS_E_INVALID
    out = C.c_double()
    assert lib.its_dot(10, P0, P0, C.byref(out), P0, 0, P0) == L.ITS_E_INVALID
    assert lib.its_dot(10, C.c_void_p(8), C.c_void_p(8), C.byref(out), P0, 0, P0) == L.ITS_E_WORKSPACE
    r = L.Result()
    o = L.Options()
    lib.its_default_options(C.byref(o))
    assert lib.its_solve(P0, C.byref(o), P0, P0, P0, 0, P0, C.byref(r)) == L.ITS_E_INVALID
    assert lib.its_cast_values(P0, P0, 7, 10, P0) == L.ITS_E_INVALID
    assert lib.its_stream_copy(P0, P0, -1, P0) == L.ITS_E_INVALID
    assert lib.its_matrix_destroy(P0) == L.ITS_OK
    assert lib.its_matrix_rows(P0) == -1
    assert lib.its_csr_pack(P0, 1.2, P0) == L.ITS_E_INVALID
    dims = (C.c_int32 * 3)(4, 4, 4)
    assert lib.its_batch_create(1, dims, C.c_void_p(8), 3, P0, C.byref(h)) == L.ITS_E_UNSUPPORTED
    bad_dims = (C.c_int32 * 3)(4, 0, 4)
    assert lib.its_batch_create(1, bad_dims, C.c_void_p(8), 4, P0, C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_batch_create(0, dims, C.c_void_p(8), 4, P0, C.byref(h)) == L.ITS_E_INVALID
    # the SpMV pass keeps in-plane offsets in 32 bits: 2^31 cells per plane are refused
    wide = (C.c_int32 * 3)(1 << 16, 1 << 15, 1)
    assert lib.its_batch_create(1, wide, C.c_void_p(8), 4, P0, C.byref(h)) == L.ITS_E_UNSUPPORTED
    wide_ok = (C.c_int32 * 3)(1 << 16, (1 << 15) - 1, 0)  # fits, but empty: rejected as invalid
    assert lib.its_batch_create(1, wide_ok, C.c_void_p(8), 4, P0, C.byref(h)) == L.ITS_E_INVALID
    assert lib.its_batch_cells(P0) == -1 and lib.its_batch_workspace_size(P0) == 0
    assert lib.its_batch_set_schedule(P0, 4, 0) == L.ITS_E_INVALID
    assert lib.its_csr_transpose(P0, P0) == L.ITS_E_INVALID
    assert lib.its_csr_value_grad(P0, P0, P0, P0, P0) == L.ITS_E_INVALID
    assert lib.its_batch_destroy(P0) == L.ITS_OK
    assert lib.its_csr_packed_slots(P0) == 0
    assert lib.its_csr_packed_column_slots(P0) == 0
    plan = (C.c_int32 * 4)()
    assert lib.its_stencil_plan(P0, plan) == L.ITS_E_INVALID
