"""its_solve_noalloc, the solve whose workspace is the library's static
device scratch: through the C ABI, two calls in a row (the second on a
smaller system, so it runs on what the first left in the scratch) give the
same status, counts and iterate, bit for bit, as its_solve with a caller
workspace; sizes beyond the scratch and the options that would create HIP
objects are refused before any device work."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2305_05988_amd import _lib as L
from paper_2305_05988_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def its():
    import paper_2305_05988_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(msg):
    print(f"no-alloc: {msg}", flush=True)


def _opts(**kw):
    o = L.Options()
    L.lib().its_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _pair(A, b, o):
    """(status, result, x) of its_solve with a torch workspace and of
    its_solve_noalloc, both from x0 = 0, called through the C ABI."""
    lib = L.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    nb = C.c_size_t()
    assert lib.its_workspace_size(A.handle, C.byref(o), C.byref(nb)) == L.ITS_OK
    assert nb.value <= L.NOALLOC_SCRATCH_BYTES
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r1 = L.Result()
    st1 = lib.its_solve(A.handle, C.byref(o), C.c_void_p(b.data_ptr()), C.c_void_p(x1.data_ptr()),
                        C.c_void_p(ws.data_ptr()), nb.value, s, C.byref(r1))
    x2 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r2 = L.Result()
    st2 = lib.its_solve_noalloc(A.handle, C.byref(o), C.c_void_p(b.data_ptr()),
                                C.c_void_p(x2.data_ptr()), s, C.byref(r2))
    torch.cuda.synchronize()
    return (st1, r1, x1.cpu().numpy()), (st2, r2, x2.cpu().numpy())


def _same(a, b):
    (st1, r1, x1), (st2, r2, x2) = a, b
    assert st1 == st2 and r1.status == r2.status
    assert r1.iters == r2.iters and r1.inner_iters == r2.inner_iters and r1.restarts == r2.restarts
    assert r1.rel_res == r2.rel_res and r1.true_rel_res == r2.true_rel_res
    assert np.array_equal(x1, x2)


def test_noalloc_two_calls_match_its_solve():
    # call 1: 48^3 Poisson in the packed CSR layout, CG to 1e-10
    say("call 1: CG, 48^3 Poisson, packed CSR")
    Acsr = inputs.poisson7_csr(48)
    A = its().CSRMatrix.from_numpy(*Acsr, pack=True)
    b = oracle.spmv(Acsr, inputs.uniform_vector(A.n, 1))
    ref, rr = oracle.cg(Acsr, b, rtol=1e-10, max_iter=2000)
    a, c = _pair(A, dev(b), _opts(method=L.ITS_CG, rtol=1e-10, max_iter=2000))
    _same(a, c)
    assert c[0] == L.ITS_OK and c[1].iters == rr.iters and np.array_equal(c[2], ref)
    # call 2: a smaller system and another method, on the scratch call 1 left
    say("call 2: BiCGStab, 20x18x16 upwind, matrix-free stencil")
    g = (20, 18, 16)
    S = its().StencilMatrix(*g, inputs.convdiff7())
    Scsr = inputs.convdiff7_csr(*g)
    b2 = oracle.spmv(Scsr, inputs.uniform_vector(S.n, 2))
    ref2, rr2 = oracle.bicgstab(Scsr, b2, rtol=1e-10, max_iter=500)
    a, c = _pair(S, dev(b2), _opts(method=L.ITS_BICGSTAB, rtol=1e-10, max_iter=500))
    _same(a, c)
    assert c[0] == L.ITS_OK and c[1].iters == rr2.iters and np.array_equal(c[2], ref2)
    # and through the binding: Jacobi, fixed sweeps
    say("call 3: Jacobi, 5 sweeps, 20x18x16 upwind, binding")
    x = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    info = its().solve_noalloc(S, dev(b2), x, method="jacobi", rtol=0.0, max_iter=5)
    refj, _ = oracle.jacobi(Scsr, b2, rtol=0.0, max_iter=5)
    assert info.iters == 5 and np.array_equal(x.cpu().numpy(), refj)


def test_noalloc_refusals():
    lib = L.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = (160, 160, 160)  # CG needs 24 B per row: more than the scratch holds
    S = its().StencilMatrix(*g, inputs.POISSON7)
    b = torch.ones(S.n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    r = L.Result()
    args = (C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), s, C.byref(r))
    o = _opts(method=L.ITS_CG)
    assert lib.its_solve_noalloc(S.handle, C.byref(o), *args) == L.ITS_E_WORKSPACE
    assert b"static buffer" in lib.its_last_error()
    small = its().StencilMatrix(8, 8, 8, inputs.POISSON7)
    b8 = torch.ones(small.n, dtype=torch.float64, device="cuda")
    x8 = torch.zeros_like(b8)
    args8 = (C.c_void_p(b8.data_ptr()), C.c_void_p(x8.data_ptr()), s, C.byref(r))
    assert lib.its_solve_noalloc(small.handle, C.byref(_opts(graph=1)), *args8) == L.ITS_E_UNSUPPORTED
    assert lib.its_solve_noalloc(small.handle, C.byref(_opts(profile=1)), *args8) == L.ITS_E_UNSUPPORTED
    assert lib.its_solve_noalloc(None, C.byref(o), *args8) == L.ITS_E_INVALID
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0 and torch.count_nonzero(x8).item() == 0
