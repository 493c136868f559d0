"""ctypes wrapper of the reference oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU library never imports it.  All arrays are numpy, on the host.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

OK, NOT_CONVERGED, BREAKDOWN, E_INVALID = 0, 1, 2, -1
RESTART_COSINE, RESTART_PAPER = 0, 1


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iters", C.c_int64),
                ("inner_iters", C.c_int64), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double)]


@dataclass
class Result:
    status: int
    iters: int
    inner_iters: int
    restarts: int
    rel_res: float
    true_rel_res: float


_lib = None


def load(path):
    """Load an oracle shared library from ``path`` and declare its signatures."""
    L = C.CDLL(path)
    P = C.c_void_p
    I64, I32, D = C.c_int64, C.c_int32, C.c_double
    L.orc_dot.restype = D
    L.orc_dot.argtypes = [I64, P, P]
    L.orc_dot_f32.restype = D
    L.orc_dot_f32.argtypes = [I64, P, P]
    L.orc_spmv.argtypes = [I64, P, P, P, P, P]
    L.orc_spmv_f32.argtypes = [I64, P, P, P, P, P]
    L.orc_jacobi.argtypes = [I64, P, P, P, P, P, D, I64, P]
    L.orc_sgs.argtypes = [I64, P, P, P, P, I32, P, P, D, I64, P]
    L.orc_cg.argtypes = [I64, P, P, P, P, P, D, I64, P]
    L.orc_cgnb.argtypes = [I64, P, P, P, P, P, D, I64, P]
    L.orc_bicgstab.argtypes = [I64, P, P, P, P, P, D, I64, D, I32, P]
    L.orc_ir_cg.argtypes = [I64, P, P, P, P, P, P, D, I64, D, I64, P]
    L.orc_lu_solve.argtypes = [I64, P, P]
    L.orc_varcoef_csr.restype = I64
    L.orc_varcoef_csr.argtypes = [I32, I32, I32, P, P, P, P]
    L.orc_varcoef_grad.restype = None
    L.orc_varcoef_grad.argtypes = [I32, I32, I32, P, P, P, P]
    for f in ("orc_jacobi", "orc_sgs", "orc_cg", "orc_cgnb", "orc_bicgstab", "orc_ir_cg",
              "orc_lu_solve"):
        getattr(L, f).restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = load(_build.LIB)
    return _lib


def use_library(L):
    """Swap the loaded library (used by the mutation tests); returns the old one."""
    global _lib
    old, _lib = _lib, L
    return old


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _csr(A):
    rp, col, val = A
    return (np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32),
            _f64(val))


def _res(r):
    return Result(int(r.status), int(r.iters), int(r.inner_iters), int(r.restarts),
                  float(r.rel_res), float(r.true_rel_res))


def dot(x, y) -> float:
    """Exact sum of x_i*y_i rounded once to double."""
    x, y = _f64(x), _f64(y)
    assert x.shape == y.shape
    return lib().orc_dot(x.size, _p(x), _p(y))


def dot_f32(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape == y.shape
    return lib().orc_dot_f32(x.size, _p(x), _p(y))


def spmv(A, x) -> np.ndarray:
    rp, col, val = _csr(A)
    x = _f64(x)
    y = np.empty(rp.size - 1, np.float64)
    lib().orc_spmv(y.size, _p(rp), _p(col), _p(val), _p(x), _p(y))
    return y


def spmv_f32(A, val32, x32) -> np.ndarray:
    rp, col, _ = _csr(A)
    v = np.ascontiguousarray(val32, dtype=np.float32)
    x = np.ascontiguousarray(x32, dtype=np.float32)
    y = np.empty(rp.size - 1, np.float32)
    lib().orc_spmv_f32(y.size, _p(rp), _p(col), _p(v), _p(x), _p(y))
    return y


def _prep(A, b, x0):
    rp, col, val = _csr(A)
    n = rp.size - 1
    b = _f64(b)
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    return rp, col, val, n, b, x


def jacobi(A, b, x0=None, rtol=1e-8, max_iter=1000):
    rp, col, val, n, b, x = _prep(A, b, x0)
    r = _Result()
    lib().orc_jacobi(n, _p(rp), _p(col), _p(val), _p(b), _p(x), rtol, max_iter, C.byref(r))
    return x, _res(r)


def sgs(A, colors, ncolors, b, x0=None, rtol=1e-8, max_iter=1000):
    rp, col, val, n, b, x = _prep(A, b, x0)
    c = np.ascontiguousarray(colors, dtype=np.uint8)
    r = _Result()
    lib().orc_sgs(n, _p(rp), _p(col), _p(val), _p(c), ncolors, _p(b), _p(x), rtol, max_iter,
                  C.byref(r))
    return x, _res(r)


def cg(A, b, x0=None, rtol=1e-8, max_iter=1000):
    rp, col, val, n, b, x = _prep(A, b, x0)
    r = _Result()
    lib().orc_cg(n, _p(rp), _p(col), _p(val), _p(b), _p(x), rtol, max_iter, C.byref(r))
    return x, _res(r)


def cgnb(A, b, x0=None, rtol=1e-8, max_iter=1000):
    """The paper's nonblocking CG (Algorithm 1, sign of the x update fixed)."""
    rp, col, val, n, b, x = _prep(A, b, x0)
    r = _Result()
    lib().orc_cgnb(n, _p(rp), _p(col), _p(val), _p(b), _p(x), rtol, max_iter, C.byref(r))
    return x, _res(r)


def bicgstab(A, b, x0=None, rtol=1e-8, max_iter=1000, restart_tol=1e-5,
             restart_mode=RESTART_COSINE):
    rp, col, val, n, b, x = _prep(A, b, x0)
    r = _Result()
    lib().orc_bicgstab(n, _p(rp), _p(col), _p(val), _p(b), _p(x), rtol, max_iter,
                       restart_tol, restart_mode, C.byref(r))
    return x, _res(r)


def ir_cg(A, val_lo, b, x0=None, rtol=1e-8, max_iter=10000, inner_rtol=1e-4, max_outer=50):
    """val_lo: the stored low-precision values (float32, or float16 widened)."""
    rp, col, val, n, b, x = _prep(A, b, x0)
    vl = np.ascontiguousarray(np.asarray(val_lo).astype(np.float32))
    r = _Result()
    lib().orc_ir_cg(n, _p(rp), _p(col), _p(val), _p(vl), _p(b), _p(x), rtol, max_iter,
                    inner_rtol, max_outer, C.byref(r))
    return x, _res(r)


def lu_solve(a, b):
    a = _f64(a).copy()
    b = _f64(b).copy()
    n = b.size
    assert a.shape == (n, n)
    st = lib().orc_lu_solve(n, _p(a), _p(b))
    if st != OK:
        raise ValueError("singular matrix")
    return b


def csr_to_dense(A) -> np.ndarray:
    rp, col, val = _csr(A)
    n = rp.size - 1
    d = np.zeros((n, n))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            d[i, col[k]] += val[k]
    return d


def varcoef_csr(nx, ny, nz, k):
    """CSR (row_ptr int64, col int32, val float64) of the variable-coefficient
    diffusion operator with per-cell coefficients k (harmonic face means,
    boundary face = the cell's own k)."""
    k = _f64(k)
    n = nx * ny * nz
    assert k.size == n
    cap = 7 * n
    rp = np.empty(n + 1, np.int64)
    col = np.empty(max(cap, 1), np.int32)
    val = np.empty(max(cap, 1), np.float64)
    nnz = lib().orc_varcoef_csr(nx, ny, nz, _p(k), _p(rp), _p(col), _p(val))
    return rp, col[:nnz].copy(), val[:nnz].copy()


def varcoef_grad(nx, ny, nz, k, x, lam):
    """dL/dk for A(k) x = b, given x and the adjoint lam (A lam = dL/dx)."""
    k, x, lam = _f64(k), _f64(x), _f64(lam)
    dk = np.empty(k.size, np.float64)
    lib().orc_varcoef_grad(nx, ny, nz, _p(k), _p(x), _p(lam), _p(dk))
    return dk
