"""Python binding of the C ABI: torch tensors in, torch tensors out.

Argument marshalling only -- device memory and streams come from torch, and
every step of every computation runs in libitsolve.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

_METHODS = {"jacobi": L.ITS_JACOBI, "sgs": L.ITS_SGS, "gs": L.ITS_SGS, "cg": L.ITS_CG,
            "bicgstab": L.ITS_BICGSTAB, "cgnb": L.ITS_CG_NB}
_DTYPES = {"f64": L.ITS_F64, "f32": L.ITS_F32, "f16": L.ITS_F16}
_RESTART = {"cosine": L.ITS_RESTART_COSINE, "paper": L.ITS_RESTART_PAPER}
_STATUS = {L.ITS_OK: "ok", L.ITS_NOT_CONVERGED: "not_converged", L.ITS_BREAKDOWN: "breakdown"}


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(device=None) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _vec(t, n, name, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} elements")
    return t


class _Matrix:
    _h = None

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if self._h is not None and L is not None and L._lib is not None:
            L._lib.its_matrix_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def plan(self):
        """Brick plan of a matrix-free operator's SpMV sweep: (x tiles, y
        tiles, z chunks, planes per chunk)."""
        p = (C.c_int32 * 4)()
        L.check(L.lib().its_stencil_plan(self._h, p), "its_stencil_plan")
        return tuple(int(v) for v in p)


class CSRMatrix(_Matrix):
    """CSR matrix on the GPU: int32 or int64 row_ptr (n+1), int32 col,
    float64 val.  The handle borrows col and val (and an int32 row_ptr; an
    int64 one is narrowed by the library into a copy the handle owns); this
    object keeps the tensors alive."""

    def __init__(self, row_ptr, col, val, val32=None, val16=None, validate=True):
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        if not isinstance(row_ptr, torch.Tensor) or row_ptr.dtype not in (torch.int32, torch.int64):
            raise TypeError("row_ptr must be an int32 or int64 CUDA tensor")
        _vec(row_ptr, self.n + 1, "row_ptr", row_ptr.dtype)
        _vec(col, self.nnz, "col", torch.int32)
        _vec(val, self.nnz, "val")
        self.row_ptr, self.col, self.val = row_ptr, col, val
        h = C.c_void_p()
        if row_ptr.dtype == torch.int64:
            L.check(L.lib().its_csr_create64(self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(val),
                                             _stream(), C.byref(h)), "its_csr_create64")
        else:
            L.check(L.lib().its_csr_create(self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(val),
                                           C.byref(h)), "its_csr_create")
        self._h = h
        self.val32 = self.val16 = None
        if validate:
            L.check(L.lib().its_csr_validate(self._h, 0, _stream()), "its_csr_validate")
        if val32 is not None:
            self.set_lowp(val32)
        if val16 is not None:
            self.set_lowp(val16)
        self.colors = None

    @classmethod
    def from_numpy(cls, row_ptr, col, val, device="cuda", lowp=(), validate=True, pack=False,
                   max_fill=1.2):
        """Uploads host CSR arrays (an int64 row_ptr stays int64 and the
        library narrows it) and, for each dtype name in ``lowp`` ("f32",
        "f16"), a low-precision copy of the values made by the library's cast
        kernel; ``pack`` then builds the library's packed device layout
        (its_csr_pack with ``max_fill``)."""
        rp = np.asarray(row_ptr)
        rdt = np.int64 if rp.dtype == np.int64 else np.int32
        t_rp = torch.from_numpy(np.ascontiguousarray(rp, dtype=rdt)).to(device)
        t_col = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        t_val = torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).to(device)
        A = cls(t_rp, t_col, t_val, validate=validate)
        for d in lowp:
            A.set_lowp(cast_values(t_val, d))
        if pack:
            A.pack(max_fill)
        return A

    def pack(self, max_fill=1.2):
        """Builds the packed (sliced ELLPACK) device copy that solves and
        spmv then use; returns the number of slots it holds.  Refused
        (ItsError, ITS_E_UNSUPPORTED) when the rows would need more than
        max_fill * nnz + 64 slots."""
        L.check(L.lib().its_csr_pack(self._h, float(max_fill), _stream()), "its_csr_pack")
        return self.packed_slots

    @property
    def packed_slots(self) -> int:
        return int(L.lib().its_csr_packed_slots(self._h))

    @property
    def packed_column_slots(self) -> int:
        """Packed slots that still store a column index (0: all offset slices)."""
        return int(L.lib().its_csr_packed_column_slots(self._h))

    def build_transpose(self):
        """Builds A^T (device memory owned by the handle) for transposed
        solves; solve(..., transpose=True) calls it on first use."""
        L.check(L.lib().its_csr_transpose(self._h, _stream()), "its_csr_transpose")
        self.has_transpose = True

    def set_lowp(self, v):
        if v.dtype == torch.float32:
            dt = L.ITS_F32
            self.val32 = v
        elif v.dtype == torch.float16:
            dt = L.ITS_F16
            self.val16 = v
        else:
            raise ValueError("low-precision values must be float32 or float16")
        _vec(v, self.nnz, "val_lo", v.dtype)
        L.check(L.lib().its_csr_set_lowp(self._h, _ptr(v), dt), "its_csr_set_lowp")

    def set_colors(self, color, ncolors):
        """Point colouring for Gauss-Seidel: uint8 tensor of n colours."""
        if not isinstance(color, torch.Tensor):
            color = torch.from_numpy(np.ascontiguousarray(color, dtype=np.uint8)).cuda()
        _vec(color, self.n, "color", torch.uint8)
        L.check(L.lib().its_csr_set_colors(self._h, _ptr(color), int(ncolors), _stream()),
                "its_csr_set_colors")
        self.colors = color


class StencilMatrix(_Matrix):
    """Matrix-free constant-coefficient 7- or 27-point stencil on nx*ny*nz."""

    def __init__(self, nx, ny, nz, coef):
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        if coef.size not in (7, 27):
            raise ValueError("coef must hold 7 or 27 values")
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.coef = coef
        h = C.c_void_p()
        L.check(L.lib().its_stencil_create(self.nx, self.ny, self.nz, coef.size,
                                           coef.ctypes.data_as(C.c_void_p), C.byref(h)),
                "its_stencil_create")
        self._h = h


class VarCoefMatrix(_Matrix):
    """Matrix-free variable-coefficient diffusion on nx*ny*nz with per-cell
    coefficients k (float64 CUDA tensor of nx*ny*nz values, borrowed: this
    object keeps it alive)."""

    def __init__(self, nx, ny, nz, k):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.k = _vec(k, self.n, "k")
        h = C.c_void_p()
        L.check(L.lib().its_varcoef_create(self.nx, self.ny, self.nz, _ptr(self.k), C.byref(h)),
                "its_varcoef_create")
        self._h = h


def varcoef_grad(A, x, lam, dk=None):
    """dL/dk of a variable-coefficient operator given the solution x and the
    adjoint lam (A lam = dL/dx)."""
    x = _vec(x, A.n, "x")
    lam = _vec(lam, A.n, "lam")
    dk = torch.empty_like(x) if dk is None else _vec(dk, A.n, "dk")
    L.check(L.lib().its_varcoef_grad(A.handle, _ptr(x), _ptr(lam), _ptr(dk), _stream()),
            "its_varcoef_grad")
    return dk


def spmv(A, x, y=None):
    x = _vec(x, A.n, "x")
    y = torch.empty_like(x) if y is None else _vec(y, A.n, "y")
    L.check(L.lib().its_spmv(A.handle, _ptr(x), _ptr(y), _stream()), "its_spmv")
    return y


def dot(x, y) -> float:
    n = x.numel()
    _vec(x, n, "x")
    _vec(y, n, "y")
    ws = torch.empty(L.lib().its_dot_workspace_size(n), dtype=torch.uint8, device=x.device)
    out = C.c_double()
    L.check(L.lib().its_dot(n, _ptr(x), _ptr(y), C.byref(out), _ptr(ws), ws.numel(), _stream()),
            "its_dot")
    return out.value


def cast_values(v, dtype: str):
    out = torch.empty(v.numel(), device=v.device,
                      dtype={"f32": torch.float32, "f16": torch.float16}[dtype])
    L.check(L.lib().its_cast_values(_ptr(v), _ptr(out), _DTYPES[dtype], v.numel(), _stream()),
            "its_cast_values")
    return out


def stream_copy(src, dst):
    L.check(L.lib().its_stream_copy(_ptr(src), _ptr(dst), src.numel(), _stream()),
            "its_stream_copy")
    return dst


@dataclass
class SolveInfo:
    status: str
    code: int
    iters: int
    inner_iters: int
    restarts: int
    rel_res: float
    true_rel_res: float
    kernel_ms: list = field(default_factory=list)
    kernel_launches: list = field(default_factory=list)


def options(method="cg", rtol=1e-8, max_iter=10000, restart_tol=1e-5, restart_mode="cosine",
            inner_dtype="f64", inner_rtol=1e-4, max_outer=30, check_every=0, profile=False,
            transpose=False, graph=False, persistent=False):
    o = L.Options()
    L.lib().its_default_options(C.byref(o))
    o.method = _METHODS[method]
    o.rtol = rtol
    o.max_iter = max_iter
    o.restart_tol = restart_tol
    o.restart_mode = _RESTART[restart_mode]
    o.inner_dtype = _DTYPES[inner_dtype]
    o.inner_rtol = inner_rtol
    o.max_outer = max_outer
    o.check_every = check_every
    o.profile = int(profile)
    o.transpose = int(bool(transpose))
    o.graph = int(bool(graph))
    o.persistent = int(bool(persistent))
    return o


def workspace_bytes(A, **opts) -> int:
    o = options(**opts)
    nb = C.c_size_t()
    L.check(L.lib().its_workspace_size(A.handle, C.byref(o), C.byref(nb)), "its_workspace_size")
    return nb.value


def solve(A, b, x0=None, workspace=None, **opts):
    """Solves A x = b.  Returns (x, SolveInfo); raises ItsError on invalid
    arguments.  x0 (optional) is copied; pass ``x=`` semantics via x0."""
    b = _vec(b, A.n, "b")
    x = torch.zeros_like(b) if x0 is None else _vec(x0, A.n, "x0").clone()
    if opts.get("transpose") and isinstance(A, CSRMatrix) and not getattr(A, "has_transpose", False):
        A.build_transpose()
    o = options(**opts)
    nb = C.c_size_t()
    L.check(L.lib().its_workspace_size(A.handle, C.byref(o), C.byref(nb)), "its_workspace_size")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=b.device)
    r = L.Result()
    st = L.check(L.lib().its_solve(A.handle, C.byref(o), _ptr(b), _ptr(x), _ptr(workspace),
                                   workspace.numel(), _stream(), C.byref(r)), "its_solve")
    info = SolveInfo(_STATUS.get(st, str(st)), st, r.iters, r.inner_iters, r.restarts,
                     r.rel_res, r.true_rel_res, list(r.kernel_ms), list(r.kernel_launches))
    return x, info


def solve_noalloc(A, b, x, **opts):
    """Solves A x = b in place of x (holding x0) with its_solve_noalloc: the
    workspace is the library's static device scratch, so this call allocates
    no device memory (b and x are the caller's).  Returns SolveInfo."""
    b = _vec(b, A.n, "b")
    x = _vec(x, A.n, "x")
    o = options(**opts)
    r = L.Result()
    st = L.check(L.lib().its_solve_noalloc(A.handle, C.byref(o), _ptr(b), _ptr(x), _stream(),
                                           C.byref(r)), "its_solve_noalloc")
    return SolveInfo(_STATUS.get(st, str(st)), st, r.iters, r.inner_iters, r.restarts,
                     r.rel_res, r.true_rel_res, list(r.kernel_ms), list(r.kernel_launches))


class _DiffusionSolve(torch.autograd.Function):
    """x = A(k)^{-1} b for the variable-coefficient diffusion operator.
    Backward: one adjoint solve A lam = dL/dx (A is symmetric), then
    dL/db = lam and dL/dk from the gradient kernel.  Only x is kept for the
    backward pass; the forward iterates are not stored."""

    @staticmethod
    def forward(ctx, k, b, shape, opts):
        A = VarCoefMatrix(*shape, k.detach())
        x, info = solve(A, b.detach(), **opts)
        if info.status != "ok":
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(k, x)
        ctx.shape, ctx.opts = shape, opts
        return x

    @staticmethod
    def backward(ctx, gx):
        k, x = ctx.saved_tensors
        A = VarCoefMatrix(*ctx.shape, k.detach())
        lam, info = solve(A, gx.contiguous(), **ctx.opts)
        if info.status != "ok":
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        dk = varcoef_grad(A, x, lam)
        return dk, lam, None, None


def diffusion_solve(k, b, shape, method="cg", rtol=1e-10, max_iter=20000, **opts):
    """Differentiable solve of the variable-coefficient diffusion system
    A(k) x = b on a grid of ``shape`` = (nx, ny, nz): gradients flow to the
    per-cell coefficients k and to b."""
    o = dict(method=method, rtol=rtol, max_iter=max_iter, **opts)
    return _DiffusionSolve.apply(k, b, tuple(int(v) for v in shape), o)


class _StencilSolve(torch.autograd.Function):
    """x = A^{-1} b for a constant stencil (any method); backward solves
    A^T lam = dL/dx with the reflected stencil (dL/db = lam)."""

    @staticmethod
    def forward(ctx, b, A, opts):
        x, info = solve(A, b.detach(), **opts)
        if info.status != "ok":
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.A, ctx.opts = A, opts
        return x

    @staticmethod
    def backward(ctx, gx):
        lam, info = solve(ctx.A, gx.contiguous(), transpose=True, **ctx.opts)
        if info.status != "ok":
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        return lam, None, None


class _CsrSolve(torch.autograd.Function):
    """x = A^{-1} b for a CSR matrix whose values are a tensor (any method
    but Gauss-Seidel).  Backward: one adjoint solve A^T lam = dL/dx, then
    dL/db = lam and dL/dval from the value-gradient kernel."""

    @staticmethod
    def forward(ctx, val, b, A, opts):
        x, info = solve(A, b.detach(), **opts)
        if info.status != "ok":
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(x)
        ctx.A, ctx.opts = A, opts
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        A = ctx.A
        lam, info = solve(A, gx.contiguous(), transpose=True, **ctx.opts)
        if info.status != "ok":
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        dval = None
        if ctx.needs_input_grad[0]:
            dval = torch.empty_like(A.val)
            L.check(L.lib().its_csr_value_grad(A.handle, _ptr(x), _ptr(lam), _ptr(dval), _stream()),
                    "its_csr_value_grad")
        return dval, lam, None, None


def csr_solve(A, b, method="bicgstab", rtol=1e-10, max_iter=20000, **opts):
    """Differentiable solve with a CSR matrix: gradients flow to b and to the
    stored values A.val (a float64 CUDA tensor; mark it requires_grad) through
    the transposed (adjoint) solve.  The values must not change while the
    graph is alive (the handle borrows them)."""
    o = dict(method=method, rtol=rtol, max_iter=max_iter, **opts)
    return _CsrSolve.apply(A.val, b, A, o)


def stencil_solve(A, b, method="bicgstab", rtol=1e-10, max_iter=20000, **opts):
    """Differentiable solve with a constant-stencil operator: gradients flow
    to b through the transposed (adjoint) solve."""
    o = dict(method=method, rtol=rtol, max_iter=max_iter, **opts)
    return _StencilSolve.apply(b, A, o)


@dataclass
class BatchInfo:
    status: str
    iters: np.ndarray       # [nsys, nrhs]
    statuses: np.ndarray    # [nsys, nrhs] ITS_OK / ITS_NOT_CONVERGED / ITS_BREAKDOWN
    tiles_per_item: int
    planes_per_brick: int
    graph_iters: int
    max_iters: int
    replays: int
    tune_ms: float
    solve_ms: float


class Batch:
    """Many variable-coefficient diffusion systems (dims: sequence of
    (nx, ny, nz)) with nrhs right-hand sides each, solved together by FP64 CG
    per (system, rhs).  k: float64 CUDA tensor of the systems' per-cell
    coefficients concatenated.  Vectors hold cells * nrhs values, (cell g,
    rhs r) at g * nrhs + r."""

    def __init__(self, dims, k, nrhs):
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1, 3))
        self.dims = d
        self.nsys, self.nrhs = d.shape[0], int(nrhs)
        self.cells = int(np.sum(np.prod(d.astype(np.int64), axis=1)))
        _vec(k, self.cells, "k")
        h = C.c_void_p()
        L.check(L.lib().its_batch_create(self.nsys, d.ctypes.data_as(C.c_void_p), _ptr(k),
                                         self.nrhs, _stream(), C.byref(h)), "its_batch_create")
        self._h = h
        self._ws = None

    def __del__(self):
        if getattr(self, "_h", None) is not None and L is not None and L._lib is not None:
            L._lib.its_batch_destroy(self._h)
            self._h = None

    def offsets(self):
        """First cell of each system."""
        n = np.prod(self.dims.astype(np.int64), axis=1)
        return np.concatenate([[0], np.cumsum(n)[:-1]])

    def set_schedule(self, tiles_per_item=0, planes_per_brick=0):
        """Fix the work-item length of the update passes (tiles of 256/nrhs
        cells) and the z planes per brick of the SpMV pass; 0 for either:
        chosen by the autotuner at the next solve."""
        L.check(L.lib().its_batch_set_schedule(self._h, int(tiles_per_item), int(planes_per_brick)),
                "its_batch_set_schedule")

    def solve(self, b, x0=None, rtol=1e-8, max_iter=10000, check_every=0):
        n = self.cells * self.nrhs
        b = _vec(b, n, "b")
        x = torch.zeros_like(b) if x0 is None else _vec(x0, n, "x0").clone()
        nb = L.lib().its_batch_workspace_size(self._h)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=b.device)
        o = options(method="cg", rtol=rtol, max_iter=max_iter, check_every=check_every)
        r = L.BatchResult()
        iters = np.zeros(self.nsys * self.nrhs, np.int64)
        stats = np.zeros(self.nsys * self.nrhs, np.int32)
        st = L.check(L.lib().its_batch_solve(self._h, C.byref(o), _ptr(b), _ptr(x), _ptr(self._ws),
                                             self._ws.numel(), _stream(), C.byref(r),
                                             iters.ctypes.data_as(C.c_void_p),
                                             stats.ctypes.data_as(C.c_void_p)), "its_batch_solve")
        info = BatchInfo(_STATUS.get(st, str(st)), iters.reshape(self.nsys, self.nrhs),
                         stats.reshape(self.nsys, self.nrhs), r.tiles_per_item, r.planes_per_brick, r.graph_iters,
                         r.max_iters, r.replays, r.tune_ms, r.solve_ms)
        return x, info
