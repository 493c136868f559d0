"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmarks.

This module defines *problems*, not the solvers: the sparsity structure and
coefficients of the finite-difference operators the paper solves, random
vectors drawn from fixed seeds, and colourings.  It contains none of the
solvers' arithmetic (no products, dots or updates), so both the oracle and the
HIP path may consume what it produces.

Operators (paper, "Description of the algorithms" and "Numerical setup"):
the paper's systems come from 7-point and 27-point centred stencils on a
three-dimensional structured hexahedral mesh, stored in CSR.  Rows are grid
nodes numbered with x fastest, ``row = i + nx*(j + ny*k)``; neighbours that
fall outside the grid are omitted (homogeneous Dirichlet boundary), so every
CSR row lists its columns in strictly ascending order.

Coefficient sets (all exact binary values):

* Poisson 7-point: centre 6, the six face neighbours -1 (h^2 scaling dropped).
* 27-point: centre 26, the 26 neighbours -1 (the HPCG-style operator).
* Upwind convection-diffusion 7-point, velocity (1,1,1), cell Peclet 10 on
  each axis: centre 6 + 3*10 = 36, upstream neighbours (i-1, j-1, k-1)
  -(1+10) = -11, downstream neighbours -1.

The stencil offsets are always listed in ascending column order, i.e. the
order in which a CSR row stores them.
"""
from __future__ import annotations

import numpy as np

# Offsets of the 7-point stencil as (dk, dj, di), ascending in column index.
OFFSETS7 = ((-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0))
# Offsets of the 27-point stencil, ascending in column index (k outer, i inner).
OFFSETS27 = tuple((dk, dj, di) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1))

POISSON7 = (-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0)
STENCIL27 = tuple(26.0 if o == (0, 0, 0) else -1.0 for o in OFFSETS27)


def convdiff7(peclet: float = 10.0) -> tuple:
    """First-order upwind convection-diffusion, velocity (1,1,1), cell Peclet
    ``peclet`` on each axis: centre 6+3Pe, upstream -(1+Pe), downstream -1."""
    lo = -(1.0 + peclet)
    return (lo, lo, lo, 6.0 + 3.0 * peclet, -1.0, -1.0, -1.0)


def stencil_csr(nx: int, ny: int, nz: int, coef, offsets=None):
    """CSR arrays (row_ptr int64, col int32, val float64) of a constant-
    coefficient stencil on an nx*ny*nz grid with neighbours outside the grid
    omitted.  ``coef`` lists one value per offset, in ascending column order."""
    coef = tuple(float(c) for c in coef)
    if offsets is None:
        offsets = OFFSETS7 if len(coef) == 7 else OFFSETS27
    assert len(offsets) == len(coef)
    n = nx * ny * nz
    if n == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float64)
    k, j, i = np.meshgrid(np.arange(nz, dtype=np.int64), np.arange(ny, dtype=np.int64),
                          np.arange(nx, dtype=np.int64), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    rows = np.arange(n, dtype=np.int64)
    npts = len(offsets)
    counts = np.zeros(n, dtype=np.int64)
    masks = []
    for (dk, dj, di) in offsets:
        m = np.ones(n, dtype=bool)
        if di:
            m &= (i + di >= 0) & (i + di < nx)
        if dj:
            m &= (j + dj >= 0) & (j + dj < ny)
        if dk:
            m &= (k + dk >= 0) & (k + dk < nz)
        masks.append(m)
        counts += m
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    # position of the next free slot in each row; offsets are visited in
    # ascending column order, so each row ends up sorted.
    pos = row_ptr[:-1].copy()
    for o, (dk, dj, di) in enumerate(offsets):
        m = masks[o]
        idx = pos[m]
        col[idx] = (rows[m] + di + nx * (dj + ny * dk)).astype(np.int32)
        val[idx] = coef[o]
        pos[m] += 1
    del masks, pos
    return row_ptr, col, val


def poisson7_csr(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return stencil_csr(nx, ny, nz, POISSON7, OFFSETS7)


def stencil27_csr(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return stencil_csr(nx, ny, nz, STENCIL27, OFFSETS27)


def convdiff7_csr(nx, ny=None, nz=None, peclet=10.0):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return stencil_csr(nx, ny, nz, convdiff7(peclet), OFFSETS7)


def nnz_stencil7(nx, ny, nz):
    """Closed form: 7n minus one per missing face neighbour."""
    n = nx * ny * nz
    return 7 * n - 2 * (ny * nz + nx * nz + nx * ny)


def nnz_stencil27(nx, ny, nz):
    """Closed form: each axis contributes (3n_d - 2) neighbour pairs."""
    return (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)


def uniform_vector(n: int, seed, low=-1.0, high=1.0) -> np.ndarray:
    """x ~ U[low, high) i.i.d. from numpy's PCG64 ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(low, high, n)


def integer_vector(n: int, seed, lo=-8, hi=8) -> np.ndarray:
    """Small random integers as float64 (products and sums with the integer
    stencils above stay exact)."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.float64)


def redblack_colors(nx, ny, nz) -> np.ndarray:
    """Point red-black colouring: colour (i+j+k) mod 2, 0 = red."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) & 1).astype(np.uint8).ravel()


def octant_colors(nx, ny, nz) -> np.ndarray:
    """Eight-colour point colouring (i mod 2) + 2 (j mod 2) + 4 (k mod 2), an
    independent-set colouring for the 27-point stencil."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i & 1) + 2 * (j & 1) + 4 * (k & 1)).astype(np.uint8).ravel()


def sine_mode(nx, ny, nz, growth=(1.0, 1.0, 1.0)) -> np.ndarray:
    """v_ijk = g_x^(i+1) sin((i+1) pi hx) * (same in y, z) with h_d = 1/(n_d+1):
    the slowest error mode of the Dirichlet stencils (growth 1), or of the
    upwind operator when ``growth`` = sqrt(lower/upper) per axis."""
    def axis(m, g):
        t = np.arange(1, m + 1, dtype=np.float64)
        return (g ** t) * np.sin(t * np.pi / (m + 1))
    vx, vy, vz = axis(nx, growth[0]), axis(ny, growth[1]), axis(nz, growth[2])
    return (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).ravel()


def gaussian_field(n: int, seed, sigma=1.0) -> np.ndarray:
    """i.i.d. N(0, sigma^2) per cell (a log-coefficient field g or theta)."""
    return np.random.default_rng(seed).standard_normal(n) * sigma


def diffusion_coefficients(g) -> np.ndarray:
    """Per-cell diffusion coefficients k = exp(g)."""
    return np.exp(np.asarray(g, dtype=np.float64))


def batch_systems(nsys: int, nrhs: int, seed=4, side_lo=16, side_hi=64, sigma=1.0):
    """Uneven variable-coefficient systems for the batched solve: system s
    draws its three grid sides from U{side_lo..side_hi}, then a N(0, sigma^2)
    log-coefficient per cell, then nrhs right-hand sides U[-1, 1) per cell,
    all from default_rng([seed, s]).  Returns (dims [nsys, 3], k concatenated
    over the systems, b [cells, nrhs] with the right-hand sides of a cell
    adjacent)."""
    dims, ks, bs = [], [], []
    for s in range(nsys):
        rng = np.random.default_rng([seed, s])
        d = rng.integers(side_lo, side_hi + 1, size=3)
        n = int(np.prod(d))
        dims.append(d)
        ks.append(np.exp(rng.standard_normal(n) * sigma))
        bs.append(rng.uniform(-1.0, 1.0, size=(n, nrhs)))
    return (np.array(dims, dtype=np.int32), np.concatenate(ks),
            np.concatenate(bs).astype(np.float64))
