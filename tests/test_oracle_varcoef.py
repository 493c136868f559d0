"""Pins of the oracle's variable-coefficient diffusion operator and of its
adjoint gradient (CPU).

The operator is pinned by reduction to the (6, -1) Laplacian at k = 1, by
exact symmetry, and against an independent assembly A = D^T K D from
face-difference incidence and series (half-cell) conductances.  The
gradient is pinned by central finite differences of L = 0.5 ||x - x_t||^2
with dense LU solves on tiny grids, independently of its formula.
"""
import numpy as np
import pytest

import oracle
from paper_2305_05988_amd import inputs


def _k(n, seed, sigma=1.0):
    return inputs.diffusion_coefficients(inputs.gaussian_field(n, seed, sigma))


def test_unit_coefficients_give_the_poisson_matrix():
    g = (5, 4, 3)
    A = oracle.varcoef_csr(*g, np.ones(60))
    P = inputs.poisson7_csr(*g)
    for a, p in zip(A, P):
        assert np.array_equal(a, p)


@pytest.mark.parametrize("g", [(1, 1, 1), (4, 3, 2), (5, 4, 3), (2, 6, 3)])
def test_operator_is_exactly_symmetric(g):
    n = int(np.prod(g))
    d = oracle.csr_to_dense(oracle.varcoef_csr(*g, _k(n, 3)))
    assert np.array_equal(d, d.T)


def _series_assembly(nx, ny, nz, k):
    """A = D^T K D: one row of D per face (interior: e_a - e_b; boundary: e_c),
    K the face conductance of two half-cells in series."""
    n = nx * ny * nz
    rows, cond = [], []
    for c in range(n):
        ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
        for axis, (pos, size, stride) in enumerate(((ix, nx, 1), (iy, ny, nx), (iz, nz, nx * ny))):
            for side in (-1, 1):
                q = pos + side
                if 0 <= q < size:
                    m = c + side * stride
                    if m < c:
                        continue  # each interior face once, from its upper cell
                    r = np.zeros(n)
                    r[c], r[m] = 1.0, -1.0
                    rows.append(r)
                    cond.append(1.0 / (1.0 / (2.0 * k[c]) + 1.0 / (2.0 * k[m])))
                else:
                    r = np.zeros(n)
                    r[c] = 1.0
                    rows.append(r)
                    cond.append(1.0 / (1.0 / (2.0 * k[c]) + 1.0 / (2.0 * k[c])))
    D = np.array(rows)
    return D.T @ np.diag(cond) @ D


@pytest.mark.parametrize("g", [(3, 3, 3), (4, 3, 2), (1, 5, 2)])
def test_operator_matches_face_flux_assembly(g):
    n = int(np.prod(g))
    k = _k(n, 11, sigma=1.5)
    d = oracle.csr_to_dense(oracle.varcoef_csr(*g, k))
    ref = _series_assembly(*g, k)
    assert np.max(np.abs(d - ref)) <= 1e-13 * np.max(np.abs(ref))


def _loss_and_solution(g, k, b, xt):
    A = oracle.csr_to_dense(oracle.varcoef_csr(*g, k))
    x = oracle.lu_solve(A, b)
    return 0.5 * float(np.sum((x - xt) ** 2)), x, A


@pytest.mark.parametrize("g", [(3, 3, 2), (4, 2, 3)])
def test_gradient_matches_central_differences(g):
    n = int(np.prod(g))
    k = _k(n, 5)
    b = inputs.uniform_vector(n, 6)
    xt = inputs.uniform_vector(n, 7)
    L, x, A = _loss_and_solution(g, k, b, xt)
    lam = oracle.lu_solve(A.T, x - xt)
    dk = oracle.varcoef_grad(*g, k, x, lam)
    fd = np.empty(n)
    for c in range(n):
        h = 1e-5 * k[c]
        kp, km = k.copy(), k.copy()
        kp[c] += h
        km[c] -= h
        fd[c] = (_loss_and_solution(g, kp, b, xt)[0] - _loss_and_solution(g, km, b, xt)[0]) / (2 * h)
    assert np.max(np.abs(dk - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_rhs_gradient_is_the_adjoint_solution():
    g = (3, 2, 2)
    n = 12
    k = _k(n, 8)
    b = inputs.uniform_vector(n, 9)
    xt = inputs.uniform_vector(n, 10)
    L, x, A = _loss_and_solution(g, k, b, xt)
    lam = oracle.lu_solve(A.T, x - xt)
    for c in range(n):
        h = 1e-4
        bp, bm = b.copy(), b.copy()
        bp[c] += h
        bm[c] -= h
        fd = (_loss_and_solution(g, k, bp, xt)[0] - _loss_and_solution(g, k, bm, xt)[0]) / (2 * h)
        assert abs(fd - lam[c]) <= 1e-7 * max(1.0, abs(lam[c]))


def test_cg_solves_the_variable_coefficient_system():
    g = (6, 5, 4)
    n = 120
    A = oracle.varcoef_csr(*g, _k(n, 12))
    xs = inputs.uniform_vector(n, 13)
    b = oracle.spmv(A, xs)
    x, r = oracle.cg(A, b, rtol=1e-12, max_iter=1000)
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    assert r.status == oracle.OK
    assert np.max(np.abs(x - ref)) <= 1e-9 * np.max(np.abs(ref))
