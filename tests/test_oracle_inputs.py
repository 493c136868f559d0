"""Pins of the problem generators (shared inputs) against independent
constructions: Kronecker sums of 1-D tridiagonal operators, closed-form nnz
counts, symmetry and row sums."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2305_05988_amd import inputs

GRIDS = [(1, 1, 1), (2, 3, 4), (5, 1, 7), (4, 4, 4), (7, 5, 3), (16, 9, 2)]


def _to_scipy(A):
    rp, col, val = A
    n = rp.size - 1
    return sp.csr_matrix((val, col.astype(np.int64), rp), shape=(n, n))


def _tri(m, lo, d, up):
    return sp.diags([np.full(m - 1, lo), np.full(m, d), np.full(m - 1, up)], [-1, 0, 1],
                    shape=(m, m))


def _kron3_sum(nx, ny, nz, tx, ty, tz):
    """Sum over axes of identity (x) T_d (x) identity, with x fastest."""
    ix, iy, iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(iz, sp.kron(iy, tx)) + sp.kron(iz, sp.kron(ty, ix)) +
            sp.kron(tz, sp.kron(iy, ix))).tocsr()


@pytest.mark.parametrize("g", GRIDS)
def test_poisson7_is_kronecker_laplacian(g):
    nx, ny, nz = g
    A = _to_scipy(inputs.poisson7_csr(nx, ny, nz))
    K = _kron3_sum(nx, ny, nz, _tri(nx, -1, 2, -1), _tri(ny, -1, 2, -1), _tri(nz, -1, 2, -1))
    assert abs(A - K).max() == 0 if A.nnz else K.nnz == 0


@pytest.mark.parametrize("g", GRIDS)
def test_convdiff7_is_kronecker_upwind(g):
    nx, ny, nz = g
    pe = 10.0
    A = _to_scipy(inputs.convdiff7_csr(nx, ny, nz, pe))
    t = lambda m: _tri(m, -(1 + pe), 2 + pe, -1)
    K = _kron3_sum(nx, ny, nz, t(nx), t(ny), t(nz))
    assert abs(A - K).max() == 0
    assert inputs.convdiff7(pe) == (-11.0, -11.0, -11.0, 36.0, -1.0, -1.0, -1.0)


@pytest.mark.parametrize("g", GRIDS)
def test_stencil27_is_27_minus_ones_band(g):
    nx, ny, nz = g
    A = _to_scipy(inputs.stencil27_csr(nx, ny, nz))
    band = lambda m: _tri(m, 1, 1, 1)
    J = sp.kron(band(nz), sp.kron(band(ny), band(nx))).tocsr()
    K = 27 * sp.identity(nx * ny * nz) - J
    assert abs(A - K).max() == 0


@pytest.mark.parametrize("g", GRIDS + [(32, 32, 32)])
def test_nnz_closed_forms(g):
    nx, ny, nz = g
    rp, col, val = inputs.poisson7_csr(nx, ny, nz)
    assert rp[-1] == col.size == val.size == inputs.nnz_stencil7(nx, ny, nz)
    rp, col, val = inputs.stencil27_csr(nx, ny, nz)
    assert rp[-1] == inputs.nnz_stencil27(nx, ny, nz)


def test_configured_sizes():
    # the sizes quoted for the workloads: 32^3 and 256^3 Poisson, 192^3 27-point
    assert inputs.nnz_stencil7(32, 32, 32) == 223232
    assert inputs.nnz_stencil7(256, 256, 256) == 117047296
    assert inputs.nnz_stencil7(192, 192, 192) == 49324032
    assert inputs.nnz_stencil27(192, 192, 192) == 189119224


@pytest.mark.parametrize("g", [(3, 4, 5), (8, 8, 8)])
def test_rows_sorted_symmetric_rowsums(g):
    nx, ny, nz = g
    rp, col, val = inputs.poisson7_csr(nx, ny, nz)
    for i in range(rp.size - 1):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert i in c
    A = _to_scipy((rp, col, val))
    assert abs(A - A.T).max() == 0
    rs = np.asarray(A.sum(axis=1)).ravel()
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    interior = ((i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    assert np.all(rs[interior] == 0)
    assert np.all(rs[~interior] > 0)


def test_colourings_are_independent_sets():
    for (nx, ny, nz) in [(4, 3, 5), (6, 6, 6)]:
        A7 = _to_scipy(inputs.poisson7_csr(nx, ny, nz)).tocoo()
        c2 = inputs.redblack_colors(nx, ny, nz)
        off = A7.row != A7.col
        assert np.all(c2[A7.row[off]] != c2[A7.col[off]])
        A27 = _to_scipy(inputs.stencil27_csr(nx, ny, nz)).tocoo()
        c8 = inputs.octant_colors(nx, ny, nz)
        off = A27.row != A27.col
        assert np.all(c8[A27.row[off]] != c8[A27.col[off]])
        # red-black is not an independent colouring of the 27-point stencil
        assert np.any(c2[A27.row[off]] == c2[A27.col[off]])


def test_seeded_vectors_reproducible():
    a = inputs.uniform_vector(1000, 1)
    b = inputs.uniform_vector(1000, 1)
    assert np.array_equal(a, b)
    assert a.min() >= -1 and a.max() < 1
    assert not np.array_equal(a, inputs.uniform_vector(1000, 2))


@pytest.mark.parametrize("gen", ["convdiff7", "stencil27"])
def test_reflected_stencil_is_the_transpose(gen):
    # A^T of a constant stencil truncated at the grid boundary is the stencil
    # with its offsets reflected: the adjoint solves rely on it
    g = (5, 4, 3)
    c = inputs.convdiff7() if gen == "convdiff7" else inputs.STENCIL27
    n = int(np.prod(g))

    def dense(csr):
        rp, col, val = csr
        return sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()

    A = dense(inputs.stencil_csr(*g, c))
    At = dense(inputs.stencil_csr(*g, tuple(reversed(c))))
    assert np.array_equal(A.T, At)
