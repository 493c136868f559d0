"""Pins of the oracle's iterative solvers against closed forms, finite
termination, dense LU and crafted breakdown cases."""
import math

import numpy as np
import pytest

import oracle
from paper_2305_05988_amd import inputs


def _system(A, seed=1):
    n = A[0].size - 1
    xs = inputs.uniform_vector(n, seed)
    return xs, oracle.spmv(A, xs)


def _int_system(A, seed=5):
    # integer x* keeps b = A x* exact, so x* is the exact solution
    n = A[0].size - 1
    xs = inputs.integer_vector(n, seed)
    return xs, oracle.spmv(A, xs)


# ----------------------------------------------------------------- Jacobi
@pytest.mark.parametrize("k", [1, 7, 60])
def test_jacobi_damps_slowest_mode_by_cos_pi_h(k):
    N = 10
    A = inputs.poisson7_csr(N)
    xs, b = _int_system(A)
    v = inputs.sine_mode(N, N, N)
    x, r = oracle.jacobi(A, b, x0=xs + v, rtol=0.0, max_iter=k)
    assert r.status == oracle.NOT_CONVERGED and r.iters == k
    mu = math.cos(math.pi / (N + 1))
    err = (x - xs) - mu ** k * v
    assert np.max(np.abs(err)) <= 1e-12 * np.max(np.abs(v))


def test_jacobi_spectral_radius_value_32():
    assert abs(math.cos(math.pi / 33) - 0.9954719) < 1e-7


@pytest.mark.parametrize("k", [1, 5, 20])
def test_jacobi_upwind_mode(k):
    # Jacobi matrix of the upwind operator: (11 E^- + E^+)/36 per axis; its
    # slowest mode grows like sqrt(11)^i and has eigenvalue sqrt(11)/6 cos(pi h)
    N = 6
    A = inputs.convdiff7_csr(N)
    xs, b = _int_system(A)
    g = math.sqrt(11.0)
    v = inputs.sine_mode(N, N, N, growth=(g, g, g))
    v = v / np.max(np.abs(v))
    x, r = oracle.jacobi(A, b, x0=xs + v, rtol=0.0, max_iter=k)
    mu = g / 6.0 * math.cos(math.pi / (N + 1))
    err = (x - xs) - mu ** k * v
    assert np.max(np.abs(err)) <= 1e-12


def test_jacobi_converges_and_stops_at_first_passing_iterate():
    A = inputs.poisson7_csr(6)
    xs, b = _system(A)
    x, r = oracle.jacobi(A, b, rtol=1e-8, max_iter=5000)
    assert r.status == oracle.OK
    assert r.rel_res <= 1e-8
    # one sweep fewer must not pass
    x1, r1 = oracle.jacobi(A, b, rtol=1e-8, max_iter=r.iters - 1)
    assert r1.status == oracle.NOT_CONVERGED and r1.rel_res > 1e-8
    assert np.max(np.abs(x - xs)) <= 1e-6


# ----------------------------------------------------------- Gauss-Seidel
@pytest.mark.parametrize("k", [1, 2, 9])
def test_redblack_sgs_mode_closed_form(k):
    # consistently ordered: red update from black multiplies by mu, so the
    # error (v_R, mu v_B) becomes (mu^(2k+2) v_R, mu^(2k+1) v_B) after k
    # symmetric R,B,B,R iterations
    N = 8
    A = inputs.poisson7_csr(N)
    xs, b = _int_system(A)
    v = inputs.sine_mode(N, N, N)
    col = inputs.redblack_colors(N, N, N)
    mu = math.cos(math.pi / (N + 1))
    red = col == 0
    e0 = np.where(red, v, mu * v)
    x, r = oracle.sgs(A, col, 2, b, x0=xs + e0, rtol=0.0, max_iter=k)
    assert r.iters == k
    pred = np.where(red, mu ** (2 * k + 2) * v, mu ** (2 * k + 1) * v)
    assert np.max(np.abs((x - xs) - pred)) <= 1e-12


def test_sgs_single_colour_is_lexicographic_symmetric_gs():
    # one colour is not an independent set for a coupled matrix -> rejected
    A = inputs.poisson7_csr(3)
    xs, b = _system(A)
    x, r = oracle.sgs(A, np.zeros(27, np.uint8), 1, b, rtol=1e-8)
    assert r.status == oracle.E_INVALID


def test_sgs_27pt_octant_colours_match_lu():
    A = inputs.stencil27_csr(5, 4, 3)
    xs, b = _system(A)
    c = inputs.octant_colors(5, 4, 3)
    x, r = oracle.sgs(A, c, 8, b, rtol=1e-12, max_iter=5000)
    assert r.status == oracle.OK
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    assert np.max(np.abs(x - ref)) <= 1e-9


def test_sgs_rejects_dependent_colouring():
    A = inputs.stencil27_csr(4)
    xs, b = _system(A)
    x, r = oracle.sgs(A, inputs.redblack_colors(4, 4, 4), 2, b)
    assert r.status == oracle.E_INVALID


# ------------------------------------------------------------------- CG
@pytest.mark.parametrize("N,distinct", [(2, 4), (3, 7)])
def test_cg_finite_termination(N, distinct):
    A = inputs.poisson7_csr(N)
    xs, b = _system(A, seed=3)
    x, r = oracle.cg(A, b, rtol=1e-13, max_iter=100)
    assert r.status == oracle.OK and r.iters <= distinct
    assert np.max(np.abs(x - xs)) <= 1e-13


def test_cg_eigenvalue_count_2cube():
    d = np.linalg.eigvalsh(oracle.csr_to_dense(inputs.poisson7_csr(2)))
    assert sorted(set(np.round(d, 10))) == [3.0, 5.0, 7.0, 9.0]


@pytest.mark.parametrize("gen,g", [(inputs.poisson7_csr, (6, 5, 4)),
                                   (inputs.stencil27_csr, (5, 5, 5))])
def test_cg_matches_dense_lu(gen, g):
    A = gen(*g)
    xs, b = _system(A, seed=11)
    x, r = oracle.cg(A, b, rtol=1e-12, max_iter=1000)
    assert r.status == oracle.OK
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_lu_matches_library_solve():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((40, 40))
    b = rng.standard_normal(40)
    assert np.allclose(oracle.lu_solve(a, b), np.linalg.solve(a, b), rtol=1e-11, atol=1e-12)
    with pytest.raises(ValueError):
        oracle.lu_solve(np.zeros((3, 3)), np.ones(3))


def test_cg_manufactured_solution_and_residual_invariant():
    N = 16
    A = inputs.poisson7_csr(N)
    xs, b = _system(A, seed=1)
    x, r = oracle.cg(A, b, rtol=1e-8, max_iter=2000)
    assert r.status == oracle.OK and r.rel_res <= 1e-8
    kappa = 1.0 / math.tan(math.pi / (2 * (N + 1))) ** 2
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-8
    # recursive and true residual agree far below the tolerance
    assert abs(r.true_rel_res - r.rel_res) <= 1e-12
    # and the iteration count respects the Chebyshev bound
    bound = 0.5 * math.sqrt(kappa) * math.log(2.0 / 1e-8) + 1
    assert r.iters <= bound


def test_cg_fixed_k_iterate_is_deterministic():
    A = inputs.poisson7_csr(7)
    xs, b = _system(A)
    x1, r1 = oracle.cg(A, b, rtol=0.0, max_iter=9)
    x2, r2 = oracle.cg(A, b, rtol=0.0, max_iter=9)
    assert r1.iters == 9 and r1.status == oracle.NOT_CONVERGED
    assert np.array_equal(x1, x2)


# ------------------------------------------------------------------ CG-NB
@pytest.mark.parametrize("N,distinct", [(2, 4), (3, 7)])
def test_cgnb_finite_termination(N, distinct):
    # arithmetically CG (Algorithm 1 only reorders it), so its residual
    # vanishes within the number of distinct eigenvalues too
    A = inputs.poisson7_csr(N)
    xs, b = _system(A, seed=3)
    x, r = oracle.cgnb(A, b, rtol=1e-13, max_iter=100)
    assert r.status == oracle.OK and r.iters <= distinct
    assert r.rel_res <= 1e-13


def test_cgnb_exact_convergence_uses_the_limit_update():
    # one unknown: r vanishes after one step, alpha_n = 0, gamma = 1/0
    A = (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([4.0]))
    x, r = oracle.cgnb(A, np.array([3.0]), rtol=1e-14)
    assert r.status == oracle.OK and r.iters == 1 and x[0] == 0.75


def test_cgnb_x_update_cancels_when_beta_collapses():
    # Algorithm 1 forms x_j from gamma (p_j - r_j) with gamma ~ 1/alpha_n,j;
    # when the residual collapses in one step (finite termination), beta ~ 0,
    # p_j - r_j cancels and the rounding error is amplified: the iterate loses
    # accuracy although the recursive residual vanished.  Classical CG does not.
    A = inputs.poisson7_csr(2)
    xs, b = _system(A, seed=3)
    x, r = oracle.cgnb(A, b, rtol=1e-13, max_iter=100)
    xc, rc = oracle.cg(A, b, rtol=1e-13, max_iter=100)
    assert r.true_rel_res > 1e-6 and rc.true_rel_res < 1e-14


@pytest.mark.parametrize("gen,g", [(inputs.poisson7_csr, (6, 5, 4)),
                                   (inputs.stencil27_csr, (5, 5, 5))])
def test_cgnb_matches_dense_lu(gen, g):
    A = gen(*g)
    xs, b = _system(A, seed=11)
    x, r = oracle.cgnb(A, b, rtol=1e-12, max_iter=1000)
    assert r.status == oracle.OK
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1, 3, 10])
def test_cgnb_iterates_track_classical_cg(k):
    # same Krylov iterates in exact arithmetic; rounding differs slightly
    A = inputs.poisson7_csr(9, 8, 7)
    xs, b = _system(A, seed=5)
    x1, r1 = oracle.cg(A, b, rtol=0.0, max_iter=k)
    x2, r2 = oracle.cgnb(A, b, rtol=0.0, max_iter=k)
    assert r1.iters == r2.iters == k
    assert np.max(np.abs(x1 - x2)) <= 1e-12 * np.max(np.abs(x1))


def test_cgnb_converges_like_cg_with_small_residual_gap():
    N = 16
    A = inputs.poisson7_csr(N)
    xs, b = _system(A, seed=1)
    xc, rc = oracle.cg(A, b, rtol=1e-8, max_iter=2000)
    xn, rn = oracle.cgnb(A, b, rtol=1e-8, max_iter=2000)
    assert rn.status == oracle.OK and abs(rn.iters - rc.iters) <= 1
    assert rn.true_rel_res <= 1.1e-8
    assert np.linalg.norm(xn - xc) / np.linalg.norm(xc) <= 1e-8


# ------------------------------------------------------------- BiCGStab
@pytest.mark.parametrize("g", [(5, 5, 5), (8, 3, 6)])
def test_bicgstab_matches_dense_lu_upwind(g):
    A = inputs.convdiff7_csr(*g)
    xs, b = _system(A, seed=2)
    x, r = oracle.bicgstab(A, b, rtol=1e-12, max_iter=500)
    assert r.status == oracle.OK
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert r.true_rel_res <= 1e-11


@pytest.mark.parametrize("N,distinct", [(2, 4), (3, 7)])
def test_bicgstab_finite_termination_upwind(N, distinct):
    # BiCGStab's residual is psi_k(A) phi_k(A) r0 with phi_k the BiCG
    # polynomial, so it terminates within the degree of A's minimal
    # polynomial: the number of distinct eigenvalues (A is diagonalisable,
    # a Kronecker sum of similar-to-symmetric tridiagonals)
    A = inputs.convdiff7_csr(N)
    ev = np.linalg.eigvals(oracle.csr_to_dense(A))
    assert np.max(np.abs(ev.imag)) < 1e-9
    assert len(set(np.round(ev.real, 8))) == distinct
    xs, b = _system(A, seed=3)
    x, r = oracle.bicgstab(A, b, rtol=1e-13, max_iter=100)
    assert r.status == oracle.OK and r.iters <= distinct
    assert np.max(np.abs(x - xs)) <= 1e-12


def test_bicgstab_matches_cg_on_spd():
    A = inputs.poisson7_csr(6)
    xs, b = _system(A, seed=4)
    xc, rc = oracle.cg(A, b, rtol=1e-12, max_iter=500)
    xb, rb = oracle.bicgstab(A, b, rtol=1e-12, max_iter=500)
    assert rc.status == rb.status == oracle.OK
    assert np.max(np.abs(xc - xb)) <= 1e-10


def test_bicgstab_one_unknown_finishes_in_one_half_step():
    A = (np.array([0, 1], np.int64), np.array([0], np.int32), np.array([4.0]))
    x, r = oracle.bicgstab(A, np.array([3.0]), rtol=1e-14)
    # s = r - (1/a) A r = 0, so t = 0: the half step x = r0/a is exact
    assert r.status == oracle.OK and r.iters == 1 and x[0] == 0.75


def test_bicgstab_restart_paths():
    A = inputs.convdiff7_csr(6)
    xs, b = _system(A, seed=8)
    ref = oracle.lu_solve(oracle.csr_to_dense(A), b)
    # a large cosine threshold forces restarts every few iterations
    x, r = oracle.bicgstab(A, b, rtol=1e-10, max_iter=2000, restart_tol=0.9)
    assert r.status == oracle.OK and r.restarts > 0
    assert np.max(np.abs(x - ref)) <= 1e-8 * np.max(np.abs(ref))
    # the paper's absolute form with a large threshold as well
    x, r = oracle.bicgstab(A, b, rtol=1e-10, max_iter=2000, restart_tol=30.0,
                           restart_mode=oracle.RESTART_PAPER)
    assert r.status == oracle.OK and r.restarts > 0
    # default threshold: no restart needed on this well-conditioned system
    x, r = oracle.bicgstab(A, b, rtol=1e-10, max_iter=2000)
    assert r.restarts == 0


# ----------------------------------------------------- mixed precision IR
@pytest.mark.parametrize("lowp", [np.float32, np.float16])
def test_ir_cg_reaches_fp64_accuracy(lowp):
    N = 10
    A = inputs.stencil27_csr(N)
    xs, b = _system(A, seed=1)
    lo = A[2].astype(lowp)
    assert np.array_equal(lo.astype(np.float64), A[2])  # 26 and -1 are exact
    x, r = oracle.ir_cg(A, lo, b, rtol=1e-10, max_iter=5000, inner_rtol=1e-4)
    assert r.status == oracle.OK and r.rel_res <= 1e-10
    assert 2 <= r.iters <= 4
    xc, rc = oracle.cg(A, b, rtol=1e-12, max_iter=5000)
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 1e-9


def test_ir_cg_outer_contraction():
    A = inputs.poisson7_csr(12)
    xs, b = _system(A, seed=2)
    lo = A[2].astype(np.float32)
    res = []
    for k in range(1, 4):
        x, r = oracle.ir_cg(A, lo, b, rtol=0.0, max_iter=10000, inner_rtol=1e-3, max_outer=k)
        res.append(r.rel_res)
    # each refinement step contracts the residual by about inner_rtol
    assert res[1] <= 5e-3 * res[0] and res[2] <= 5e-3 * res[1]


# --------------------------------------------------------- status codes
@pytest.mark.parametrize("solver", ["jacobi", "cg", "bicgstab"])
def test_zero_rhs_returns_zero(solver):
    A = inputs.poisson7_csr(3)
    x, r = getattr(oracle, solver)(A, np.zeros(27), x0=np.ones(27))
    assert r.status == oracle.OK and r.iters == 0 and not x.any()


@pytest.mark.parametrize("solver", ["jacobi", "cg", "bicgstab"])
def test_nan_rhs_is_invalid(solver):
    A = inputs.poisson7_csr(3)
    b = np.ones(27)
    b[5] = np.nan
    x, r = getattr(oracle, solver)(A, b)
    assert r.status == oracle.E_INVALID


@pytest.mark.parametrize("solver", ["jacobi", "cg", "bicgstab"])
def test_max_iter_not_converged(solver):
    A = inputs.poisson7_csr(8)
    xs, b = _system(A)
    x, r = getattr(oracle, solver)(A, b, rtol=1e-12, max_iter=3)
    assert r.status == oracle.NOT_CONVERGED and r.iters == 3


def test_cg_breakdown_on_indefinite():
    # diag(1,-1), b = (1,1): p = r = b, A p . p = 0
    A = (np.array([0, 1, 2], np.int64), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    x, r = oracle.cg(A, np.array([1.0, 1.0]))
    assert r.status == oracle.BREAKDOWN and r.iters == 0 and not x.any()


def test_bicgstab_breakdown_alpha_d_zero():
    # A = [[0,1],[1,0]], b = (1,0): v = A r = (0,1) is orthogonal to r' = (1,0)
    A = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    x, r = oracle.bicgstab(A, np.array([1.0, 0.0]))
    assert r.status == oracle.BREAKDOWN and r.iters == 0


def test_jacobi_requires_diagonal():
    A = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    x, r = oracle.jacobi(A, np.array([1.0, 0.0]))
    assert r.status == oracle.E_INVALID
