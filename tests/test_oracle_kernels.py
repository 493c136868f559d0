"""Pins of the oracle's dot products and SpMV against exact rational
arithmetic and dense products."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2305_05988_amd import inputs


def _exact_dot(x, y):
    s = sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))
    return float(s)  # Fraction -> float rounds to nearest, ties to even


@pytest.mark.parametrize("seed", range(6))
def test_dot_is_correctly_rounded_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    x = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)
    y = rng.standard_normal(n)
    assert oracle.dot(x, y) == _exact_dot(x, y)


@pytest.mark.parametrize("seed", range(4))
def test_dot_correctly_rounded_under_cancellation(seed):
    rng = np.random.default_rng(100 + seed)
    n = 200
    x = rng.standard_normal(n) * 2.0 ** rng.integers(-60, 60, n)
    y = rng.standard_normal(n)
    # append the negated terms except a small remainder: massive cancellation
    x2 = np.concatenate([x, -x, rng.standard_normal(5) * 1e-30])
    y2 = np.concatenate([y, y * (1 + 2.0 ** -40), rng.standard_normal(5)])
    assert oracle.dot(x2, y2) == _exact_dot(x2, y2)


def test_dot_half_way_cases():
    # exact value 1 + 2^-53 + 2^-106 lies just above the midpoint between 1
    # and 1 + 2^-52, so it must round up (plain summation returns 1.0)
    x = np.array([1.0, 2.0 ** -53, 2.0 ** -106])
    y = np.ones(3)
    assert oracle.dot(x, y) == 1.0 + 2.0 ** -52
    # exactly half-way: ties to even -> 1.0
    x = np.array([1.0, 2.0 ** -53])
    assert oracle.dot(x, np.ones(2)) == 1.0
    x = np.array([1.0 + 2.0 ** -52, 2.0 ** -53])
    assert oracle.dot(x, np.ones(2)) == 1.0 + 2.0 ** -51


def test_dot_products_split_exactly():
    # x*y with an error term below the product's ulp
    a = 1.0 + 2.0 ** -30
    x = np.array([a, -1.0])
    y = np.array([a, 1.0 + 2.0 ** -29])
    # a*a - (1 + 2^-29) = 2^-60 exactly
    assert oracle.dot(x, y) == 2.0 ** -60


def test_dot_special_values():
    assert oracle.dot(np.zeros(0), np.zeros(0)) == 0.0
    assert np.isnan(oracle.dot(np.array([np.nan, 1.0]), np.ones(2)))
    assert oracle.dot(np.array([np.inf, 1.0]), np.ones(2)) == np.inf
    assert np.isnan(oracle.dot(np.array([np.inf, -np.inf]), np.ones(2)))


@pytest.mark.parametrize("seed", range(4))
def test_dot_f32_is_correctly_rounded(seed):
    rng = np.random.default_rng(200 + seed)
    n = 300
    x = (rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    assert oracle.dot_f32(x, y) == _exact_dot(x.astype(np.float64), y.astype(np.float64))


def _scipy(A):
    rp, col, val = A
    n = rp.size - 1
    return sp.csr_matrix((val, col.astype(np.int64), rp), shape=(n, n))


@pytest.mark.parametrize("gen,g", [(inputs.poisson7_csr, (5, 4, 3)),
                                   (inputs.stencil27_csr, (4, 5, 6)),
                                   (inputs.convdiff7_csr, (6, 3, 5))])
def test_spmv_exact_on_integers(gen, g):
    A = gen(*g)
    n = A[0].size - 1
    x = inputs.integer_vector(n, 7, -1000, 1000)
    y = oracle.spmv(A, x)
    assert np.array_equal(y, _scipy(A) @ x)


@pytest.mark.parametrize("gen,g", [(inputs.poisson7_csr, (9, 8, 7)),
                                   (inputs.stencil27_csr, (6, 6, 6))])
def test_spmv_random_close_to_dense(gen, g):
    A = gen(*g)
    n = A[0].size - 1
    x = inputs.uniform_vector(n, 3)
    y = oracle.spmv(A, x)
    ref = oracle.csr_to_dense(A) @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spmv_is_an_fma_chain_in_stored_order():
    # row [a, -b] . [a, 1] with a*a = 1 + 2^-29 + 2^-60 and b = 1 + 2^-29:
    # in stored order the chain is fma(-b, 1, round(a*a)) = 0; with the
    # entries stored the other way round it is fma(a, a, -b) = 2^-60 exactly.
    a, b = 1.0 + 2.0 ** -30, 1.0 + 2.0 ** -29
    x = np.array([a, 1.0])
    fwd = (np.array([0, 2, 3], np.int64), np.array([0, 1, 1], np.int32), np.array([a, -b, 1.0]))
    rev = (np.array([0, 2, 3], np.int64), np.array([1, 0, 1], np.int32), np.array([-b, a, 1.0]))
    assert oracle.spmv(fwd, x)[0] == 0.0
    assert oracle.spmv(rev, x)[0] == 2.0 ** -60


def test_spmv_f32_exact_on_integers():
    A = inputs.stencil27_csr(5, 4, 3)
    n = A[0].size - 1
    x = inputs.integer_vector(n, 9, -100, 100).astype(np.float32)
    y = oracle.spmv_f32(A, A[2].astype(np.float32), x)
    assert np.array_equal(y.astype(np.float64), _scipy(A) @ x.astype(np.float64))


def test_spmv_f32_close_on_random():
    A = inputs.poisson7_csr(8, 8, 8)
    n = A[0].size - 1
    x = inputs.uniform_vector(n, 4).astype(np.float32)
    y = oracle.spmv_f32(A, A[2].astype(np.float32), x)
    ref = _scipy(A) @ x.astype(np.float64)
    assert np.max(np.abs(y - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_spmv_f32_is_an_fp32_fma_chain_in_stored_order():
    # Three rows whose FP32 chain differs from every plausible alternative:
    #  row 0: [1, 1, 1] . [1, 2^-24, 2^-24].  In FP32 each 2^-24 is half an
    #         ulp of 1 and rounds away (ties to even): exactly 1.  Summed in
    #         double and rounded once it is 1 + 2^-23.
    #  row 1: [a, -c] . [a, 1] with a = 1 + 2^-12, c = 1 + 2^-11: a*a is
    #         1 + 2^-11 + 2^-24, whose FP32 rounding is c, so the fma chain
    #         gives fma(-c, 1, round(a*a)) = 0; a product rounded before the
    #         add, or the entries taken in reverse order
    #         (fma(a, a, -c) = 2^-24), do not.
    #  row 2: [-c, a] . [1, a]: the same entries stored the other way round,
    #         whose chain is fma(a, a, -c) = 2^-24 exactly.
    a = np.float32(1.0 + 2.0 ** -12)
    c = np.float32(1.0 + 2.0 ** -11)
    tiny = np.float32(2.0 ** -24)
    # columns: 0 -> 1, 1 -> 2^-24, 2 -> 2^-24, 3 -> a, 4 -> 1
    x = np.array([1.0, tiny, tiny, a, 1.0], np.float32)
    rp = np.array([0, 3, 5, 7, 8, 9], np.int64)
    col = np.array([0, 1, 2, 3, 4, 4, 3, 3, 4], np.int32)
    val32 = np.array([1, 1, 1, a, -c, -c, a, 1, 1], np.float32)
    A = (rp, col, val32.astype(np.float64))
    y = oracle.spmv_f32(A, val32, x)
    assert y.dtype == np.float32
    assert y[0] == np.float32(1.0)
    assert y[1] == np.float32(0.0)
    assert y[2] == tiny
    assert y[3] == a and y[4] == np.float32(1.0)
