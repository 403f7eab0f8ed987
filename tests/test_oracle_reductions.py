"""Pins of the oracle's exact references and float-float accumulations.

The long accumulator is checked against Python's ``math.fsum`` (Shewchuk's
correctly rounded summation, an independent implementation) and against
brute-force Fraction sums; the float-float accumulations are checked against
closed forms (one term, integer data), the identity matrix and the error
bound that follows from the Add22 theorem.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac


def _np(t):
    return t.cpu().numpy()


# ------------------------------------------------------- long accumulator

@pytest.mark.parametrize("emin,emax", [(-20, 20), (-120, 120)])
def test_exact_dot_rounds_to_fsum(emin, emax):
    for seed in range(4):
        n = 5000 + 777 * seed
        x = _np(fi.random_f32(n, 1000 + seed, emin, emax))
        y = _np(fi.random_f32(n, 2000 + seed, emin, emax))
        exact = oracle.exact_dot(x, y)
        prods = (x.astype(np.float64) * y.astype(np.float64)).tolist()   # exact products
        assert float(exact) == math.fsum(prods)


def test_exact_dot_brute_force_and_extremes():
    tiny = np.float32(2.0 ** -149)
    big = np.float32(np.finfo(np.float32).max)
    x = np.array([tiny, big, -big, 1.0, 3.0, -0.1], np.float32)
    y = np.array([tiny, big, big, 2.0 ** -100, -7.0, 0.3], np.float32)
    exact = oracle.exact_dot(x, y)
    assert exact == sum(frac(a) * frac(b) for a, b in zip(x, y))
    for seed in range(8):
        x = _np(fi.random_f32(64, 3000 + seed, -126, 120))
        y = _np(fi.random_f32(64, 4000 + seed, -126, 120))
        assert oracle.exact_dot(x, y) == sum(frac(a) * frac(b) for a, b in zip(x, y))
    # subnormal operands (bit patterns below the smallest normal)
    sub = np.arange(1, 65, dtype=np.uint32).view(np.float32) * np.float32(-1) ** np.arange(64)
    z = _np(fi.random_f32(64, 3999, -126, 0))
    assert oracle.exact_dot(sub, z) == sum(frac(a) * frac(b) for a, b in zip(sub, z))


def test_exact_dot_ff_brute_force():
    for seed in range(6):
        a = _np(fi.random_ff(200, 5000 + seed, -60, 60))
        b = _np(fi.random_ff(200, 6000 + seed, -60, 60))
        want = sum(ff_value(a[0, i], a[1, i]) * ff_value(b[0, i], b[1, i]) for i in range(200))
        assert oracle.exact_dot_ff(a[0], a[1], b[0], b[1]) == want


def test_exact_dot_cancels_exactly():
    x = np.array([2.0 ** 60, 1.0, -(2.0 ** 60)], np.float32)
    y = np.array([2.0 ** 50, 2.0 ** -100, 2.0 ** 50], np.float32)
    assert oracle.exact_dot(x, y) == Fraction(1, 1 << 100)


def test_exact_dot_batched_is_per_vector():
    x, y, offs = fi.batched_dot(7, nvec=50, max_total=20000)
    x, y, offs = _np(x), _np(y), _np(offs)
    got = oracle.exact_dot_batched(x, y, offs)
    for v in range(50):
        s, e = offs[v], offs[v + 1]
        assert got[v] == sum(frac(a) * frac(b) for a, b in zip(x[s:e], y[s:e]))


# ------------------------------------------------- float-float accumulation

def test_dot_seq_single_term_is_the_exact_product_pair():
    x = _np(fi.random_f32(500, 7001, -30, 30))
    y = _np(fi.random_f32(500, 7002, -30, 30))
    for a, b in zip(x, y):
        h, l = oracle.dot_seq([a], [b])
        assert np.float32(h) == np.float32(np.float64(a) * np.float64(b))
        assert frac(h) + frac(l) == frac(a) * frac(b)


def test_dot_seq_integer_data_is_exact():
    # integers with an exactly representable float-float sum: no rounding at all
    rng = np.random.default_rng(7003)
    x = rng.integers(-2 ** 11, 2 ** 11, 10000).astype(np.float32)
    y = rng.integers(-2 ** 11, 2 ** 11, 10000).astype(np.float32)
    h, l = oracle.dot_seq(x, y)
    assert frac(h) + frac(l) == sum(int(a) * int(b) for a, b in zip(x, y))


def _dot_bound(n, abs_sum):
    # Each Add22 step errs by at most 2^-44 (|acc| + |p_i|) (Add22 theorem,
    # with normalised low words), and |acc| never exceeds the sum of |terms|.
    return n * Fraction(1, 1 << 44) * abs_sum


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 20000])
def test_dot_seq_error_bound(n):
    x = _np(fi.gaussian_f32((n,), 7100 + n))
    y = _np(fi.gaussian_f32((n,), 7200 + n))
    h, l = oracle.dot_seq(x, y)
    exact = oracle.exact_dot(x, y)
    abs_sum = oracle.exact_dot(np.abs(x), np.abs(y))
    err = abs(frac(h) + frac(l) - exact)
    assert err <= _dot_bound(n, abs_sum)
    # and, on this random data, the normwise error is far below 2^-44
    assert err <= Fraction(1, 1 << 44) * abs_sum


def test_dot_seq_batched_is_per_vector():
    x, y, offs = fi.batched_dot(9, nvec=40, max_total=30000)
    x, y, offs = _np(x), _np(y), _np(offs)
    hs, ls = oracle.dot_seq_batched(x, y, offs)
    exact = oracle.exact_dot_batched(x, y, offs)
    for v in range(40):
        s, e = offs[v], offs[v + 1]
        h, l = oracle.dot_seq(x[s:e], y[s:e])
        assert (np.float32(h), np.float32(l)) == (hs[v], ls[v])
        abs_sum = oracle.exact_dot(np.abs(x[s:e]), np.abs(y[s:e]))
        assert abs(frac(h) + frac(l) - exact[v]) <= _dot_bound(e - s, abs_sum)


def test_dot_ff_seq_error_bound():
    a = _np(fi.gaussian_ff((3000,), 7301))
    b = _np(fi.gaussian_ff((3000,), 7302))
    h, l = oracle.dot_ff_seq(a[0], a[1], b[0], b[1])
    exact = oracle.exact_dot_ff(a[0], a[1], b[0], b[1])
    err = abs(frac(h) + frac(l) - exact)
    abs_sum = oracle.exact_dot_ff(np.abs(a[0]), np.sign(a[0]) * a[1],
                                  np.abs(b[0]), np.sign(b[0]) * b[1])
    assert err <= Fraction(1, 1 << 44) * abs_sum


# ------------------------------------------------------------------ GEMM

def test_gemm_identity_returns_a():
    A = _np(fi.gaussian_ff((24, 40), 7401))
    I = np.eye(40, dtype=np.float32)
    Z = np.zeros_like(I)
    Ch, Cl = oracle.gemm_ff_seq(A[0], A[1], I, Z)
    assert np.array_equal(Ch, A[0]) and np.array_equal(Cl, A[1])


def test_gemm_integer_matrices_exact():
    rng = np.random.default_rng(7402)
    Ai = rng.integers(-100, 100, (16, 50))
    Bi = rng.integers(-100, 100, (50, 12))
    Z1, Z2 = np.zeros((16, 50), np.float32), np.zeros((50, 12), np.float32)
    Ch, Cl = oracle.gemm_ff_seq(Ai.astype(np.float32), Z1, Bi.astype(np.float32), Z2)
    assert np.array_equal(Ch.astype(np.int64) + Cl.astype(np.int64), Ai @ Bi)


def test_gemm_block_and_exact_entries():
    A = _np(fi.gaussian_ff((20, 64), 7403))
    B = _np(fi.gaussian_ff((64, 18), 7404))
    Ch, Cl = oracle.gemm_ff_seq(A[0], A[1], B[0], B[1])
    bh, bl = oracle.gemm_ff_seq(A[0], A[1], B[0], B[1], rows=(3, 9), cols=(5, 17))
    assert np.array_equal(bh, Ch[3:9, 5:17]) and np.array_equal(bl, Cl[3:9, 5:17])
    rows, cols = np.array([0, 7, 19, 4]), np.array([0, 17, 3, 11])
    exact = oracle.exact_gemm_entries(A[0], A[1], B[0], B[1], rows, cols)
    scale = oracle.exact_absgemm_entries(A[0], A[1], B[0], B[1], rows, cols)
    for t, (i, j) in enumerate(zip(rows, cols)):
        want = sum(ff_value(A[0, i, k], A[1, i, k]) * ff_value(B[0, k, j], B[1, k, j])
                   for k in range(64))
        want_abs = sum(abs(ff_value(A[0, i, k], A[1, i, k]) * ff_value(B[0, k, j], B[1, k, j]))
                       for k in range(64))
        assert exact[t] == want and scale[t] == want_abs
        err = abs(frac(Ch[i, j]) + frac(Cl[i, j]) - want)
        assert err <= 64 * Fraction(1, 1 << 44) * want_abs
