"""Pins of the oracle's compensated algorithms Sum2 and Dot2 (Ogita, Rump
and Oishi, SIAM J. Sci. Comput. 2005), the paper's named future work
(section 7), against exact arithmetic.

* empty and single-term inputs: (0, 0), (x, 0), the exact TwoProduct pair;
* integer data whose partial sums stay representable: exact;
* the published error bounds, measured exactly with the long accumulator:
  Sum2  |res - sum x_i|  <= u |sum x_i|  + gamma_{n-1}^2 sum |x_i|
  Dot2  |res - x.y|      <= u |x.y|      + gamma_n^2     sum |x_i y_i|
  (res = p (+) s, u = 2^-24, gamma_k = k u / (1 - k u)) on random and on
  ill-conditioned data up to condition number 2^55;
* where the naive binary32 sum is wrong in every digit, Dot2 is accurate;
* the batched forms are the per-vector ones.
"""
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import frac

U = Fraction(1, 1 << 24)


def gamma(k):
    return k * U / (1 - k * U)


def _res(p, s):
    return frac(np.float32(np.float32(p) + np.float32(s)))


def test_empty_and_single_terms():
    e = np.zeros(0, np.float32)
    assert oracle.sum2(e) == (0.0, 0.0) and oracle.dot2(e, e) == (0.0, 0.0)
    xs = fi.random_f32(300, 11, -40, 40).numpy()
    ys = fi.random_f32(300, 12, -40, 40).numpy()
    for x, y in zip(xs, ys):
        assert oracle.sum2(np.float32([x])) == (x, 0.0)
        p, s = oracle.dot2(np.float32([x]), np.float32([y]))
        assert frac(p) + frac(s) == frac(x) * frac(y)
        assert p == np.float32(x * y)


def test_integer_data_is_exact():
    rng = np.random.default_rng(3)
    for n in (2, 17, 1000):
        x = rng.integers(-2000, 2000, n).astype(np.float32)
        y = rng.integers(-2000, 2000, n).astype(np.float32)
        p, s = oracle.sum2(x)
        assert _res(p, s) == int(x.astype(np.int64).sum())
        p, s = oracle.dot2(x, y)
        assert _res(p, s) == int((x.astype(np.int64) * y.astype(np.int64)).sum())


@pytest.mark.parametrize("n", [2, 10, 100, 3000])
def test_sum2_error_bound_random(n):
    for seed in range(5):
        x = fi.random_f32(n, 100 + seed, -30, 30).numpy()
        p, s = oracle.sum2(x)
        exact = oracle.exact_dot(x, np.ones_like(x))
        absum = oracle.exact_dot(np.abs(x), np.ones_like(x))
        assert abs(_res(p, s) - exact) <= U * abs(exact) + gamma(n - 1) ** 2 * absum


@pytest.mark.parametrize("log2_cond", [10, 25, 40, 55])
def test_dot2_error_bound_ill_conditioned(log2_cond):
    n = 1000
    x, y = fi.ill_conditioned_dot(n, 200 + log2_cond, log2_cond)
    x, y = x.numpy(), y.numpy()
    p, s = oracle.dot2(x, y)
    exact = oracle.exact_dot(x, y)
    absum = oracle.exact_dot(np.abs(x), np.abs(y))
    assert abs(_res(p, s) - exact) <= U * abs(exact) + gamma(n) ** 2 * absum
    # Sum2 on the products' exact halves behaves alike: the sum of the
    # TwoProduct pairs equals x.y exactly
    h, r = oracle.mul12(x, y)
    both = np.concatenate([h, r])
    p2, s2 = oracle.sum2(both)
    assert abs(_res(p2, s2) - exact) <= U * abs(exact) + gamma(2 * n - 1) ** 2 * 2 * absum


def test_dot2_where_the_naive_sum_fails():
    n = 2000
    x, y = fi.ill_conditioned_dot(n, 77, 24)
    x, y = x.numpy(), y.numpy()
    exact = oracle.exact_dot(x, y)
    naive = np.float32(0.0)
    for a, b in zip(x, y):
        naive = np.float32(naive + np.float32(a * b))
    p, s = oracle.dot2(x, y)
    assert abs(frac(naive) - exact) > abs(exact) / 2            # no correct digit
    assert abs(_res(p, s) - exact) < abs(exact) * Fraction(1, 1 << 10)


@pytest.mark.parametrize("n", [2, 5, 40])
def test_brute_force_small(n):
    for seed in range(20):
        x = fi.random_f32(n, 300 + seed, -12, 12).numpy()
        y = fi.random_f32(n, 400 + seed, -12, 12).numpy()
        x[n // 2:] = -x[: n - n // 2] * np.float32(1 + 2.0 ** -20)   # cancellation
        exact = sum(frac(a) * frac(b) for a, b in zip(x, y))
        absum = sum(abs(frac(a) * frac(b)) for a, b in zip(x, y))
        p, s = oracle.dot2(x, y)
        assert abs(_res(p, s) - exact) <= U * abs(exact) + gamma(n) ** 2 * absum
        exact_s = sum(frac(a) for a in x)
        p, s = oracle.sum2(x)
        assert abs(_res(p, s) - exact_s) <= U * abs(exact_s) + gamma(n - 1) ** 2 * sum(abs(frac(a)) for a in x)


def test_batched_forms_are_per_vector():
    x, y, offs = fi.batched_dot(5, nvec=16, log2_max=10)
    x, y, offs = x.numpy(), y.numpy(), offs.numpy()
    p, s = oracle.dot2_batched(x, y, offs)
    q, t = oracle.sum2_batched(x, offs)
    for v in range(16):
        a, b = offs[v], offs[v + 1]
        assert (p[v], s[v]) == oracle.dot2(x[a:b], y[a:b])
        assert (q[v], t[v]) == oracle.sum2(x[a:b])
