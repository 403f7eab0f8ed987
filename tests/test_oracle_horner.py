"""Pins of the oracle's polynomial evaluation: Horner's rule in binary32,
compensated Horner (CompHorner of Graillat, Langlois and Louvet, 2005/2009;
compensated algorithms are the paper's future work, section 7) and
float-float Horner (the paper's Mul22 and Add22, section 4.1, per step).

* degree 0 returns the constant; integer data whose every intermediate value
  is representable is exact for all three (closed form: integer evaluation);
* the closed form (x - 1)^n of the expanded binomial, whose magnitude
  polynomial is (1 + |x|)^n, and random polynomials evaluated exactly with
  Fraction, against the error bounds:
    Horner        |err| <= gamma_2n(u) p~(|x|)            (u = 2^-24)
    CompHorner    |err| <= u |p(x)| + gamma_2n(u)^2 p~(|x|)
    ff Horner     |err| <= gamma_2n(2^-44) p~(|x|)
  with gamma_k(v) = k v / (1 - k v) and p~(|x|) = sum |a_i| |x|^i.  The ff
  bound follows from the Mul22 theorem (relative 2^-44) and the Add22
  theorem: for normalised operands max(2^-24 |al + bl|, 2^-44 |a + b|) is at
  most 2^-44 (|a| + |b|), so each step perturbs both of its terms by at most
  2^-44 relative and the classical Horner analysis applies;
* near the root of (x - 1)^5, Horner in binary32 has no correct digit while
  CompHorner is accurate to about u + cond u^2;
* float-float coefficients and points: the low words count.
"""
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac, same_bits

U = Fraction(1, 1 << 24)
V = Fraction(1, 1 << 44)


def gamma(k, v):
    return k * v / (1 - k * v)


def _exact_poly(coeffs, x):
    """sum_i a_i x^i in exact rational arithmetic (coefficients and point as
    Fractions)."""
    total, power = Fraction(0), Fraction(1)
    for a in coeffs:
        total += a * power
        power *= x
    return total


def _abs_poly(coeffs, x):
    return _exact_poly([abs(a) for a in coeffs], abs(x))


def _zeros(n):
    return np.zeros(n, np.float32)


def test_degree_zero_returns_the_constant():
    x = fi.random_f32(1000, 1401, -20, 20).numpy()
    for c in (np.float32(3.25), np.float32(-1e-30)):
        a = np.array([c], np.float32)
        assert np.all(oracle.horner_f32(a, x) == c)
        assert np.all(oracle.horner_comp(a, x) == c)
        yh, yl = oracle.horner_ff(a, _zeros(1), x, _zeros(x.size))
        assert np.all(yh == c) and np.all(yl == 0)


def test_integer_polynomials_are_exact():
    rng = np.random.default_rng(1411)
    for degree in (1, 3, 6):
        a = rng.integers(-8, 9, degree + 1).astype(np.float32)
        x = rng.integers(-4, 5, 400).astype(np.float32)
        want = np.array([sum(int(a[i]) * int(v) ** i for i in range(degree + 1)) for v in x])
        assert np.all(np.abs(want) < 2 ** 24)
        assert np.array_equal(oracle.horner_f32(a, x), want.astype(np.float32))
        assert np.array_equal(oracle.horner_comp(a, x), want.astype(np.float32))
        yh, yl = oracle.horner_ff(a, _zeros(a.size), x, _zeros(x.size))
        assert np.array_equal(yh, want.astype(np.float32)) and np.all(yl == 0)


def _check_bounds(a, x, label):
    """Horner, CompHorner and ff Horner against their bounds at points x
    (binary32 coefficients a)."""
    n = a.size - 1
    coeffs = [frac(c) for c in a]
    h = oracle.horner_f32(a, x)
    c = oracle.horner_comp(a, x)
    fh, fl = oracle.horner_ff(a, _zeros(a.size), x, _zeros(x.size))
    for k in range(x.size):
        xk = frac(x[k])
        exact = _exact_poly(coeffs, xk)
        mag = _abs_poly(coeffs, xk)
        assert abs(frac(h[k]) - exact) <= gamma(2 * n, U) * mag, (label, "horner", k)
        assert abs(frac(c[k]) - exact) <= U * abs(exact) + gamma(2 * n, U) ** 2 * mag, \
            (label, "comp", k)
        assert abs(ff_value(fh[k], fl[k]) - exact) <= gamma(2 * n, V) * mag, (label, "ff", k)
    return h, c, (fh, fl)


@pytest.mark.parametrize("n", [3, 7, 11, 25])
def test_binomial_closed_form(n):
    a = fi.binomial_poly(n).numpy()
    far = fi.horner_points(300, 1421 + n, 0.5, 1.5).numpy()
    near = fi.horner_points(300, 1431 + n, 1 - 2.0 ** -6, 1 + 2.0 ** -6).numpy()
    for x, label in ((far, "far"), (near, "near")):
        h, c, (fh, fl) = _check_bounds(a, x, label)
        # the closed form, independent of any evaluation scheme: p(x) =
        # (x - 1)^n and p~(|x|) = (1 + |x|)^n for these coefficients
        for k in range(0, x.size, 5):
            xk = frac(x[k])
            exact, mag = (xk - 1) ** n, (1 + abs(xk)) ** n
            assert abs(frac(c[k]) - exact) <= U * abs(exact) + gamma(2 * n, U) ** 2 * mag
            assert abs(ff_value(fh[k], fl[k]) - exact) <= gamma(2 * n, V) * mag


@pytest.mark.parametrize("degree", [1, 8, 40])
def test_random_polynomials(degree):
    a = fi.random_poly(degree, 1441 + degree).numpy()
    x = fi.horner_points(300, 1451 + degree, -1.5, 1.5).numpy()
    _check_bounds(a, x, f"random degree {degree}")


def test_compensated_is_as_if_twice_the_precision():
    # (x - 1)^5 at 1 +- 2^-4: condition numbers up to ~2^30 and beyond
    n = 5
    a = fi.binomial_poly(n).numpy()
    x = fi.horner_points(400, 1461, 1 - 2.0 ** -4, 1 + 2.0 ** -4).numpy()
    h, c = oracle.horner_f32(a, x), oracle.horner_comp(a, x)
    worst_h, checked = Fraction(0), 0
    for k in range(x.size):
        xk = frac(x[k])
        exact = (xk - 1) ** n
        if exact == 0:
            continue
        cond = (1 + abs(xk)) ** n / abs(exact)
        rel_c = abs(frac(c[k]) - exact) / abs(exact)
        assert rel_c <= U + gamma(2 * n, U) ** 2 * cond
        if cond < 2 ** 30:
            checked += 1
            assert rel_c <= Fraction(1, 1 << 12)
            worst_h = max(worst_h, abs(frac(h[k]) - exact) / abs(exact))
    assert checked > 100
    assert worst_h > 1      # Horner in binary32: no correct digit there


def test_float_float_coefficients_and_points():
    degree = 12
    a = fi.random_poly(degree, 1471, ff=True).numpy()
    xs = fi.split_f64(fi.horner_points(300, 1472, -1.2, 1.2).double()
                      + 1e-9 * fi.horner_points(300, 1473, -1, 1).double()).numpy()
    assert np.count_nonzero(a[1]) > degree // 2 and np.count_nonzero(xs[1]) > 200
    yh, yl = oracle.horner_ff(a[0], a[1], xs[0], xs[1])
    coeffs = [ff_value(a[0][i], a[1][i]) for i in range(degree + 1)]
    for k in range(xs.shape[1]):
        xk = ff_value(xs[0][k], xs[1][k])
        exact = _exact_poly(coeffs, xk)
        assert abs(ff_value(yh[k], yl[k]) - exact) <= gamma(2 * degree, V) * _abs_poly(coeffs, xk), k


def test_sign_symmetry():
    # p(-x) with a_i (-1)^i is p(x), and -p with -a: bit for bit
    a = fi.random_poly(9, 1481).numpy()
    x = fi.horner_points(500, 1482, -1.5, 1.5).numpy()
    alt = (a * np.array([(-1.0) ** i for i in range(a.size)], np.float32)).astype(np.float32)
    for fn in (oracle.horner_f32, oracle.horner_comp):
        r = fn(a, x)
        assert same_bits(fn(alt, -x), r)
        neg = fn(-a, x)
        nz = r != 0
        assert same_bits(neg[nz], -r[nz])
