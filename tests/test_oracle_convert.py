"""Pins of the oracle's binary64 <-> float-float conversions.

* from binary64: hi is x rounded to binary32 (numpy's cast, an independent
  implementation); lo is normalised (|lo| <= ulp(hi)/2) and hi + lo is x to
  within 2^-48 |x| (exact Fraction error) over the normal range;
* to binary64: (double) hi + (double) lo is hi + lo rounded once to
  binary64 (Python's correctly rounded Fraction -> float conversion), also
  for pairs whose words are far apart; a pair whose bits fit in 53 comes back
  exactly, and converting it again returns the same pair.
"""
from fractions import Fraction

import numpy as np

import ff_inputs as fi
import oracle
from fpexact import frac, same_bits, ulp32


def _random_f64(n, seed, emin=-100, emax=100):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    return np.ldexp(m, rng.integers(emin, emax + 1, n))


def test_from_f64_rounds_hi_and_keeps_48_bits():
    x = _random_f64(20000, 2001)
    hi, lo = oracle.from_f64(x)
    assert same_bits(hi, x.astype(np.float32))
    for i in range(0, x.size, 7):
        xi = Fraction(float(x[i]))
        err = abs(frac(hi[i]) + frac(lo[i]) - xi)
        assert err <= Fraction(1, 1 << 48) * abs(xi), i
        assert abs(frac(lo[i])) <= ulp32(hi[i]) / 2
        assert np.float32(hi[i]) + np.float32(lo[i]) == np.float32(hi[i])


def test_from_f64_of_binary32_values_is_exact():
    x = fi.random_f32(5000, 2002, -100, 100).numpy()
    hi, lo = oracle.from_f64(x.astype(np.float64))
    assert same_bits(hi, x) and np.all(lo == 0)


def test_to_f64_rounds_once():
    pairs = fi.random_ff(20000, 2003, -60, 60, max_gap=40).numpy()
    x = oracle.to_f64(pairs[0], pairs[1])
    for i in range(0, x.shape[0], 5):
        assert x[i] == float(frac(pairs[0][i]) + frac(pairs[1][i])), i


def test_round_trip_where_the_bits_fit():
    x = _random_f64(20000, 2004, -60, 60)
    hi, lo = oracle.from_f64(x)
    back = oracle.to_f64(hi, lo)
    checked = 0
    for i in range(x.size):
        if lo[i] == 0:
            continue
        span = np.frexp(hi[i])[1] - (np.frexp(lo[i])[1] - 24)
        if span <= 53:
            checked += 1
            assert Fraction(float(back[i])) == frac(hi[i]) + frac(lo[i]), i
            h2, l2 = oracle.from_f64(back[i:i + 1])
            assert same_bits(h2, hi[i:i + 1]) and same_bits(l2, lo[i:i + 1]), i
    assert checked > 10000
