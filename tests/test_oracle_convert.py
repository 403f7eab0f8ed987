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


# Values outside the float-float range: the documented operation sequence
# still fixes every word (IEEE binary32/binary64 rules), though the pairs are
# not float-float numbers.
_FMAX = float(np.finfo(np.float32).max)
_THRESH = _FMAX + 2.0 ** 103          # binary32 overflow threshold (ties to even: inf)


def _special_inputs():
    return np.array([np.inf, -np.inf, np.nan, _FMAX, -_FMAX, _THRESH, -_THRESH,
                     np.nextafter(_THRESH, 0.0), 1e39, -1e300, 0.0, -0.0, 5e-324, 1e-46],
                    dtype=np.float64)


def test_from_f64_special_values_closed_forms():
    x = _special_inputs()
    hi, lo = oracle.from_f64(x)
    inf = np.float32(np.inf)
    # infinities: hi = x, lo = fl32(inf - inf) = NaN
    assert hi[0] == inf and np.isnan(lo[0]) and hi[1] == -inf and np.isnan(lo[1])
    assert np.isnan(hi[2]) and np.isnan(lo[2])
    # FLT_MAX is a binary32 value: exact, lo = +0
    assert hi[3] == np.float32(_FMAX) and lo[3] == 0 and not np.signbit(lo[3])
    assert hi[4] == -np.float32(_FMAX) and lo[4] == 0
    # at the overflow threshold hi rounds to inf and lo = fl32(x - inf) = -inf
    assert hi[5] == inf and lo[5] == -inf and hi[6] == -inf and lo[6] == inf
    # just below it hi = FLT_MAX and lo = fl32(x - FLT_MAX) = fl32(2^103 - 2^75)
    # = 2^103: a valid pair within 2^-48 |x| (here 2^-53) of x
    assert hi[7] == np.float32(_FMAX) and lo[7] == np.float32(2.0 ** 103)
    xi = Fraction(float(x[7]))
    assert abs(frac(hi[7]) + frac(lo[7]) - xi) <= Fraction(1, 1 << 48) * xi
    assert hi[8] == inf and lo[8] == -inf and hi[9] == -inf and lo[9] == inf
    # signed zeros: hi keeps the sign, lo = fl32(x - hi) = +0
    assert hi[10] == 0 and not np.signbit(hi[10]) and lo[10] == 0 and not np.signbit(lo[10])
    assert hi[11] == 0 and np.signbit(hi[11]) and lo[11] == 0 and not np.signbit(lo[11])
    # below half the smallest binary32 subnormal: hi = 0, lo = fl32(x) = 0
    assert hi[12] == 0 and lo[12] == 0 and hi[13] == 0 and lo[13] == 0


def test_to_f64_special_pairs_closed_forms():
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    hi = np.array([inf, inf, -inf, nan, inf, np.float32(_FMAX), 0.0], np.float32)
    lo = np.array([0.0, nan, inf, 1.0, -inf, np.float32(_FMAX), -0.0], np.float32)
    x = oracle.to_f64(hi, lo)
    assert x[0] == np.inf and np.isnan(x[1]) and np.isnan(x[2]) and np.isnan(x[3])
    assert np.isnan(x[4])
    assert x[5] == 2.0 * _FMAX                      # finite in binary64
    assert x[6] == 0 and not np.signbit(x[6])       # +0 + -0 = +0
