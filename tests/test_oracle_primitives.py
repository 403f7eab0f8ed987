"""Pins of the oracle's error-free transformations (section 4.1 theorems).

Each check compares the oracle with mathematics that does not depend on it:
exact rational arithmetic (Fraction), the exactness of binary32 products in
binary64, NumPy's own IEEE binary32 rounding, and exhaustive enumeration.
"""
import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import exponent32, frac, sigbits, same_bits, ulp32


def _np(t):
    return t.cpu().numpy()


# ------------------------------------------------------------------ Add12

@pytest.mark.parametrize("emin,emax", [(-40, 40), (-120, 120), (-8, 8)])
def test_add12_is_exact_and_rounds_like_ieee(emin, emax):
    a = _np(fi.random_f32(4096, 11, emin, emax))
    b = _np(fi.random_f32(4096, 12, emin, emax))
    s, r = oracle.add12(a, b)
    # s is the IEEE binary32 sum (NumPy rounds float32 addition itself)
    assert same_bits(s, (a + b).astype(np.float32))
    for ai, bi, si, ri in zip(a, b, s, r):
        assert frac(si) + frac(ri) == frac(ai) + frac(bi)
        assert abs(frac(ri)) <= ulp32(si) / 2


def test_add12_opposite_signs_non_overlapping():
    # The failure class named in the accuracy discussion (section 6.1):
    # opposite signs and non-overlapping significands.  On round-to-nearest
    # hardware Add12 must stay exact.
    a = _np(fi.random_f32(4096, 21, -10, 10))
    gaps = np.arange(4096) % 60 + 1
    b = (-np.sign(a) * np.abs(a) * np.ldexp(1.0, -gaps)).astype(np.float32)
    b = b * (1 + (np.arange(4096) % 7) / 8.0).astype(np.float32)
    for x, y in ((a, b), (b, a)):
        s, r = oracle.add12(x, y)
        for ai, bi, si, ri in zip(x, y, s, r):
            assert frac(si) + frac(ri) == frac(ai) + frac(bi)


def test_add12_sterbenz_pairs_have_zero_error():
    # Sterbenz lemma (section 4.1): y/2 <= x <= 2y  =>  x - y is exact, so the
    # Add12 error word of (x, -y) is zero.
    x = _np(fi.random_f32(4096, 31, -20, 20))
    f = (1.0 + (np.arange(4096) % 97) / 97.0).astype(np.float32)   # in [1, 2)
    y = np.abs(x) * f
    x = np.abs(x)
    s, r = oracle.add12(x, -y)
    assert np.all(r == 0)
    assert np.all(s.astype(np.float64) == x.astype(np.float64) - y.astype(np.float64))


def test_fast_add12_exact_when_ordered_and_matches_add12():
    a = _np(fi.random_f32(4096, 41, -30, 30))
    b = _np(fi.random_f32(4096, 42, -30, 30))
    big = np.where(np.abs(a) >= np.abs(b), a, b)
    small = np.where(np.abs(a) >= np.abs(b), b, a)
    s, r = oracle.fast_add12(big, small)
    s2, r2 = oracle.add12(big, small)
    for ai, bi, si, ri in zip(big, small, s, r):
        assert frac(si) + frac(ri) == frac(ai) + frac(bi)
    assert same_bits(s, s2) and same_bits(r, r2)


# ------------------------------------------------------------------ Split

def _check_split(a, hi, lo):
    a64, hi64, lo64 = (v.astype(np.float64) for v in (a, hi, lo))
    assert np.all(hi64 + lo64 == a64)                  # exact: hi + lo = a
    assert np.all(np.abs(hi64) >= np.abs(lo64))
    e = np.frexp(a64)[1] - 1                           # 2^e <= |a| < 2^(e+1)
    # hi holds p - s = 12 bits: a multiple of 2^(e - 11) ...
    assert np.all(np.ldexp(hi64, 11 - e) == np.round(np.ldexp(hi64, 11 - e)))
    # ... and lo (s = 12 bits) is at most half that granule, so they do not
    # overlap; lo is a multiple of ulp(a) = 2^(e - 23) by construction.
    assert np.all(np.abs(lo64) <= np.ldexp(1.0, e - 12))
    assert np.all(np.ldexp(lo64, 23 - e) == np.round(np.ldexp(lo64, 23 - e)))


def test_split_exhaustive_unit_binade():
    # Every binary32 value in [1, 2): 2^23 inputs.
    a = (np.arange(1 << 23, dtype=np.uint32) | np.uint32(127 << 23)).view(np.float32)
    hi, lo = oracle.split(a)
    _check_split(a, hi, lo)
    # the low word needs at most 11 significant bits (sign carries the 12th)
    lo_bits = max(sigbits(v) for v in lo[:: 4099])
    assert lo_bits <= 12
    nz = lo[lo != 0]
    assert nz.size > 0


def test_split_exhaustive_negative_binade_is_symmetric():
    a = (np.arange(1 << 23, dtype=np.uint32) | np.uint32((127 << 23) | (1 << 31))).view(np.float32)
    hi, lo = oracle.split(a)
    hi_p, lo_p = oracle.split(-a)
    # symmetric in value (an exact zero low word is +0 for either sign)
    assert np.array_equal(hi, -hi_p) and np.array_equal(lo, -lo_p)
    _check_split(a, hi, lo)


@pytest.mark.parametrize("e", list(range(-110, 111, 13)))
def test_split_other_binades(e):
    frac_bits = np.random.default_rng(e + 500).integers(0, 1 << 23, 1 << 15, dtype=np.uint32)
    a = (frac_bits | np.uint32((127 + e) << 23)).view(np.float32)
    hi, lo = oracle.split(a)
    _check_split(a, hi, lo)


# ------------------------------------------------------------------ Mul12

@pytest.mark.parametrize("dekker", [False, True])
@pytest.mark.parametrize("emin,emax", [(-50, 50), (-8, 8)])
def test_mul12_is_exact(dekker, emin, emax):
    # Mul12 theorem (section 4.1): exact when no underflow occurs; exponents
    # >= -50 keep the error word (>= 2^-150 * 2^48) in the normal range.
    a = _np(fi.random_f32(1 << 16, 51, emin, emax))
    b = _np(fi.random_f32(1 << 16, 52, emin, emax))
    x, y = oracle.mul12(a, b, dekker=dekker)
    p = a.astype(np.float64) * b.astype(np.float64)    # exact: 48-bit product
    assert same_bits(x, p.astype(np.float32))           # x is the rounded product
    # x + y = a*b exactly.  If y is right, x + y has <= 48 bits and the binary64
    # sum below is exact; the Fraction check on a subset removes any doubt.
    assert np.all(x.astype(np.float64) + y.astype(np.float64) == p)
    for i in range(0, a.size, 64):
        assert frac(x[i]) + frac(y[i]) == frac(a[i]) * frac(b[i])
        assert abs(frac(y[i])) <= ulp32(x[i]) / 2


def test_mul12_dekker_equals_fma_in_range():
    # Both forms return the unique (x, y) with x = fl(a*b), y = a*b - x
    # whenever that error is representable (no underflow, no overflow).
    a = _np(fi.random_f32(1 << 16, 61, -50, 50))
    b = _np(fi.random_f32(1 << 16, 62, -50, 50))
    x1, y1 = oracle.mul12(a, b, dekker=False)
    x2, y2 = oracle.mul12(a, b, dekker=True)
    assert same_bits(x1, x2) and same_bits(y1, y2)


def test_mul12_special_small_cases():
    # closed forms: powers of two multiply exactly (error 0); (1 + 2^-12)^2
    # = 1 + 2^-11 + 2^-24 whose last bit is the exact error.
    a = np.array([2.0 ** 10, 1 + 2.0 ** -12, 3.0], np.float32)
    b = np.array([1.5, 1 + 2.0 ** -12, 1.0 / 3.0], np.float32)
    for dekker in (False, True):
        x, y = oracle.mul12(a, b, dekker=dekker)
        assert x[0] == 1536.0 and y[0] == 0.0
        assert x[1] == np.float32(1 + 2.0 ** -11) and y[1] == np.float32(2.0 ** -24)
        assert frac(x[2]) + frac(y[2]) == frac(a[2]) * frac(b[2])


def test_exponent_helper_sanity():
    assert exponent32(1.0) == 0 and exponent32(1.5) == 0 and exponent32(0.75) == -1
