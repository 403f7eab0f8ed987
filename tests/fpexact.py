"""Exact-arithmetic helpers for the tests (no float-float operators here).

Values are converted to ``fractions.Fraction`` (exact for every finite
binary32/binary64 number) or to integer significand/exponent pairs, so that
the tests can check identities such as s + r == a + b without any rounding.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

F32_MIN_NORMAL_EXP = -126


def frac(v) -> Fraction:
    """Exact value of a float (binary32 or binary64) as a Fraction."""
    return Fraction(float(v))


def ff_value(hi, lo) -> Fraction:
    """Exact value hi + lo of a float-float pair."""
    return frac(hi) + frac(lo)


def exponent32(v: float) -> int:
    """E with 2^E <= |v| < 2^(E+1) for a nonzero binary32 value."""
    m, e = math.frexp(float(v))
    return e - 1


def ulp32(v: float) -> Fraction:
    """Unit in the last place of a binary32 number (subnormal spacing 2^-149)."""
    if v == 0:
        return Fraction(1, 1 << 149)
    e = max(exponent32(v), F32_MIN_NORMAL_EXP)
    return Fraction(2) ** (e - 23)


def sigbits(v: float) -> int:
    """Number of bits from the leading one to the trailing one of |v|."""
    if v == 0:
        return 0
    f = Fraction(abs(float(v)))
    num, den = f.numerator, f.denominator
    # v = num / den with den a power of two; strip trailing zeros of num
    tz = (num & -num).bit_length() - 1
    return num.bit_length() - tz


def bits32(a) -> np.ndarray:
    """Raw binary32 bit patterns (uint32) of an array."""
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def same_bits(a, b) -> bool:
    """Bitwise equality of two float32 arrays, any NaN equal to any NaN."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    nan = np.isnan(a) & np.isnan(b)
    return bool(np.all((bits32(a) == bits32(b)) | nan))


def mismatch_report(a, b, limit: int = 5) -> str:
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    bad = np.nonzero((bits32(a) != bits32(b)) & ~(np.isnan(a) & np.isnan(b)))[0]
    rows = [f"{len(bad)} mismatches"]
    for i in bad[:limit]:
        rows.append(f"  [{i}] {a[i]!r} ({bits32(a)[i]:08x}) vs {b[i]!r} ({bits32(b)[i]:08x})")
    return "\n".join(rows)


def log2_abs(x: Fraction) -> float:
    """log2 |x| for a Fraction (-inf for zero)."""
    if x == 0:
        return float("-inf")
    x = abs(x)
    return math.log2(x.numerator) - math.log2(x.denominator)


def round_to_f32(q: Fraction) -> float:
    """The binary32 value nearest to q, ties to even (subnormals included,
    no overflow handling: |q| must stay below 2^128)."""
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1                       # now 2^e <= q < 2^(e+1)
    quantum = Fraction(2) ** (max(e, F32_MIN_NORMAL_EXP) - 23)
    m = q / quantum
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return sign * float(lo * quantum)
