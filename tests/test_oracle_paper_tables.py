"""Pins of the oracle routines behind the paper's measurement tables
(section 6): the binary32 reference operators timed beside the float-float
ones (Tables 3 and 4), and the exact error measurement of the accuracy table
(section 6.1, Table 5).

* add and multiply against numpy's binary32 arithmetic (an independent IEEE
  implementation);
* multiply-add against the exact a*b + c rounded once to binary32 (Fraction);
* the error measurement against Fraction arithmetic on perturbed results,
  exact results, and the zero-exact-value edge case.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac, round_to_f32, same_bits, ulp32


def _np(t):
    return t.cpu().numpy()


def test_round_to_f32_helper():
    # the helper itself: representable values, halfway ties, subnormals
    assert round_to_f32(Fraction(3, 2)) == 1.5
    one_ulp = Fraction(1, 1 << 23)
    assert round_to_f32(1 + one_ulp / 2) == 1.0                        # tie to even
    assert round_to_f32(1 + 3 * one_ulp / 2) == float(1 + 2 * one_ulp)  # tie to even
    assert round_to_f32(Fraction(1, 1 << 149) * Fraction(3, 4)) == 2.0 ** -149
    assert round_to_f32(-Fraction(1, 1 << 150)) == 0.0                 # tie to even (0)
    for v in _np(fi.random_f32(200, 3, -126, 100)):
        assert round_to_f32(frac(v)) == float(v)


@pytest.mark.parametrize("op", ["add", "mul"])
def test_f32_add_mul_match_numpy(op):
    a = _np(fi.random_f32(20000, 11, -60, 60))
    b = _np(fi.random_f32(20000, 12, -60, 60))
    # subnormal results and operands
    a[:200] = _np(fi.random_f32(200, 13, -126, -100))
    b[:200] = _np(fi.random_f32(200, 14, -126, -100))
    want = (a + b) if op == "add" else (a * b)
    assert same_bits(oracle.f32_ref(op, a, b), want.astype(np.float32))


def test_f32_mad_is_a_single_rounding():
    a = _np(fi.random_f32(3000, 21, -30, 30))
    b = _np(fi.random_f32(3000, 22, -30, 30))
    c = _np(fi.random_f32(3000, 23, -30, 30))
    # c close to -a*b: the cases where a separate product rounding shows
    c[:1000] = -(a[:1000].astype(np.float64) * b[:1000]).astype(np.float32)
    r = oracle.f32_ref("mad", a, b, c)
    differs = 0
    for i in range(a.size):
        want = round_to_f32(frac(a[i]) * frac(b[i]) + frac(c[i]))
        assert float(r[i]) == want, (i, a[i], b[i], c[i])
        differs += float(np.float32(np.float32(a[i] * b[i]) + c[i])) != want
    assert differs > 100      # the pin distinguishes fused from unfused


def _expected_errors(op, ah, al, bh, bl, rh, rl):
    """(rel, ratio) with Fraction arithmetic."""
    if op == "add22":
        exact = ff_value(ah, al) + ff_value(bh, bl)
        bound = max(abs(frac(al) + frac(bl)) / 2 ** 24, abs(exact) / 2 ** 44)
    elif op == "mul22":
        exact = ff_value(ah, al) * ff_value(bh, bl)
        bound = abs(exact) / 2 ** 44
    elif op == "add12":
        exact, bound = frac(ah) + frac(bh), Fraction(0)
    else:
        exact, bound = frac(ah) * frac(bh), Fraction(0)
    err = abs(ff_value(rh, rl) - exact)
    if err == 0:
        return 0.0, 0.0
    rel = math.inf if exact == 0 else float(err / abs(exact))
    ratio = math.inf if bound == 0 else float(err / bound)
    return rel, ratio


@pytest.mark.parametrize("op", ["add22", "mul22", "add12", "mul12"])
def test_ff_errors_against_fractions(op):
    n = 1500
    a, b = _np(fi.random_ff(n, 31, -20, 20)), _np(fi.random_ff(n, 32, -20, 20))
    if op in ("add12", "mul12"):
        a[1] = 0.0
        b[1] = 0.0
    ah, al, bh, bl = a[0], a[1], b[0], b[1]
    fn = {"add22": oracle.add22, "mul22": oracle.mul22}.get(op)
    if fn is not None:
        rh, rl = fn(ah, al, bh, bl)
    elif op == "add12":
        rh, rl = oracle.add12(ah, bh)
    else:
        rh, rl = oracle.mul12(ah, bh)
    rh, rl = rh.copy(), rl.copy()
    # perturb a third of the results by one unit of the low word (or of hi's
    # last place when lo is zero), so that the errors are nonzero and varied
    k = np.arange(n) % 3 == 0
    step = np.where(rl != 0, np.abs(rl) * np.float32(2.0 ** -20), np.float32(0.0))
    rl[k] = (rl[k] + step[k]).astype(np.float32)
    rel, ratio = oracle.ff_errors(op, ah, al, bh, bl, rh, rl)
    for i in range(n):
        wr, wq = _expected_errors(op, ah[i], al[i], bh[i], bl[i], rh[i], rl[i])
        for got, want in ((rel[i], wr), (ratio[i], wq)):
            if math.isinf(want) or want == 0.0:
                assert got == want, (op, i, got, want)
            else:
                assert abs(got - want) <= 1e-12 * want, (op, i, got, want)
    if op in ("add22", "mul22"):
        assert np.all(ratio[~k] <= 1.0)       # the unperturbed results meet the theorems
    else:
        assert np.all(ratio[~k] == 0.0)       # exact transforms


def test_ff_errors_edge_cases():
    one, z = np.float32([1.0]), np.float32([0.0])
    # exact zero result of a cancelling sum: no error
    rel, ratio = oracle.ff_errors("add22", one, z, -one, z, z, z)
    assert rel[0] == 0.0 and ratio[0] == 0.0
    # nonzero result where the exact value is zero: infinite relative error
    rel, ratio = oracle.ff_errors("add22", one, z, -one, z, np.float32([2.0 ** -30]), z)
    assert math.isinf(rel[0]) and math.isinf(ratio[0])
    # an error of 2^-52 on 1 + 2^-30: relative 2^-52 / (1 + 2^-30)
    rel, ratio = oracle.ff_errors("add12", one, z, np.float32([2.0 ** -30]), z, one,
                                  np.float32([2.0 ** -30 + 2.0 ** -52]))
    assert rel[0] == pytest.approx(2.0 ** -52 / (1 + 2.0 ** -30), rel=1e-12, abs=0)
    assert math.isinf(ratio[0])
    # negative exact value far below its largest term (cancellation inside
    # the accumulator): -(2^-100) from 2^20 + (-2^20 - 2^-100)
    big = np.float32([2.0 ** 20])
    rel, ratio = oracle.ff_errors("add22", big, z, -big, np.float32([-(2.0 ** -100)]),
                                  np.float32([-(2.0 ** -100) * (1 + 2.0 ** -10)]), z)
    assert rel[0] == pytest.approx(2.0 ** -10, rel=1e-12, abs=0)
