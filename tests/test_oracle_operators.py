"""Pins of the oracle's float-float operators (section 4.1: Add22 and Mul22
theorems; Div22 after Dekker's div2).

Checks: closed forms (zero low words reduce Add22/Mul22 to the exact Add12 /
Mul12 pair), identities (a + 0, a - a, a * 1, a / 1, a / a), bitwise
commutativity, exact scaling by powers of two, normalised outputs, and the
paper's error bounds measured exactly with Fraction on random, cancellation
and exponent-gap inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac, same_bits, ulp32

TWO_M24 = Fraction(1, 1 << 24)
TWO_M44 = Fraction(1, 1 << 44)


def _np(t):
    return t.cpu().numpy()


def _operands(kind: str, n: int, seed: int):
    """(ah, al, bh, bl) numpy planes for one input family."""
    if kind == "random":
        a, b = fi.random_ff(n, seed, -30, 30), fi.random_ff(n, seed + 1, -30, 30)
    elif kind == "near":       # similar magnitudes: many Add22 branch flips
        a, b = fi.random_ff(n, seed, -2, 2), fi.random_ff(n, seed + 1, -2, 2)
    elif kind == "mixed":      # the elementwise workload (cancellation + gaps)
        a, b, _ = fi.mixed_ff_pair(n, seed)
    elif kind == "cancel":
        a, b, _ = fi.mixed_ff_pair(n, seed, p_cancel=1.0, p_gap=0.0)
    elif kind == "gap":
        a, b, _ = fi.mixed_ff_pair(n, seed, p_cancel=0.0, p_gap=1.0)
    else:
        raise ValueError(kind)
    a, b = _np(a), _np(b)
    return a[0], a[1], b[0], b[1]


def _assert_normalised(rh, rl):
    for h, l in zip(rh, rl):
        assert abs(frac(l)) <= ulp32(h) / 2
        assert np.float32(h) + np.float32(l) == np.float32(h)


FAMILIES = ["random", "near", "mixed", "cancel", "gap"]


# ------------------------------------------------------------------ Add22

def test_add22_zero_low_words_is_the_exact_add12_pair():
    ah, _, bh, _ = _operands("random", 4096, 101)
    z = np.zeros_like(ah)
    rh, rl = oracle.add22(ah, z, bh, z)
    assert same_bits(rh, (ah + bh).astype(np.float32))
    for a, b, h, l in zip(ah, bh, rh, rl):
        assert frac(h) + frac(l) == frac(a) + frac(b)


def test_add22_identities():
    ah, al, bh, bl = _operands("random", 4096, 111)
    z = np.zeros_like(ah)
    rh, rl = oracle.add22(ah, al, z, z)                      # a + 0 = a
    assert same_bits(rh, ah) and np.array_equal(rl, al)
    rh, rl = oracle.add22(ah, al, -ah, -al)                  # a - a = +0
    assert np.all(rh == 0) and np.all(rl == 0)
    assert not np.any(np.signbit(rh))
    rh, rl = oracle.sub22(ah, al, ah, al)
    assert np.all(rh == 0) and np.all(rl == 0)


@pytest.mark.parametrize("kind", FAMILIES)
def test_add22_commutes_bitwise(kind):
    ah, al, bh, bl = _operands(kind, 1 << 14, 121)
    r1 = oracle.add22(ah, al, bh, bl)
    r2 = oracle.add22(bh, bl, ah, al)
    assert same_bits(r1[0], r2[0]) and same_bits(r1[1], r2[1])


def test_add22_sign_symmetry_and_power_of_two_scaling():
    ah, al, bh, bl = _operands("random", 1 << 14, 131)
    rh, rl = oracle.add22(ah, al, bh, bl)
    nh, nl = oracle.add22(-ah, -al, -bh, -bl)
    assert np.array_equal(nh, -rh) and np.array_equal(nl, -rl)
    for k in (-20, 7, 33):
        s = np.float32(2.0 ** k)
        sh, sl = oracle.add22(ah * s, al * s, bh * s, bl * s)
        assert np.array_equal(sh, rh * s) and np.array_equal(sl, rl * s)


def test_sub22_is_add22_of_the_negation():
    ah, al, bh, bl = _operands("mixed", 1 << 14, 141)
    d = oracle.sub22(ah, al, bh, bl)
    s = oracle.add22(ah, al, -bh, -bl)
    assert same_bits(d[0], s[0]) and same_bits(d[1], s[1])


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("op", ["add", "sub"])
def test_add22_error_bound(kind, op):
    # Add22 theorem: |delta| <= max(2^-24 |al + bl|, 2^-44 |a + b|).
    ah, al, bh, bl = _operands(kind, 3000, 151)
    if op == "sub":
        rh, rl = oracle.sub22(ah, al, bh, bl)
        bh, bl = -bh, -bl
    else:
        rh, rl = oracle.add22(ah, al, bh, bl)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) + ff_value(bh[i], bl[i])
        delta = ff_value(rh[i], rl[i]) - exact
        bound = max(TWO_M24 * abs(frac(al[i]) + frac(bl[i])), TWO_M44 * abs(exact))
        assert abs(delta) <= bound, (i, ah[i], al[i], bh[i], bl[i])
    _assert_normalised(rh[:512], rl[:512])


def test_add22_relative_bound_without_cancellation():
    # same signs: the bound above is relative, |delta| <= 2^-44 |a + b|
    ah, al, bh, bl = _operands("random", 4000, 161)
    # make both values positive: scaling both words by sign(hi) is exact
    sa, sb = np.sign(ah), np.sign(bh)
    ah, al, bh, bl = ah * sa, al * sa, bh * sb, bl * sb
    rh, rl = oracle.add22(ah, al, bh, bl)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) + ff_value(bh[i], bl[i])
        assert abs(ff_value(rh[i], rl[i]) - exact) <= TWO_M44 * abs(exact)


# ------------------------------------------------------------------ Mul22

@pytest.mark.parametrize("dekker", [False, True])
def test_mul22_zero_low_words_is_the_exact_product_pair(dekker):
    ah, _, bh, _ = _operands("random", 4096, 201)
    z = np.zeros_like(ah)
    rh, rl = oracle.mul22(ah, z, bh, z, dekker=dekker)
    assert same_bits(rh, (ah.astype(np.float64) * bh.astype(np.float64)).astype(np.float32))
    for a, b, h, l in zip(ah, bh, rh, rl):
        assert frac(h) + frac(l) == frac(a) * frac(b)


@pytest.mark.parametrize("dekker", [False, True])
def test_mul22_identities_commutation_scaling(dekker):
    ah, al, bh, bl = _operands("random", 1 << 14, 211)
    one, z = np.ones_like(ah), np.zeros_like(ah)
    rh, rl = oracle.mul22(ah, al, one, z, dekker=dekker)     # a * 1 = a
    assert same_bits(rh, ah) and np.array_equal(rl, al)
    r1 = oracle.mul22(ah, al, bh, bl, dekker=dekker)
    r2 = oracle.mul22(bh, bl, ah, al, dekker=dekker)
    assert same_bits(r1[0], r2[0]) and same_bits(r1[1], r2[1])
    for k in (-9, 13):
        s = np.float32(2.0 ** k)
        sh, sl = oracle.mul22(ah * s, al * s, bh, bl, dekker=dekker)
        assert np.array_equal(sh, r1[0] * s) and np.array_equal(sl, r1[1] * s)


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("dekker", [False, True])
def test_mul22_relative_error_bound(kind, dekker):
    # Mul22 theorem: rh + rl = a*b (1 + eps), |eps| <= 2^-44.
    ah, al, bh, bl = _operands(kind, 3000, 221)
    rh, rl = oracle.mul22(ah, al, bh, bl, dekker=dekker)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) * ff_value(bh[i], bl[i])
        err = ff_value(rh[i], rl[i]) - exact
        if abs(exact) < Fraction(2) ** -96:
            continue    # error words near the subnormal range: bound not claimed
        assert abs(err) <= TWO_M44 * abs(exact), (i, ah[i], al[i], bh[i], bl[i])
    _assert_normalised(rh[:512], rl[:512])


# ------------------------------------------------------------------ Div22

def test_div22_identities():
    ah, al, bh, bl = _operands("random", 1 << 14, 301)
    one, z = np.ones_like(ah), np.zeros_like(ah)
    rh, rl = oracle.div22(ah, al, one, z)                      # a / 1 = a
    assert same_bits(rh, ah) and np.array_equal(rl, al)
    rh, rl = oracle.div22(ah, al, ah, al)                      # a / a = 1
    assert np.all(rh == 1.0) and np.all(rl == 0.0)
    r1 = oracle.div22(ah, al, bh, bl)
    for k in (-11, 5):
        s = np.float32(2.0 ** k)
        sh, sl = oracle.div22(ah * s, al * s, bh, bl)
        assert np.array_equal(sh, r1[0] * s) and np.array_equal(sl, r1[1] * s)
        sh, sl = oracle.div22(ah, al, bh * s, bl * s)
        assert np.array_equal(sh, r1[0] / s) and np.array_equal(sl, r1[1] / s)


def test_div22_exact_quotients():
    # q * b / b: when q*b is held exactly as a float-float (zero low words,
    # Mul12 pair), the quotient of that value by b is q itself, which Div22
    # must return as (q, 0): c = fl(th/b) = q exactly is not guaranteed, so
    # only the value is asserted, within the relative bound.
    q = _np(fi.random_f32(2048, 311, -10, 10))
    b = _np(fi.random_f32(2048, 312, -10, 10))
    z = np.zeros_like(q)
    th, tl = oracle.mul22(q, z, b, z)
    rh, rl = oracle.div22(th, tl, b, z)
    for i in range(q.size):
        assert abs(ff_value(rh[i], rl[i]) - frac(q[i])) <= TWO_M44 * abs(frac(q[i]))


@pytest.mark.parametrize("kind", FAMILIES)
@pytest.mark.parametrize("dekker", [False, True])
def test_div22_relative_error_bound(kind, dekker):
    # Stated bound for Dekker's div2 in binary32: |eps| <= 2^-44 (the known
    # double-word division bounds are below 16 u^2 = 2^-44 for u = 2^-24).
    ah, al, bh, bl = _operands(kind, 3000, 321)
    rh, rl = oracle.div22(ah, al, bh, bl, dekker=dekker)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) / ff_value(bh[i], bl[i])
        err = ff_value(rh[i], rl[i]) - exact
        if abs(exact) < Fraction(2) ** -96:
            continue
        assert abs(err) <= TWO_M44 * abs(exact), (i, ah[i], al[i], bh[i], bl[i])
    _assert_normalised(rh[:512], rl[:512])


# ------------------------------------------------------- dispatch by opcode

def test_elementwise_dispatch_matches_named_entry_points():
    ah, al, bh, bl = _operands("mixed", 4096, 401)
    named = {
        "add": oracle.add22(ah, al, bh, bl),
        "sub": oracle.sub22(ah, al, bh, bl),
        "mul": oracle.mul22(ah, al, bh, bl),
        "mul_dekker": oracle.mul22(ah, al, bh, bl, dekker=True),
        "div": oracle.div22(ah, al, bh, bl),
    }
    for op, (h, l) in named.items():
        rh, rl = oracle.elementwise(op, ah, al, bh, bl)
        assert same_bits(rh, h) and same_bits(rl, l)
