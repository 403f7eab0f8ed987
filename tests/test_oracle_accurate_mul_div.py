"""Pins of the oracle's FMA-based float-float product and reciprocal-based
division (the DWTimesDW3 and DWDivDW3 algorithms of Joldes, Muller and
Popescu, ACM TOMS 2017), alternatives to the paper's Mul22 (section 4.1,
Mul22 theorem, bound 2^-44) and to Dekker's division, with smaller published
bounds: 5u^2 and 9.8u^2 relative, u = 2^-24.

* zero low words reduce the product to the exact TwoProd pair (closed form);
* a * 1 = a and a / 1 = a bit for bit; sign symmetry and power-of-two
  scaling, bit for bit;
* hand-derived cases (golden file): a rounding tie that only the al*bl term
  decides; 1/3; 1/(1 + 2^-24), which goes through the divisor's low word;
  1/(3 + 2^-23), whose Newton residual needs a low word of its own;
* the published relative bounds, measured exactly with Fraction on random,
  near, cancellation and exponent-gap inputs; quotients of exactly held
  products return the factor within the bound;
* the error measurement of the oracle for divisions against Fraction.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac, same_bits
from test_oracle_operators import FAMILIES, _assert_normalised, _operands

U = Fraction(1, 1 << 24)
MUL_BOUND = 5 * U * U
DIV_BOUND = Fraction(98, 10) * U * U
TINY = Fraction(2) ** -96       # below: error words near the subnormal range

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_cases.txt")


def _np(t):
    return t.cpu().numpy()


# ------------------------------------------------------------------ product

def test_mul_zero_low_words_is_the_exact_product_pair():
    ah, _, bh, _ = _operands("random", 4096, 1201)
    z = np.zeros_like(ah)
    rh, rl = oracle.mul22_accurate(ah, z, bh, z)
    assert same_bits(rh, (ah * bh).astype(np.float32))
    for i in range(0, ah.size, 7):
        assert ff_value(rh[i], rl[i]) == frac(ah[i]) * frac(bh[i]), i
    _assert_normalised(rh[:512], rl[:512])


def test_mul_identities():
    ah, al, _, _ = _operands("random", 4096, 1211)
    one, z = np.ones_like(ah), np.zeros_like(ah)
    rh, rl = oracle.mul22_accurate(ah, al, one, z)
    assert same_bits(rh, ah) and same_bits(rl, al)
    rh, rl = oracle.mul22_accurate(one, z, ah, al)
    assert same_bits(rh, ah) and same_bits(rl, al)


@pytest.mark.parametrize("kind", ["random", "mixed"])
def test_mul_sign_symmetry_and_scaling(kind):
    ah, al, bh, bl = _operands(kind, 4096, 1221)
    r1 = oracle.mul22_accurate(ah, al, bh, bl)
    r2 = oracle.mul22_accurate(-ah, -al, bh, bl)
    for w in (0, 1):
        assert np.array_equal(r1[w], -r2[w])
        nz = r1[w] != 0
        assert same_bits(r1[w][nz], -r2[w][nz])
    for k in (-9, 13):
        s = np.float32(2.0 ** k)
        qh, ql = oracle.mul22_accurate(ah * s, al * s, bh, bl)
        assert same_bits(qh, r1[0] * s) and same_bits(ql, r1[1] * s)


@pytest.mark.parametrize("kind", FAMILIES)
def test_mul_relative_error_bound(kind):
    ah, al, bh, bl = _operands(kind, 3000, 1231)
    rh, rl = oracle.mul22_accurate(ah, al, bh, bl)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) * ff_value(bh[i], bl[i])
        if abs(exact) < TINY:
            continue
        err = abs(ff_value(rh[i], rl[i]) - exact)
        assert err <= MUL_BOUND * abs(exact), (kind, i)
    _assert_normalised(rh[:512], rl[:512])


# ----------------------------------------------------------------- division

def test_div_identities():
    ah, al, _, _ = _operands("random", 4096, 1301)
    one, z = np.ones_like(ah), np.zeros_like(ah)
    rh, rl = oracle.div22_accurate(ah, al, one, z)
    assert same_bits(rh, ah) and same_bits(rl, al)


@pytest.mark.parametrize("kind", ["random", "mixed"])
def test_div_sign_symmetry_and_scaling(kind):
    ah, al, bh, bl = _operands(kind, 4096, 1311)
    r1 = oracle.div22_accurate(ah, al, bh, bl)
    for a_sign, b_sign in ((-1, 1), (1, -1)):
        sa, sb = np.float32(a_sign), np.float32(b_sign)
        r2 = oracle.div22_accurate(ah * sa, al * sa, bh * sb, bl * sb)
        for w in (0, 1):
            assert np.array_equal(r1[w], -r2[w])
            nz = r1[w] != 0
            assert same_bits(r1[w][nz], -r2[w][nz])
    for k in (-11, 5):
        s = np.float32(2.0 ** k)
        qh, ql = oracle.div22_accurate(ah * s, al * s, bh, bl)
        assert same_bits(qh, r1[0] * s) and same_bits(ql, r1[1] * s)
        qh, ql = oracle.div22_accurate(ah, al, bh * s, bl * s)
        assert same_bits(qh, r1[0] / s) and same_bits(ql, r1[1] / s)


@pytest.mark.parametrize("kind", FAMILIES)
def test_div_relative_error_bound(kind):
    ah, al, bh, bl = _operands(kind, 3000, 1321)
    rh, rl = oracle.div22_accurate(ah, al, bh, bl)
    for i in range(ah.size):
        exact = ff_value(ah[i], al[i]) / ff_value(bh[i], bl[i])
        if abs(exact) < TINY:
            continue
        err = abs(ff_value(rh[i], rl[i]) - exact)
        assert err <= DIV_BOUND * abs(exact), (kind, i)
    _assert_normalised(rh[:512], rl[:512])


def test_div_of_an_exact_product_returns_the_factor():
    q = _np(fi.random_f32(2048, 1331, -10, 10))
    b = _np(fi.random_f32(2048, 1332, -10, 10))
    z = np.zeros_like(q)
    th, tl = oracle.mul12(q, b)            # q*b held exactly (Mul12 theorem)
    rh, rl = oracle.div22_accurate(th, tl, b, z)
    for i in range(q.size):
        assert abs(ff_value(rh[i], rl[i]) - frac(q[i])) <= DIV_BOUND * abs(frac(q[i])), i


# ------------------------------------------------------------- hand cases

def _hand_rows(ops):
    with open(_GOLD) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                cols = [c.strip() for c in line.split("|")]
                if cols[0] in ops:
                    yield cols


def _f(word):
    return np.array([int(word, 16)], np.uint32).view(np.float32)


def test_hand_derived_cases():
    rows = list(_hand_rows(("mul_accurate", "div_accurate")))
    assert len(rows) == 4
    for op, ins, outs, why in rows:
        a = [_f(w) for w in ins.split()]
        fn = oracle.mul22_accurate if op == "mul_accurate" else oracle.div22_accurate
        got = fn(*a)
        want = [int(w, 16) for w in outs.split()]
        assert [int(g.view(np.uint32)[0]) for g in got] == want, (op, why)


# ------------------------------------------------------- error measurement

@pytest.mark.parametrize("op", ["div22", "div22_accurate", "mul22_accurate"])
def test_ff_errors_against_fractions(op):
    ah, al, bh, bl = _operands("mixed", 500, 1341)
    fn = {"div22": oracle.div22, "div22_accurate": oracle.div22_accurate,
          "mul22_accurate": oracle.mul22_accurate}[op]
    rh, rl = fn(ah, al, bh, bl)
    rel, ratio = oracle.ff_errors(op, ah, al, bh, bl, rh, rl)
    bound = {"div22": Fraction(1, 1 << 44), "div22_accurate": DIV_BOUND,
             "mul22_accurate": MUL_BOUND}[op]
    for i in range(ah.size):
        a, b = ff_value(ah[i], al[i]), ff_value(bh[i], bl[i])
        exact = a / b if op.startswith("div") else a * b
        want = abs(ff_value(rh[i], rl[i]) - exact) / abs(exact)
        assert rel[i] == pytest.approx(float(want), rel=1e-12, abs=0), i
        assert ratio[i] == pytest.approx(float(want / bound), rel=1e-12, abs=0), i


def test_elementwise_dispatch():
    ah, al, bh, bl = _operands("mixed", 1000, 1351)
    for op, fn in (("mul_accurate", oracle.mul22_accurate),
                   ("div_accurate", oracle.div22_accurate)):
        a = oracle.elementwise(op, ah, al, bh, bl)
        b = fn(ah, al, bh, bl)
        assert same_bits(a[0], b[0]) and same_bits(a[1], b[1])
