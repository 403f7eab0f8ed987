"""GPU parity of polynomial evaluation (Horner's rule in binary32,
compensated Horner, float-float Horner): every result bit for bit against
the oracle, whose operation sequences the kernels follow.

Covered: degrees 0, 1, 7, 25 and 64; point counts with ragged tails
(1 .. 4099, 2^16 + 3); binary32 and float-float coefficients and points
(null low words); unaligned planes (the one-point-per-lane kernel); results
written in place over the points; the benchmark's workload (the expanded
(x - 1)^25 at 2^26 points), checked on every point; and the accuracy of the
three forms against the condition number of (x - 1)^n near its root, exact
errors in Fraction.
"""
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import ff_value, frac, mismatch_report, same_bits

pytestmark = pytest.mark.gpu

ALGOS = ["f32", "comp", "ff"]


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu(algo, coef, x, ff_points=True, out=None):
    ff = _ff()
    if algo == "f32":
        r = ff.ff_horner_f32(coef, x, out=out)
    elif algo == "comp":
        r = ff.ff_horner_comp(coef, x, out=out)
    else:
        r = ff.ff_horner_ff(coef, x, out=out, ff_points=ff_points)
    torch.cuda.synchronize()
    return r.cpu().numpy()


def _want(algo, coef, x):
    """Oracle results; coef and x numpy, binary32 (1-D) or float-float (2, .)."""
    if algo == "f32":
        return oracle.horner_f32(coef, x)
    if algo == "comp":
        return oracle.horner_comp(coef, x)
    ch, cl = (coef[0], coef[1]) if coef.ndim == 2 else (coef, np.zeros_like(coef))
    xh, xl = (x[0], x[1]) if x.ndim == 2 else (x, np.zeros_like(x))
    return np.stack(oracle.horner_ff(ch, cl, xh, xl))


def _check(got, want, label):
    got, want = np.atleast_2d(got), np.atleast_2d(want)
    for w in range(want.shape[0]):
        assert same_bits(got[w], want[w]), f"{label} word {w}:\n{mismatch_report(got[w], want[w])}"


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("degree", [0, 1, 7, 25, 64])
def test_bitexact_random_polynomials(algo, degree):
    _announce(f"[gpu] horner {algo} degree {degree}")
    coef = fi.random_poly(degree, 1500 + degree)
    for n in (1, 3, 5, 1027, 4099, (1 << 16) + 3):
        x = fi.horner_points(n, 1600 + n, -1.3, 1.3)
        got = _gpu(algo, coef.cuda(), x.cuda(), ff_points=False)
        _check(got, _want(algo, coef.numpy(), x.numpy()), f"{algo} degree {degree} n={n}")


@pytest.mark.parametrize("coef_ff,points_ff", [(True, True), (True, False), (False, True)])
def test_float_float_inputs(coef_ff, points_ff):
    degree, n = 19, 10007
    _announce(f"[gpu] horner ff: float-float coefficients {coef_ff}, points {points_ff}")
    coef = fi.random_poly(degree, 1701, ff=coef_ff)
    x = fi.horner_points(n, 1702, -1.1, 1.1).double() + \
        1e-9 * fi.horner_points(n, 1703, -1, 1).double()
    x = fi.split_f64(x) if points_ff else x.float()
    got = _gpu("ff", coef.cuda(), x.cuda(), ff_points=points_ff)
    _check(got, _want("ff", coef.numpy(), x.numpy()), f"coef_ff={coef_ff} points_ff={points_ff}")


@pytest.mark.parametrize("algo", ALGOS)
def test_unaligned_and_in_place(algo):
    _announce(f"[gpu] horner {algo}: unaligned planes, in place")
    ff = _ff()
    degree, n = 11, 4103
    coef = fi.random_poly(degree, 1801, ff=(algo == "ff"))
    cd = coef.cuda()
    base = fi.horner_points(n + 1, 1802, -1.2, 1.2)
    want = _want(algo, coef.numpy(), base[1:].numpy())
    # offset 1: 4-byte aligned only, the one-point-per-lane kernel
    xd = base.cuda()[1:]
    if algo == "ff":
        out = ff.ff_zeros((n + 1,), device="cuda")[:, 1:]
        got = _gpu("ff", cd, xd, ff_points=False, out=out)
    else:
        got = _gpu(algo, cd, xd, out=torch.zeros(n + 1, device="cuda")[1:])
    _check(got, want, "unaligned")
    # in place: the results overwrite the points
    if algo == "ff":
        pts = torch.stack([base[1:], torch.zeros(n)]).cuda()
        want_ff = _want("ff", coef.numpy(), pts.cpu().numpy())
        ff.ff_horner_ff(cd, pts, out=pts)
        torch.cuda.synchronize()
        _check(pts.cpu().numpy(), want_ff, "in place")
    else:
        pts = base[1:].clone().cuda()
        got = _gpu(algo, cd, pts, out=pts)
        _check(got, want, "in place")


@pytest.mark.parametrize("algo", ALGOS)
def test_benchmark_workload_every_point(algo):
    # the benchmark's launch: (x - 1)^25 expanded, 2^26 points in [0.75, 1.25];
    # every point against the oracle, in pieces of 2^22
    n, degree = 1 << 26, 25
    _announce(f"[gpu] horner {algo} at the benchmark size (2^26 points, degree 25)")
    coef = fi.binomial_poly(degree)
    x = fi.horner_points(n, 115041, 0.75, 1.25, device="cuda")
    got = _gpu(algo, coef.cuda(), x, ff_points=False)
    xs = x.cpu().numpy()
    piece = 1 << 22
    for lo in range(0, n, piece):
        _check(got[..., lo:lo + piece], _want(algo, coef.numpy(), xs[lo:lo + piece]),
               f"points {lo}..{lo + piece}")
    del x
    torch.cuda.empty_cache()


def test_accuracy_against_condition_number():
    # (x - 1)^n near its root: the relative error of Horner grows like
    # cond * u, CompHorner's like u + cond * u^2, and the float-float
    # result's like cond * 2^-44 -- measured exactly on the GPU results
    _announce("[gpu] horner accuracy against the condition number")
    U = Fraction(1, 1 << 24)
    rows = []
    for n, width in ((5, 2.0 ** -3), (9, 2.0 ** -4)):
        coef = fi.binomial_poly(n)
        x = fi.horner_points(2048, 1900 + n, 1 - width, 1 + width)
        xd, cd = x.cuda(), coef.cuda()
        h = _gpu("f32", cd, xd)
        c = _gpu("comp", cd, xd)
        fh = _gpu("ff", cd, xd, ff_points=False)
        buckets = {}
        for k, xv in enumerate(x.numpy()):
            xk = frac(xv)
            exact = (xk - 1) ** n
            if exact == 0:
                continue
            cond = (1 + abs(xk)) ** n / abs(exact)
            rel = [abs(frac(h[k]) - exact) / abs(exact), abs(frac(c[k]) - exact) / abs(exact),
                   abs(ff_value(fh[0][k], fh[1][k]) - exact) / abs(exact)]
            gam = 2 * n * U / (1 - 2 * n * U)
            assert rel[1] <= U + gam * gam * cond
            b = int(np.floor(np.log2(float(cond)) / 8) * 8)
            cur = buckets.setdefault(b, [Fraction(0)] * 3)
            buckets[b] = [max(a, r) for a, r in zip(cur, rel)]
        for b in sorted(buckets):
            lg = [float(np.log2(float(r))) if r > 0 else None for r in buckets[b]]
            rows.append((n, b, lg))
    for n, b, lg in rows:
        fmt = ["exact" if v is None else f"2^{v:.1f}" for v in lg]
        _announce(f"  n={n} cond 2^[{b},{b + 8}): max rel error Horner {fmt[0]}, "
                  f"CompHorner {fmt[1]}, ff Horner {fmt[2]}")
