"""GPU parity of the compensated batched reductions Dot2 / Sum2 (Ogita,
Rump and Oishi 2005; the paper's named future work, section 7).

The accumulation order is the implementation's, so results are compared
with the exact values (the oracle's long accumulator) under the algorithm's
published bound, with a factor 2 for the tree-shaped order:
    |out_hi - exact| <= u |exact| + 2 gamma_n^2 sum |terms|,
u = 2^-24, gamma_n = n u / (1 - n u), n the vector's length; out_hi must be
the rounding of out_hi + out_lo.  Closed forms (single terms, integer data,
empty vectors) are exact; results are bitwise reproducible.  On
ill-conditioned dot products the sequential oracle Dot2 meets the same bound,
and the measured errors of Dot2 and of float-float accumulation are printed
(run with -s).
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import frac

pytestmark = pytest.mark.gpu

U = Fraction(1, 1 << 24)


def gamma(k):
    return k * U / (1 - k * U)


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def check(x, y, offs, got, label):
    """got (2, nvec) against the exact dots (y None: sums)."""
    xn = x.cpu().numpy()
    yn = np.ones_like(xn) if y is None else y.cpu().numpy()
    offs = offs.cpu().numpy()
    got = got.cpu().numpy()
    exact = oracle.exact_dot_batched(xn, yn, offs)
    absum = oracle.exact_dot_batched(np.abs(xn), np.abs(yn), offs)
    worst = 0.0
    for v in range(len(exact)):
        n = int(offs[v + 1] - offs[v])
        hi, lo = got[0, v], got[1, v]
        assert np.float32(hi + lo) == hi, (label, v)                  # normalised pair
        err = abs(frac(hi) - exact[v])
        if n == 0:
            assert hi == 0 and lo == 0
            continue
        assert err <= U * abs(exact[v]) + 2 * gamma(n) ** 2 * absum[v], (label, v, n)
        if exact[v] != 0:
            worst = max(worst, float(err / abs(exact[v])))
    return worst


@pytest.mark.parametrize("cfg", [(0, 0, 0, 0), (64, 256, 0, 4), (512, 4096, 0, 8), (256, 8192, 0, 32)])
def test_dot2_and_sum2_uneven_lengths(cfg):
    ff = _ff()
    x, y, offs = fi.batched_dot(31, nvec=300, log2_max=15, device="cuda")
    check(x, y, offs, ff.ff_dot2_batched(x, y, offs, cfg=cfg), f"dot2 {cfg}")
    check(x, None, offs, ff.ff_sum2_batched(x, offs, cfg=cfg), f"sum2 {cfg}")


def test_closed_forms_and_edges():
    ff = _ff()
    # single terms: Add12 of the exact TwoProduct pair, i.e. the pair itself
    x = fi.random_f32(1000, 41, -40, 40, device="cuda")
    y = fi.random_f32(1000, 42, -40, 40, device="cuda")
    offs = torch.arange(1001, dtype=torch.int64, device="cuda")
    r = ff.ff_dot2_batched(x, y, offs).cpu().numpy()
    h, l = oracle.mul12(x.cpu().numpy(), y.cpu().numpy())
    assert np.array_equal(r[0], h) and np.array_equal(r[1], l)
    # integer data with representable partial sums: exact
    rng = np.random.default_rng(5)
    xi = torch.from_numpy(rng.integers(-1000, 1000, 50000).astype(np.float32)).cuda()
    yi = torch.from_numpy(rng.integers(-1000, 1000, 50000).astype(np.float32)).cuda()
    offs = torch.tensor([0, 10, 10, 4097, 50000], dtype=torch.int64, device="cuda")
    r = ff.ff_dot2_batched(xi, yi, offs).cpu().numpy()
    s = ff.ff_sum2_batched(xi, offs).cpu().numpy()
    o = offs.cpu().numpy()
    a, b = xi.cpu().numpy().astype(np.int64), yi.cpu().numpy().astype(np.int64)
    for v in range(4):
        want = int((a[o[v]:o[v + 1]] * b[o[v]:o[v + 1]]).sum())
        assert frac(r[0, v]) + frac(r[1, v]) == want
        assert frac(s[0, v]) + frac(s[1, v]) == int(a[o[v]:o[v + 1]].sum())
    assert r[0, 1] == 0 and r[1, 1] == 0                    # empty vector
    # unaligned planes take the element path; repeat runs are identical
    x, y, offs = fi.batched_dot(43, nvec=40, log2_max=12, device="cuda")
    xu, yu = torch.empty(x.numel() + 1, device="cuda"), torch.empty(y.numel() + 1, device="cuda")
    xu[1:], yu[1:] = x, y
    check(xu[1:], yu[1:], offs, ff.ff_dot2_batched(xu[1:], yu[1:], offs), "unaligned")
    r1 = ff.ff_dot2_batched(x, y, offs).clone()
    r2 = ff.ff_dot2_batched(x, y, offs)
    assert torch.equal(r1.view(torch.int32), r2.view(torch.int32))


def test_full_batch_4096_vectors():
    ff = _ff()
    _announce("[gpu] dot2 / sum2: 4096 vectors, lengths floor(2^U[6,20])")
    x, y, offs = fi.batched_dot(115003, device="cuda")
    w_dot = check(x, y, offs, ff.ff_dot2_batched(x, y, offs), "dot2 full")
    w_sum = check(x, None, offs, ff.ff_sum2_batched(x, offs), "sum2 full")
    _announce(f"  worst relative error: dot2 {w_dot:.3g}, sum2 {w_sum:.3g}")


def test_ill_conditioned_dots_against_ff_accumulation():
    # 24 vectors with condition numbers 2^16 .. 2^60: Dot2 and the sequential
    # oracle Dot2 meet the bound; float-float accumulation is printed beside
    ff = _ff()
    xs, ys, lens = [], [], []
    for k in range(24):
        n = 1000 + 400 * k
        x, y = fi.ill_conditioned_dot(n, 500 + k, 16 + 2 * k)
        xs.append(x), ys.append(y), lens.append(n)
    x = torch.cat(xs).cuda()
    y = torch.cat(ys).cuda()
    offs = torch.tensor(np.concatenate([[0], np.cumsum(lens)]), dtype=torch.int64, device="cuda")
    d2 = ff.ff_dot2_batched(x, y, offs)
    fd = ff.ff_dot_batched(x, y, offs)
    check(x, y, offs, d2, "dot2 ill-conditioned")
    xn, yn, on = x.cpu().numpy(), y.cpu().numpy(), offs.cpu().numpy()
    exact = oracle.exact_dot_batched(xn, yn, on)
    absum = oracle.exact_dot_batched(np.abs(xn), np.abs(yn), on)
    p, s = oracle.dot2_batched(xn, yn, on)
    d2n, fdn = d2.cpu().numpy(), fd.cpu().numpy()
    for v in range(24):
        n = lens[v]
        seq = frac(np.float32(p[v] + s[v]))
        assert abs(seq - exact[v]) <= U * abs(exact[v]) + gamma(n) ** 2 * absum[v]
        cond = float(2 * absum[v] / abs(exact[v]))
        e_d2 = float(abs(frac(d2n[0, v]) - exact[v]) / abs(exact[v]))
        e_ff = float(abs(frac(fdn[0, v]) + frac(fdn[1, v]) - exact[v]) / abs(exact[v]))
        _announce(f"  cond 2^{math.log2(cond):5.1f}: rel error Dot2 {e_d2:.2e}  "
                  f"float-float {e_ff:.2e}")
