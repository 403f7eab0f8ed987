"""GPU parity of the batched float-float dot products.

Reductions have many correct results (the accumulation order is the
implementation's), so each result is compared with the EXACT dot product
computed by the oracle's long accumulator:
  * a rigorous bound: |err| <= D * 2^-44 * sum|x_i y_i|, D the depth of the
    accumulation tree (each Add22 errs by at most 2^-44 (|a| + |b|) on
    normalised inputs, section 4.1 Add22 theorem);
  * the stated accuracy target: normwise |err| / sum|x_i y_i| <= 2^-44;
  * closed forms (single terms, integer data) exactly;
  * bitwise run-to-run reproducibility for a fixed launch configuration.
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

TWO_M44 = Fraction(1, 1 << 44)


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def tree_depth(lengths, cfg, default=(256, 32)):
    """Longest chain of Add22s behind a result: a thread's `unroll` terms in
    order, the 6-level butterfly, the wavefronts of the workgroup in order,
    then the chunk partials lane-strided, a second butterfly, and slack.
    `default` is the entry point's (block, unroll) for zero fields."""
    block, chunk, _, unroll = cfg
    block = block or default[0]
    if not unroll:
        unroll = chunk // block if chunk else default[1]
    chunk = block * unroll
    nch = max(1, max(math.ceil(int(n) / chunk) for n in lengths))
    return unroll + 6 + block // 64 + math.ceil(nch / 64) + 6 + 2


def check_against_exact(x, y, offs, got, cfg, label, target=TWO_M44):
    x, y, offs = (t.cpu().numpy() for t in (x, y, offs))
    got = got.cpu().numpy()
    exact = oracle.exact_dot_batched(x, y, offs)
    absum = oracle.exact_dot_batched(np.abs(x), np.abs(y), offs)
    lengths = np.diff(offs)
    depth = tree_depth(lengths, cfg)
    worst = -math.inf
    for v in range(len(exact)):
        err = abs(frac(got[0, v]) + frac(got[1, v]) - exact[v])
        if absum[v] == 0:
            assert err == 0, (label, v)
            continue
        assert err <= depth * TWO_M44 * absum[v] * (1 + Fraction(1, 1 << 20)), (label, v, float(err / absum[v]))
        assert err <= target * absum[v], (label, v, float(err / absum[v]))
        if err:
            worst = max(worst, math.log2(err / absum[v]))
    return worst


CFGS = [(0, 0, 0, 0), (64, 256, 0, 4), (128, 1024, 0, 0), (256, 0, 0, 2), (512, 16384, 0, 32),
        (0, 2048, 0, 0)]


@pytest.mark.parametrize("cfg", CFGS, ids=[str(c) for c in CFGS])
def test_batched_dot_uneven_lengths(cfg):
    _announce(f"[gpu] dot batched cfg={cfg}")
    x, y, offs = fi.batched_dot(115003, nvec=300, max_total=1 << 21)
    # add empty and tiny vectors at both ends
    lens = torch.diff(offs)
    lens = torch.cat([torch.tensor([0, 1, 2, 3, 5, 0]), lens, torch.tensor([7, 0, 1])])
    offs = torch.zeros(lens.numel() + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(lens, 0)
    x = fi.scaled_normal(int(offs[-1]), 115004)
    y = fi.scaled_normal(int(offs[-1]), 115005)
    ff = _ff()
    got = ff.ff_dot_batched(x.cuda(), y.cuda(), offs.cuda(), cfg=cfg)
    again = ff.ff_dot_batched(x.cuda(), y.cuda(), offs.cuda(), cfg=cfg)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), again.view(torch.int32)), "not reproducible"
    worst = check_against_exact(x, y, offs, got, cfg, f"cfg={cfg}")
    _announce(f"  worst normwise log2 error {worst:.1f}")


def test_single_terms_give_the_exact_product_pair():
    n = 5000
    x = fi.random_f32(n, 51, -30, 30)
    y = fi.random_f32(n, 52, -30, 30)
    offs = torch.arange(n + 1, dtype=torch.int64)
    got = _ff().ff_dot_batched(x.cuda(), y.cuda(), offs.cuda()).cpu().numpy()
    xn, yn = x.numpy(), y.numpy()
    p64 = xn.astype(np.float64) * yn.astype(np.float64)
    assert np.array_equal(got[0], p64.astype(np.float32))
    assert np.all(got[0].astype(np.float64) + got[1].astype(np.float64) == p64)


def test_integer_data_is_exact():
    rng = np.random.default_rng(7)
    lens = rng.integers(1, 40000, 64)
    offs = np.zeros(65, np.int64)
    offs[1:] = np.cumsum(lens)
    x = rng.integers(-2 ** 11, 2 ** 11, offs[-1]).astype(np.float32)
    y = rng.integers(-2 ** 11, 2 ** 11, offs[-1]).astype(np.float32)
    got = _ff().ff_dot_batched(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                               torch.from_numpy(offs).cuda()).cpu().numpy()
    for v in range(64):
        s, e = offs[v], offs[v + 1]
        want = int(np.dot(x[s:e].astype(np.int64), y[s:e].astype(np.int64)))
        assert frac(got[0, v]) + frac(got[1, v]) == want


def test_unaligned_inputs():
    x, y, offs = fi.batched_dot(99, nvec=40, max_total=200000)
    xb = torch.cat([torch.zeros(1), x]).cuda()[1:]
    yb = torch.cat([torch.zeros(3), y]).cuda()[3:]
    got = _ff().ff_dot_batched(xb, yb, offs.cuda(), cfg=(256, 1024, 0, 4))
    check_against_exact(x, y, offs, got, (256, 1024, 0, 4), "unaligned")


def test_empty_batch_and_empty_vectors():
    ff = _ff()
    x = torch.zeros(0, device="cuda")
    out = ff.ff_dot_batched(x, x, torch.zeros(1, dtype=torch.int64, device="cuda"))
    assert out.shape == (2, 0)
    out = ff.ff_dot_batched(x, x, torch.zeros(5, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0


def test_ff_inputs_batched():
    _announce("[gpu] dot ff batched")
    a = fi.gaussian_ff((1 << 20,), 61)
    b = fi.gaussian_ff((1 << 20,), 62)
    lens = torch.tensor([1, 17, 1000, 65536, 3, 0, 400000, 0])
    lens[-1] = (1 << 20) - int(lens.sum())
    offs = torch.zeros(lens.numel() + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(lens, 0)
    got = _ff().ff_dot_ff_batched(a.cuda(), b.cuda(), offs.cuda()).cpu().numpy()
    an, bn, on = a.numpy(), b.numpy(), offs.numpy()
    for v in range(lens.numel()):
        s, e = on[v], on[v + 1]
        exact = oracle.exact_dot_ff(an[0, s:e], an[1, s:e], bn[0, s:e], bn[1, s:e])
        absum = oracle.exact_dot_ff(np.abs(an[0, s:e]), np.sign(an[0, s:e]) * an[1, s:e],
                                    np.abs(bn[0, s:e]), np.sign(bn[0, s:e]) * bn[1, s:e])
        err = abs(frac(got[0, v]) + frac(got[1, v]) - exact)
        assert err <= TWO_M44 * absum, (v, float(err / absum) if absum else err)


def test_full_batch_4096_vectors():
    # The uneven batch at full size: 4096 vectors, lengths floor(2^U),
    # U ~ U[6, 20] (about 442 M elements); every vector checked exactly.
    _announce("[gpu] dot batched full size (4096 vectors)")
    x, y, offs = fi.batched_dot(115003, device="cuda")
    got = _ff().ff_dot_batched(x, y, offs)
    again = _ff().ff_dot_batched(x, y, offs)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), again.view(torch.int32))
    _announce(f"  total elements {int(offs[-1])}")
    worst = check_against_exact(x, y, offs, got, (0, 0, 0, 0), "full")
    _announce(f"  worst normwise log2 error {worst:.1f}")
    del x, y
    torch.cuda.empty_cache()


def _check_exact(got, exact, absum, depth, label):
    worst = -math.inf
    for v in range(len(exact)):
        err = abs(frac(got[0, v]) + frac(got[1, v]) - exact[v])
        if absum[v] == 0:
            assert err == 0, (label, v)
            continue
        assert err <= depth * TWO_M44 * absum[v] * (1 + Fraction(1, 1 << 20)), (label, v)
        assert err <= TWO_M44 * absum[v], (label, v, float(err / absum[v]))
        if err:
            worst = max(worst, math.log2(err / absum[v]))
    return worst


def test_family_full_batch_as_benchmarked():
    """The other entry points of the family on the 4096-vector batch, each at
    its default shape, as the benchmark launches them: the float-float dot of
    the values as (2, N) float-float vectors (zero low words, so its exact
    value is the binary32 dot's), and the binary32 and float-float sums;
    every vector against the exact value."""
    _announce("[gpu] dot family at full size (4096 vectors)")
    ff = _ff()
    x, y, offs = fi.batched_dot(115003, device="cuda")
    xf = torch.stack([x, torch.zeros_like(x)])
    yf = torch.stack([y, torch.zeros_like(y)])
    dot_ff = ff.ff_dot_ff_batched(xf, yf, offs).cpu().numpy()
    del yf
    sum_f32 = ff.ff_sum_batched(x, offs).cpu().numpy()
    sum_ff = ff.ff_sum_ff_batched(xf, offs).cpu().numpy()
    del xf
    xn, yn, on = x.cpu().numpy(), y.cpu().numpy(), offs.cpu().numpy()
    del x, y
    torch.cuda.empty_cache()
    depth = tree_depth(np.diff(on), (0, 0, 0, 0))
    _announce("  exact dots")
    exact = oracle.exact_dot_batched(xn, yn, on)
    absum = oracle.exact_dot_batched(np.abs(xn), np.abs(yn), on)
    w = _check_exact(dot_ff, exact, absum, depth, "ff_dot_ff_batched")
    _announce(f"  ff-input dot worst normwise log2 error {w:.1f}")
    del yn
    _announce("  exact sums")
    ones = np.ones_like(xn)
    exact = oracle.exact_dot_batched(xn, ones, on)
    absum = oracle.exact_dot_batched(np.abs(xn), ones, on)
    for got, label in ((sum_f32, "ff_sum_batched"), (sum_ff, "ff_sum_ff_batched")):
        w = _check_exact(got, exact, absum, depth, label)
        _announce(f"  {label} worst normwise log2 error {w:.1f}")


def test_batched_sums_binary32_and_float_float():
    _announce("[gpu] sum batched")
    ff = _ff()
    x, _, offs = fi.batched_dot(7, nvec=200, max_total=1 << 21)
    got = ff.ff_sum_batched(x.cuda(), offs.cuda()).cpu().numpy()
    xn, on = x.numpy(), offs.numpy()
    ones = np.ones_like(xn)
    exact = oracle.exact_dot_batched(xn, ones, on)
    absum = oracle.exact_dot_batched(np.abs(xn), ones, on)
    for v in range(200):
        err = abs(frac(got[0, v]) + frac(got[1, v]) - exact[v])
        assert err <= TWO_M44 * absum[v]
    a = fi.gaussian_ff((1 << 20,), 8)
    lens = torch.tensor([5, 1000, 300000, 0, 12345])
    lens = torch.cat([lens, torch.tensor([(1 << 20) - int(lens.sum())])])
    offs = torch.zeros(lens.numel() + 1, dtype=torch.int64)
    offs[1:] = torch.cumsum(lens, 0)
    got = ff.ff_sum_ff_batched(a.cuda(), offs.cuda()).cpu().numpy()
    an, on = a.numpy(), offs.numpy()
    one = np.ones(1 << 20, np.float32)
    zero = np.zeros(1 << 20, np.float32)
    for v in range(lens.numel()):
        s, e = on[v], on[v + 1]
        exact = oracle.exact_dot_ff(an[0, s:e], an[1, s:e], one[s:e], zero[s:e])
        absum = oracle.exact_dot_ff(np.abs(an[0, s:e]), np.sign(an[0, s:e]) * an[1, s:e],
                                    one[s:e], zero[s:e])
        err = abs(frac(got[0, v]) + frac(got[1, v]) - exact)
        assert err <= TWO_M44 * absum


def test_autotuner_returns_a_valid_fast_shape(tmp_path, monkeypatch):
    _announce("[gpu] dot autotune")
    monkeypatch.setenv("FF_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_cs_0603115_amd import autotune
    autotune._MEMO = None
    x, y, offs = fi.batched_dot(115003, nvec=512, max_total=1 << 24, device="cuda")
    cfg = autotune.dot_cfg(x, y, offs)
    assert cfg[0] in (64, 128, 256, 512) and cfg[3] in (4, 8, 16, 32)
    assert cfg[1] == cfg[0] * cfg[3] and cfg[2] == 0
    assert (tmp_path / "tune.json").exists()
    autotune._MEMO = None
    assert autotune.dot_cfg(x, y, offs, search=False) == cfg      # served from the file
    got = _ff().ff_dot_batched(x, y, offs, cfg=cfg)
    check_against_exact(x, y, offs, got, cfg, "tuned")


def test_out_of_range_offsets_are_clamped():
    # offsets outside [0, total] are clamped on the device (no access outside
    # the arrays): vector 0 = [0, total), vector 1 = [total, total) empty,
    # vector 2 = [0, 10)
    ff = _ff()
    x, y, _ = fi.batched_dot(61, nvec=2, log2_max=12)
    total = x.numel()
    offs = torch.tensor([0, total + 100, -5, 10], dtype=torch.int64)
    got = ff.ff_dot_batched(x.cuda(), y.cuda(), offs.cuda()).cpu().numpy()
    xn, yn = x.numpy(), y.numpy()
    ex0 = oracle.exact_dot(xn, yn)
    ab0 = oracle.exact_dot(np.abs(xn), np.abs(yn))
    assert abs(frac(got[0, 0]) + frac(got[1, 0]) - ex0) <= TWO_M44 * ab0
    assert got[0, 1] == 0 and got[1, 1] == 0
    ex2 = oracle.exact_dot(xn[:10], yn[:10])
    assert abs(frac(got[0, 2]) + frac(got[1, 2]) - ex2) <= TWO_M44 * oracle.exact_dot(
        np.abs(xn[:10]), np.abs(yn[:10]))
