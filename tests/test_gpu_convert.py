"""GPU parity of the binary64 <-> float-float conversions: every word bit
for bit against the oracle, on wide exponent ranges (low words down to the
subnormal range, signed zeros), ragged sizes, planes aligned to 4 or 8 bytes
only, a 2^24-element run and every element at the benchmark's 2^28; infinities, NaN and values beyond the binary32
range on 16-byte aligned and unaligned planes; the Python short names are
the same entry points."""
import sys

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import mismatch_report, same_bits

pytestmark = pytest.mark.gpu


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _f64(n, seed, emin=-120, emax=120):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    x = np.ldexp(m, rng.integers(emin, emax + 1, n))
    x[:: 97] = 0.0
    x[1:: 97] = -0.0
    return x


@pytest.mark.parametrize("n", [1, 3, 5, 1027, 4099, (1 << 16) + 7, 1 << 24])
def test_from_and_to_f64_bitexact(n):
    print(f"[gpu] conversions n={n}", file=sys.stderr, flush=True)
    ff = _ff()
    x = _f64(n, 2100 + n % 1000)
    got = ff.ff_from_f64(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    hi, lo = oracle.from_f64(x)
    assert same_bits(g[0], hi), mismatch_report(g[0], hi)
    assert same_bits(g[1], lo), mismatch_report(g[1], lo)
    pairs = fi.random_ff(n, 2200 + n % 1000, -100, 100, max_gap=40)
    back = ff.ff_to_f64(pairs.cuda())
    torch.cuda.synchronize()
    want = oracle.to_f64(pairs[0].numpy(), pairs[1].numpy())
    assert np.array_equal(back.cpu().numpy().view(np.uint64), want.view(np.uint64))


def test_benchmark_size_every_element():
    # N = 2^28, the benchmark's size and launch shape: wide-exponent binary64
    # values (low words down to the subnormal range) to float-float and back,
    # every word against the oracle
    n = 1 << 28
    print(f"[gpu] conversions at the benchmark size n={n}", file=sys.stderr, flush=True)
    ff = _ff()
    x = _f64(n, 2300)
    xd = torch.from_numpy(x).cuda()
    pair = ff.ff_from_f64(xd)
    back = ff.ff_to_f64(pair)
    torch.cuda.synchronize()
    del xd
    g, b = pair.cpu().numpy(), back.cpu().numpy()
    del pair, back
    torch.cuda.empty_cache()
    hi, lo = oracle.from_f64(x)
    assert same_bits(g[0], hi), mismatch_report(g[0], hi)
    assert same_bits(g[1], lo), mismatch_report(g[1], lo)
    assert np.array_equal(b.view(np.uint64), oracle.to_f64(hi, lo).view(np.uint64))


def test_unaligned_planes_and_short_names():
    ff = _ff()
    n = 4099
    x = _f64(n + 1, 2301)
    xd = torch.from_numpy(x).cuda()[1:]                    # 8-byte aligned only
    out = ff.ff_zeros((n + 1,), device="cuda")[:, 1:]       # 4-byte aligned planes
    ff.from_float64(xd, out=out)
    torch.cuda.synchronize()
    hi, lo = oracle.from_f64(x[1:])
    o = out.cpu().numpy()
    assert same_bits(o[0], hi) and same_bits(o[1], lo)
    back = torch.zeros(n + 1, dtype=torch.float64, device="cuda")[1:]
    ff.to_float64(out, out=back)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy().view(np.uint64),
                          oracle.to_f64(hi, lo).view(np.uint64))
    a, b, _ = fi.mixed_ff_pair(1000, 2302, device="cuda")
    assert torch.equal(ff.add(a, b), ff.ff_add(a, b))
    assert torch.equal(ff.div(a, b), ff.ff_div(a, b))


def _same_or_both_nan(a, b, view):
    """Bitwise equal, except that any NaN matches any NaN (NaN payloads are
    not specified by IEEE arithmetic and differ between the GPU and x86)."""
    both_nan = np.isnan(a) & np.isnan(b)
    return bool(np.all(both_nan | (a.view(view) == b.view(view))))


@pytest.mark.parametrize("vec", [True, False])
def test_special_values_match_the_oracle(vec):
    # infinities, NaN, FLT_MAX, the binary32 overflow threshold and its
    # neighbour, finite values beyond binary32, signed zeros, values below the
    # smallest subnormal, on 16-byte aligned and on merely 4/8-byte aligned planes
    print(f"[gpu] conversions of special values (vec={vec})", file=sys.stderr, flush=True)
    ff = _ff()
    fmax = float(np.finfo(np.float32).max)
    thresh = fmax + 2.0 ** 103
    base = np.array([np.inf, -np.inf, np.nan, fmax, -fmax, thresh, -thresh,
                     np.nextafter(thresh, 0.0), 1e39, -1e300, 0.0, -0.0, 5e-324, 1e-46,
                     1e-40, -3e-39], dtype=np.float64)
    x = np.tile(base, 9)                                   # 144 values
    xd = torch.from_numpy(x).cuda() if vec else torch.from_numpy(np.r_[0.0, x]).cuda()[1:]
    got = ff.ff_from_f64(xd) if vec else ff.ff_from_f64(
        xd, out=ff.ff_zeros((x.size + 1,), device="cuda")[:, 1:])
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    hi, lo = oracle.from_f64(x)
    assert _same_or_both_nan(g[0], hi, np.uint32) and _same_or_both_nan(g[1], lo, np.uint32)
    # and back: the same pairs (including inf / NaN words) joined in binary64
    pairs = torch.from_numpy(np.stack([hi, lo]))
    back = ff.ff_to_f64(pairs.cuda()).cpu().numpy()
    assert _same_or_both_nan(back, oracle.to_f64(hi, lo), np.uint64)
