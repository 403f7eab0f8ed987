"""GPU parity of the elementwise operators: bit-exact against the oracle.

Every case generates seeded inputs, runs the HIP kernel through the C ABI
(via the thin binding) and the CPU oracle on the same inputs, and compares
all output words bit for bit (any NaN equal to any NaN).
"""
import sys

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import mismatch_report, same_bits

pytestmark = pytest.mark.gpu

OPS = ["add", "sub", "mul", "mul_dekker", "div", "add_accurate", "sub_accurate",
       "mul_accurate", "div_accurate"]


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def gpu_op(op, a, b, out=None):
    ff = _ff()
    fn = {"add": ff.ff_add, "sub": ff.ff_sub, "mul": ff.ff_mul,
          "mul_dekker": ff.ff_mul_dekker, "div": ff.ff_div,
          "add_accurate": ff.ff_add_accurate, "sub_accurate": ff.ff_sub_accurate,
          "mul_accurate": ff.ff_mul_accurate, "div_accurate": ff.ff_div_accurate}[op]
    r = fn(a, b, out=out)
    torch.cuda.synchronize()
    return r


def assert_parity(op, a, b, r, label):
    """r (GPU result, any device) against the oracle on a, b."""
    a_, b_, r_ = (t.cpu().numpy() for t in (a, b, r))
    rh, rl = oracle.elementwise(op, a_[0], a_[1], b_[0], b_[1])
    ok_h, ok_l = same_bits(r_[0], rh), same_bits(r_[1], rl)
    assert ok_h and ok_l, f"{label} {op}:\n hi {mismatch_report(r_[0], rh)}\n lo {mismatch_report(r_[1], rl)}"


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.parametrize("op", OPS)
def test_base_workload_n2_20(op):
    # elementwise workload on 2^20 pairs: x = +-2^t, t ~ U[-20, 20]
    _announce(f"[gpu] elementwise base n=2^20 op={op}")
    a = fi.base_ff(1 << 20, 115001).cuda()
    b = fi.base_ff(1 << 20, 115011).cuda()
    assert_parity(op, a, b, gpu_op(op, a, b), "base 2^20")


@pytest.mark.parametrize("op", OPS)
def test_mixed_workload_ragged(op):
    # cancellation (25 %) and exponent-gap (10 %) pairs; several workgroup
    # tiles plus a ragged scalar tail
    n = 3 * (1 << 20) + 13
    _announce(f"[gpu] elementwise mixed n={n} op={op}")
    a, b, _ = fi.mixed_ff_pair(n, 115002)
    a, b = a.cuda(), b.cuda()
    assert_parity(op, a, b, gpu_op(op, a, b), "mixed ragged")


@pytest.mark.parametrize("op", OPS)
def test_wide_exponents_and_subnormal_words(op):
    # exponents down to the subnormal boundary: low words, cross products and
    # TwoProd error words fall into the subnormal range on both sides
    _announce(f"[gpu] elementwise wide exponents op={op}")
    a = torch.cat([fi.random_ff(1 << 16, 7, -90, 90), fi.random_ff(1 << 16, 8, -101, -60)], 1)
    b = torch.cat([fi.random_ff(1 << 16, 9, -90, 90), fi.random_ff(1 << 16, 10, -40, 10)], 1)
    a, b = a.contiguous().cuda(), b.contiguous().cuda()
    assert_parity(op, a, b, gpu_op(op, a, b), "wide exponents")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 255, 1023, 1025, 4096 * 4 + 3])
def test_small_and_tail_sizes(op, n):
    a, b, _ = fi.mixed_ff_pair(n, 1000 + n)
    a, b = a.cuda(), b.cuda()
    assert_parity(op, a, b, gpu_op(op, a, b), f"n={n}")


@pytest.mark.parametrize("op", OPS)
def test_unaligned_planes_take_the_scalar_path(op):
    _announce(f"[gpu] elementwise unaligned op={op}")
    n = 50001
    a, b, _ = fi.mixed_ff_pair(n + 1, 4242)
    a, b = a.cuda(), b.cuda()
    av, bv = a[:, 1:], b[:, 1:]                      # planes start 4 bytes past 16-byte alignment
    out = torch.empty(2, n + 1, device="cuda")[:, 1:]
    gpu_op(op, av, bv, out=out)
    assert_parity(op, av, bv, out, "unaligned")


@pytest.mark.parametrize("op", OPS)
def test_in_place_output(op):
    n = 100003
    a, b, _ = fi.mixed_ff_pair(n, 777)
    a, b = a.cuda(), b.cuda()
    a_copy = a.clone()
    gpu_op(op, a, b, out=a)                          # r aliases a exactly
    assert_parity(op, a_copy, b, a, "in-place")


def _special_pairs(tile):
    """Every pair of special high words (signed zeros, +-1, +-inf, NaN, the
    largest finite, the smallest normal, a subnormal, 3), each with a zero
    and a small low word, tiled to reach the requested size."""
    f32 = np.float32
    hi = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, np.finfo(f32).max,
                   -np.finfo(f32).max, np.finfo(f32).tiny, 1e-40, 3.0], dtype=f32)
    lo_of = lambda h: np.where(np.isfinite(h) & (np.abs(h) >= f32(2.0 ** -100)),
                               (h * f32(2.0 ** -30)).astype(f32), f32(0.0))
    ah, bh = np.meshgrid(hi, hi, indexing="ij")
    ah, bh = ah.ravel(), bh.ravel()
    al_small, bl_small = lo_of(ah), lo_of(bh)
    z = np.zeros_like(ah)
    a = np.concatenate([np.stack([ah, z]), np.stack([ah, al_small]), np.stack([ah, z]),
                        np.stack([ah, al_small])], axis=1)
    b = np.concatenate([np.stack([bh, z]), np.stack([bh, z]), np.stack([bh, bl_small]),
                        np.stack([bh, bl_small])], axis=1)
    reps = -(-tile // a.shape[1])
    return (torch.from_numpy(np.tile(a, (1, reps))[:, :tile].copy()),
            torch.from_numpy(np.tile(b, (1, reps))[:, :tile].copy()))


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [576, (1 << 22) + 3])
def test_special_values_match_the_oracle(op, n):
    # the paper excludes NaN, infinities and overflow from its inputs; the
    # kernels still follow the oracle through them (IEEE propagation along
    # the same operation sequences; any NaN equals any NaN).  n covers the
    # float4 form (below 2^22) and the lane-contiguous form.
    _announce(f"[gpu] elementwise special values op={op} n={n}")
    a, b = _special_pairs(n)
    a, b = a.cuda(), b.cuda()
    assert_parity(op, a, b, gpu_op(op, a, b), f"specials n={n}")


def test_concurrent_host_threads_on_separate_streams():
    # the entry points keep no mutable global state: four host threads, each
    # with its own stream and data, issue the operators at the same time (the
    # foreign calls release the interpreter lock); every result is the oracle's
    import threading
    _announce("[gpu] elementwise from four host threads on four streams")
    ff = _ff()
    n = (1 << 20) + 5
    jobs = []
    for k in range(4):
        a, b, _ = fi.mixed_ff_pair(n, 3300 + k)
        jobs.append((a, b, a.cuda(), b.cuda(), torch.cuda.Stream()))
    torch.cuda.synchronize()
    results = [dict() for _ in jobs]
    errors = []
    fns = {"add": ff.ff_add, "mul": ff.ff_mul, "div": ff.ff_div,
           "add_accurate": ff.ff_add_accurate}

    def work(k):
        try:
            _, _, ad, bd, st = jobs[k]
            with torch.cuda.stream(st):
                for rep in range(20):
                    for op in ("add", "mul", "div", "add_accurate"):
                        results[k][op] = fns[op](ad, bd, stream=st)
            st.synchronize()
        except Exception as exc:   # surfaced in the main thread
            errors.append(exc)

    threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k, (a, b, _, _, _) in enumerate(jobs):
        for op, got in results[k].items():
            g = got.cpu().numpy()
            rh, rl = oracle.elementwise(op, a[0].numpy(), a[1].numpy(), b[0].numpy(), b[1].numpy())
            assert same_bits(g[0], rh) and same_bits(g[1], rl), (k, op)


def test_zero_length_is_a_noop():
    a = torch.empty(2, 0, device="cuda")
    r = gpu_op("add", a, a)
    assert r.shape == (2, 0)


def test_repeat_runs_are_bitwise_identical():
    a, b, _ = fi.mixed_ff_pair(1 << 20, 31337)
    a, b = a.cuda(), b.cuda()
    for op in OPS:
        r1 = gpu_op(op, a, b).clone()
        r2 = gpu_op(op, a, b)
        assert torch.equal(r1.view(torch.int32), r2.view(torch.int32))


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div", "add_accurate", "div_accurate"])
def test_full_size_n2_28_bitexact(op):
    # the full operator-set workload: 2^28 pairs generated on the device, in
    # the launch configuration the benchmark times; every output word checked
    n = 1 << 28
    _announce(f"[gpu] elementwise full size n=2^28 op={op}")
    a, b, _ = fi.mixed_ff_pair(n, 115002, device="cuda")
    r = gpu_op(op, a, b)
    assert_parity(op, a, b, r, "full 2^28")
    del a, b, r
    torch.cuda.empty_cache()
