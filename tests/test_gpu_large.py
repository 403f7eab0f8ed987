"""Maximum sizes: every entry point on inputs of more than 2^31 elements,
where any 32-bit element index would wrap.  The HBM of one MI355X (288 GB)
holds these comfortably; each case frees its tensors before the next.

* elementwise Add22 at N = 2^31 + 7 (mixed workload): bit-exact against the
  oracle on the last 2^20 pairs, a window across index 2^31 and a strided
  sample;
* batched dot with a vector of 2^31 + 3 ones times ones: the exact result
  2^31 + 3 (sums of integers below 2^48 are exact in float-float);
* matvec forward and backward on a 65536 x 32769 matrix of ones: y = 32769
  and dx = 65536 exactly, dA = g x^T bit for bit on sampled rows;
* sliced GEMM (int8 digits) with A of 65536 x 32800 (> 2^31 entries, K split
  into chunks): sampled entries within 2^-44 (|A||B|) of the exact product;
* compensated Horner and the binary64 conversions at 2^31 + 5 points:
  bit-exact on the tail, the 2^31 window and a strided sample;
* the batched dot backward over a vector of 2^31 + 3 ones (plus elements
  outside every vector) and the single-dot backward at 2^31 + 9: every
  sampled gradient word equals its closed form (Mul22(g, 1) = g);
* the paper's Add12 stream operator and the copy probe at 2^31 + 11
  elements (closed forms).
"""
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import ff_value, same_bits

pytestmark = pytest.mark.gpu

BIG = 1 << 31


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def _sample_index(n, device):
    """Indices below n: the last 2^20, the window [2^31 - 2048, 2^31 + 2048)
    clipped to n, and every 1000003rd element.  Checked on the host before
    any gather uses them."""
    parts = [torch.arange(n - (1 << 20), n), torch.arange(BIG - 2048, min(n, BIG + 2048)),
             torch.arange(0, n, 1000003)]
    idx = torch.unique(torch.cat(parts))
    assert int(idx.min()) >= 0 and int(idx.max()) < n, "sample index out of range"
    return idx.to(device)


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_elementwise_beyond_2p31():
    n = BIG + 7
    _announce(f"[gpu] large: ff_add at n={n}")
    ff = _ff()
    a, b, _ = fi.mixed_ff_pair(n, 3101, device="cuda")
    r = ff.ff_add(a, b)
    idx = _sample_index(n, "cuda")
    an, bn, rn = (t[:, idx].cpu().numpy() for t in (a, b, r))
    del a, b, r
    _free()
    rh, rl = oracle.elementwise("add", an[0], an[1], bn[0], bn[1])
    assert same_bits(rn[0], rh) and same_bits(rn[1], rl)


def test_batched_dot_vector_beyond_2p31():
    lengths = [5, BIG + 3, 7]
    _announce(f"[gpu] large: batched dot, vector lengths {lengths}")
    ff = _ff()
    total = sum(lengths)
    x = torch.ones(total, device="cuda")
    y = torch.ones(total, device="cuda")
    offs = torch.tensor(np.concatenate([[0], np.cumsum(lengths)]), dtype=torch.int64,
                        device="cuda")
    d = ff.ff_dot_batched(x, y, offs).cpu().numpy()
    del x, y, offs
    _free()
    for v, length in enumerate(lengths):
        assert ff_value(d[0, v], d[1, v]) == length, (v, d[:, v])


def test_matvec_beyond_2p31():
    M, N = 1 << 16, (1 << 15) + 1
    _announce(f"[gpu] large: matvec {M} x {N} of ones, forward and backward")
    ff = _ff()
    A = torch.zeros((2, M, N), device="cuda")
    A[0].fill_(1.0)
    x = torch.zeros((2, N), device="cuda")
    x[0].fill_(1.0)
    y = ff.ff_matvec(A, x).cpu().numpy()
    assert np.all(y[0] == N) and np.all(y[1] == 0)
    g = torch.stack([fi.gaussian_f32((M,), 3102, device="cuda"), torch.zeros(M, device="cuda")])
    dA, dx = ff.ff_matvec_backward(A, x, g)
    rows = torch.tensor([0, 1, M // 2, M - 2, M - 1], device="cuda")
    dAs = dA[:, rows].cpu().numpy()
    gn = g.cpu().numpy()
    dxn = dx.cpu().numpy()
    del A, x, dA, dx, g
    _free()
    # dA = g x^T with x = 1: every entry of row i is Mul22((g_i, 0), (1, 0)) = (g_i, 0)
    for k, i in enumerate(rows.cpu().numpy()):
        assert np.all(dAs[0, k] == gn[0, i]) and np.all(dAs[1, k] == 0)
    # dx = A^T g: every column sums all of g, exactly as a float-float value
    # to within 2^-44 of the exact sum of |g|
    exact = sum((Fraction(float(v)) for v in gn[0]), Fraction(0))
    scale = sum((abs(Fraction(float(v))) for v in gn[0]), Fraction(0))
    for j in (0, 1, N // 2, N - 1):
        assert abs(ff_value(dxn[0, j], dxn[1, j]) - exact) <= scale / 2 ** 44, j


def test_gemm_operand_beyond_2p31():
    M, K, N = 1 << 16, 32800, 64
    _announce(f"[gpu] large: sliced GEMM {M} x {K} x {N}")
    ff = _ff()
    A = fi.gaussian_ff((M, K), 3103, device="cuda")
    B = fi.gaussian_ff((K, N), 3104, device="cuda")
    C = ff.ff_gemm(A, B, algo=ff.GEMM_SLICED_I8).cpu().numpy()
    rows = np.array([0, 1, M // 2, M - 1])
    Asub = A[:, torch.from_numpy(rows).cuda()].cpu().numpy()
    Bn = B.cpu().numpy()
    del A, B
    _free()
    cols = np.array([0, 17, N - 1])
    rr, cc = np.meshgrid(np.arange(rows.size), cols, indexing="ij")
    ex = oracle.exact_gemm_entries(Asub[0], Asub[1], Bn[0], Bn[1], rr.ravel(), cc.ravel())
    ab = oracle.exact_absgemm_entries(Asub[0], Asub[1], Bn[0], Bn[1], rr.ravel(), cc.ravel())
    for t, (i, j) in enumerate(zip(rr.ravel(), cc.ravel())):
        got = ff_value(C[0, rows[i], j], C[1, rows[i], j])
        assert abs(got - ex[t]) <= ab[t] / 2 ** 44, (rows[i], j)


def test_horner_and_conversions_beyond_2p31():
    n = BIG + 5
    _announce(f"[gpu] large: compensated Horner and conversions at n={n}")
    ff = _ff()
    coef = fi.random_poly(3, 3105)
    x = fi.horner_points(n, 3106, -1.5, 1.5, device="cuda")
    y = ff.ff_horner_comp(coef.cuda(), x)
    idx = _sample_index(n, "cuda")
    xs, ys = x[idx].cpu().numpy(), y[idx].cpu().numpy()
    del y
    _free()
    assert same_bits(ys, oracle.horner_comp(coef.numpy(), xs))
    # binary64 -> float-float -> binary64 over the same points
    xd = x.double()
    del x
    _free()
    pair = ff.ff_from_f64(xd)
    ps = pair[:, idx].cpu().numpy()
    xds = xd[idx].cpu().numpy()
    del xd
    _free()
    back = ff.ff_to_f64(pair)
    bs = back[idx].cpu().numpy()
    del pair, back
    _free()
    hi, lo = oracle.from_f64(xds)
    assert same_bits(ps[0], hi) and same_bits(ps[1], lo)
    assert np.array_equal(bs.view(np.uint64), oracle.to_f64(hi, lo).view(np.uint64))


def test_dot_backward_beyond_2p31():
    # x = y = 1: Mul22(g, (1, 0)) = g exactly, so every gradient word is a
    # closed form; the batched form gives each vector's own g and zeros
    # outside all vectors
    lengths = [5, BIG + 3, 7]
    lead, trail = 2, 3
    total = lead + sum(lengths) + trail
    _announce(f"[gpu] large: batched dot backward, total {total}")
    ff = _ff()
    offs_h = np.concatenate([[lead], lead + np.cumsum(lengths)]).astype(np.int64)
    x = torch.ones(total, device="cuda")
    g = torch.tensor([[1.5, -2.0, 0.75], [2.0 ** -30, 2.0 ** -31, -(2.0 ** -27)]], device="cuda")
    dx, dy = ff.ff_dot_batched_backward(g, x, x, torch.from_numpy(offs_h).cuda())
    idx = _sample_index(total, "cuda")
    dxs, dys = dx[:, idx].cpu().numpy(), dy[:, idx].cpu().numpy()
    # every element, segment by segment: a vector's words are its g, the rest zero
    bounds = [0] + [int(o) for o in offs_h] + [total]
    for seg in range(len(bounds) - 1):
        a, b = bounds[seg], bounds[seg + 1]
        v = seg - 1
        for plane in range(2):
            want = float(g[plane, v]) if 0 <= v < len(lengths) else 0.0
            for t in (dx, dy):
                assert bool((t[plane, a:b] == want).all()), (seg, plane)
    del dx, dy
    _free()
    owner = np.searchsorted(offs_h, idx.cpu().numpy(), side="right") - 1
    gn = g.cpu().numpy()
    for k, v in enumerate(owner):
        want = gn[:, v] if 0 <= v < len(lengths) else np.zeros(2, np.float32)
        assert np.array_equal(dxs[:, k], want) and np.array_equal(dys[:, k], want), (k, v)
    # the single-dot backward over float-float inputs of the same length
    n = BIG + 9
    _announce(f"[gpu] large: dot backward, n {n}")
    del x
    _free()
    xf = torch.zeros((2, n), device="cuda")
    xf[0].fill_(1.0)
    g1 = torch.tensor([-3.25, 2.0 ** -29], device="cuda")
    dx, dy = ff.ff_dot_backward(g1, xf, xf)
    idx = _sample_index(n, "cuda")
    dxs, dys = dx[:, idx].cpu().numpy(), dy[:, idx].cpu().numpy()
    del dx, dy, xf
    _free()
    want = g1.cpu().numpy()[:, None]
    assert np.all(dxs == want) and np.all(dys == want)


def test_stream_operators_and_copy_beyond_2p31():
    # Add12 of a = 1 + k 2^-10 (k = i mod 1024) and b = 2^-30: s = a exactly
    # (b is below half an ulp of a), r = b; the copy probe on the same data
    n = BIG + 11
    _announce(f"[gpu] large: Add12 and the copy probe at n={n}")
    ff = _ff()
    a = (torch.arange(n, device="cuda", dtype=torch.int64) % 1024).to(torch.float32)
    a.mul_(2.0 ** -10).add_(1.0)
    b = torch.full((n,), 2.0 ** -30, device="cuda")
    out = ff.ff_add12(a, b)
    idx = _sample_index(n, "cuda")
    outs, as_ = out[:, idx].cpu().numpy(), a[idx].cpu().numpy()
    del out, b
    _free()
    assert np.array_equal(outs[0], as_) and np.all(outs[1] == np.float32(2.0 ** -30))
    dst = torch.empty_like(a)
    ff.ff_copy(a, dst)
    ds = dst[idx].cpu().numpy()
    del a, dst
    _free()
    assert np.array_equal(ds, as_)
