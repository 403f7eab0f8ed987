"""GPU parity of the batched dot's backward pass (per-vector gradients
through Mul22): every gradient word bit for bit against the oracle, and the
autograd Function against an FP64 reference gradient and FP64 central
differences of the bilinear loss L = sum_v w_v s_v.

Cases: float-float and binary32 inputs (null low words), one output only,
leading and trailing elements outside every vector, empty vectors and runs
of them, vectors of one or two elements (more vector starts in a
wavefront's range than the kernel walks, so each lane searches), exactly
as many starts as it walks and one more, vectors longer than a block, total
lengths not a multiple of the block, planes at 4-byte offsets, no vectors
at all, preallocated outputs and workspace, and the 4096-vector batch of
the benchmark (438 M elements) on every element.
"""
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


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def _offsets(lengths, lead=0):
    return np.concatenate([[lead], lead + np.cumsum(lengths)]).astype(np.int64)


def _check(got, want, label):
    for k, (g, w) in enumerate(zip(got, want)):
        assert same_bits(g, w), f"{label} word {k}:\n{mismatch_report(g, w)}"


def _run(g, x, y, offs, want_dx=True, want_dy=True):
    ff = _ff()
    dx, dy = ff.ff_dot_batched_backward(g, x, y, offs, want_dx=want_dx, want_dy=want_dy)
    torch.cuda.synchronize()
    return (dx.cpu().numpy() if dx is not None else None,
            dy.cpu().numpy() if dy is not None else None)


def _planes(t):
    t = t.cpu().numpy()
    return (t[0], t[1]) if t.ndim == 2 else (t, np.zeros_like(t))


CASES = {
    "mixed": ([3, 1, 0, 5, 8190, 2, 9000, 0, 17, 4, 20000], 3, 11),
    "tiny": ([1] * 300 + [2] * 100, 1, 2),
    "one_long": ([50001], 0, 0),
    "no_vectors": ([], 37, 0),
    # a run of 20 empty vectors at one position: longer than the walk
    "empty_run": ([5] + [0] * 20 + [7, 300, 0, 0, 0, 1000], 0, 5),
    # after the block's first vector, 8 vector starts inside the first
    # wavefront's 64 elements (as many as the walk takes); in the next
    # block 9 (one more)
    "walk_edge": ([7] * 8 + [200] + [6] * 9 + [300], 0, 3),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("inputs", ["ff", "f32"])
def test_bitexact_against_oracle(case, inputs):
    lengths, lead, trail = CASES[case]
    _announce(f"[gpu] dot backward {case} ({inputs} inputs)")
    offs = _offsets(lengths, lead)
    total = int(offs[-1]) + trail
    if inputs == "ff":
        x, y = fi.random_ff(total, 5001, -20, 20), fi.random_ff(total, 5002, -20, 20)
    else:
        x, y = fi.random_f32(total, 5003, -20, 20), fi.random_f32(total, 5004, -20, 20)
    g = fi.random_ff(len(lengths), 5005, -4, 4)
    od = torch.from_numpy(offs).cuda()
    dx, dy = _run(g.cuda(), x.cuda(), y.cuda(), od)
    xh, xl = _planes(x)
    yh, yl = _planes(y)
    want = oracle.dot_batched_backward(g[0].numpy(), g[1].numpy(), offs, xh, xl, yh, yl)
    _check(dx, want[:2], f"{case} dx")
    _check(dy, want[2:], f"{case} dy")
    # one output only
    dx1, dy1 = _run(g.cuda(), x.cuda(), y.cuda(), od, want_dy=False)
    assert dy1 is None
    _check(dx1, want[:2], f"{case} dx alone")


def test_unaligned_planes():
    _announce("[gpu] dot backward, unaligned planes")
    ff = _ff()
    lengths = [5, 4099, 1, 3000]
    offs = _offsets(lengths, 2)
    total = int(offs[-1]) + 3
    x = fi.random_ff(total + 1, 5011, -20, 20)
    y = fi.random_ff(total + 1, 5012, -20, 20)
    g = fi.random_ff(len(lengths), 5013, -4, 4)
    xd, yd = x.cuda()[:, 1:], y.cuda()[:, 1:]        # 4-byte aligned planes only
    dx, dy = ff.ff_dot_batched_backward(g.cuda(), xd, yd, torch.from_numpy(offs).cuda())
    torch.cuda.synchronize()
    want = oracle.dot_batched_backward(g[0].numpy(), g[1].numpy(), offs, x[0, 1:].numpy(),
                                       x[1, 1:].numpy(), y[0, 1:].numpy(), y[1, 1:].numpy())
    _check(dx.cpu().numpy(), want[:2], "dx")
    _check(dy.cpu().numpy(), want[2:], "dy")


def test_benchmark_batch_every_element():
    # the 4096-vector batch (binary32 inputs), the launch the benchmark
    # times: every gradient word against the oracle, in pieces of whole
    # vectors to bound host memory
    _announce("[gpu] dot backward on the 4096-vector batch")
    ff = _ff()
    x, y, offs = fi.batched_dot(115003, device="cuda")
    nvec = offs.numel() - 1
    total = x.numel()
    g = fi.random_ff(nvec, 5021, -4, 4).cuda()
    dx, dy = ff.ff_empty((total,)), ff.ff_empty((total,))
    ws = torch.empty(ff.ff_dot_batched_backward_workspace_size(total), dtype=torch.uint8,
                     device="cuda")
    ff.ff_dot_batched_backward(g, x, y, offs, dx_out=dx, dy_out=dy, workspace=ws)
    torch.cuda.synchronize()
    _announce("  checking every element")
    oh = offs.cpu().numpy()
    gn = g.cpu().numpy()
    step = 256
    for v0 in range(0, nvec, step):
        v1 = min(nvec, v0 + step)
        s, e = int(oh[v0]), int(oh[v1])
        sub = oh[v0:v1 + 1] - s
        xs, ys = x[s:e].cpu().numpy(), y[s:e].cpu().numpy()
        z = np.zeros_like(xs)
        want = oracle.dot_batched_backward(gn[0, v0:v1], gn[1, v0:v1], sub, xs, z, ys, z)
        _check(dx[:, s:e].cpu().numpy(), want[:2], f"vectors {v0}..{v1} dx")
        _check(dy[:, s:e].cpu().numpy(), want[2:], f"vectors {v0}..{v1} dy")
    assert int(oh[0]) == 0 and int(oh[-1]) == total          # no element outside a vector
    del x, y, dx, dy, ws
    torch.cuda.empty_cache()


def test_preallocated_outputs_and_workspace():
    """dx_out, dy_out and a caller's workspace give the bits of the
    allocating call, on two calls in a row (the second shorter, reusing the
    workspace); too small a workspace or wrongly shaped outputs are refused
    before any launch."""
    _announce("[gpu] dot backward into preallocated outputs")
    ff = _ff()
    lengths = [3, 700, 0, 1, 2, 5000, 9, 64, 65]
    offs = _offsets(lengths, 4)
    total = int(offs[-1]) + 6
    x = fi.random_ff(total, 5031, -20, 20).cuda()
    y = fi.random_ff(total, 5032, -20, 20).cuda()
    g = fi.random_ff(len(lengths), 5033, -4, 4).cuda()
    od = torch.from_numpy(offs).cuda()
    ws = torch.empty(ff.ff_dot_batched_backward_workspace_size(total), dtype=torch.uint8,
                     device="cuda")
    for cut in (len(lengths), 4):
        o = od[:cut + 1]
        n = int(offs[cut]) + 1
        want_dx, want_dy = ff.ff_dot_batched_backward(g[:, :cut].contiguous(), x[:, :n], y[:, :n], o)
        dx = torch.full((2, n), float("nan"), device="cuda")
        dy = torch.full((2, n), float("nan"), device="cuda")
        rx, ry = ff.ff_dot_batched_backward(g[:, :cut].contiguous(), x[:, :n], y[:, :n], o,
                                            dx_out=dx, dy_out=dy, workspace=ws)
        assert rx is dx and ry is dy
        assert torch.equal(dx.view(torch.int32), want_dx.view(torch.int32))
        assert torch.equal(dy.view(torch.int32), want_dy.view(torch.int32))
    small = torch.empty(ff.ff_dot_batched_backward_workspace_size(total) - 16, dtype=torch.uint8,
                        device="cuda")
    with pytest.raises(ValueError):
        ff.ff_dot_batched_backward(g, x, y, od, workspace=small)
    with pytest.raises(ValueError):
        ff.ff_dot_batched_backward(g, x, y, od, dx_out=ff.ff_empty((total - 1,)))


def test_autograd_against_fp64_gradient_and_finite_differences():
    _announce("[gpu] FFDotBatched autograd")
    from paper_cs_0603115_amd.autograd import FFDotBatched
    lengths = [7, 300, 0, 1025, 64]
    offs = _offsets(lengths)
    total = int(offs[-1])
    x = fi.gaussian_ff((total,), 5031).cuda().requires_grad_(True)
    y = fi.gaussian_ff((total,), 5032).cuda().requires_grad_(True)
    w = fi.gaussian_f32((len(lengths),), 5033)
    od = torch.from_numpy(offs).cuda()
    s = FFDotBatched.apply(x, y, od)
    # L = sum_v w_v s_v: the upstream gradient of s_v is (w_v, 0)
    s.backward(torch.stack([w, torch.zeros_like(w)]).cuda())
    dx = x.grad.cpu().numpy().astype(np.float64)
    dx = dx[0] + dx[1]
    xv = x.detach().cpu().numpy().astype(np.float64)
    yv = y.detach().cpu().numpy().astype(np.float64)
    xv, yv = xv[0] + xv[1], yv[0] + yv[1]
    owner = np.repeat(np.arange(len(lengths)), lengths)
    ref = w.numpy().astype(np.float64)[owner] * yv
    assert np.all(np.abs(dx - ref) <= 2.0 ** -43 * np.abs(ref) + 1e-300)

    def loss(xx):
        return sum(float(w[v]) * float(np.dot(xx[offs[v]:offs[v + 1]], yv[offs[v]:offs[v + 1]]))
                   for v in range(len(lengths)))

    rng = np.random.default_rng(5034)
    for i in rng.choice(total, 32, replace=False):
        h = 2.0 ** -12 * max(abs(xv[i]), 1.0)
        xp, xm = xv.copy(), xv.copy()
        xp[i] += h
        xm[i] -= h
        fd = (loss(xp) - loss(xm)) / (2 * h)
        assert abs(fd - dx[i]) <= 1e-9 * max(1.0, abs(fd)), (i, fd, dx[i])


def test_autograd_under_ordinary_torch_ops():
    """Losses built from the dots' values with ordinary torch operations send
    the same derivative to both planes; the backward functions read it as
    that binary32 value, so the gradients are Mul22((c, 0), .), bit for bit."""
    _announce("[gpu] FFDotBatched and FFDot under ordinary torch ops")
    from paper_cs_0603115_amd.autograd import FFDot, FFDotBatched
    lengths = [5, 0, 130, 1000, 3]
    offs = _offsets(lengths, lead=2)
    total = int(offs[-1]) + 4
    x = fi.gaussian_ff((total,), 5041).cuda().requires_grad_(True)
    y = fi.gaussian_ff((total,), 5042).cuda().requires_grad_(True)
    w = fi.gaussian_f32((len(lengths),), 5043).cuda()
    s = FFDotBatched.apply(x, y, torch.from_numpy(offs).cuda())
    (w * (s[0] + s[1])).sum().backward()
    g = torch.stack([w, torch.zeros_like(w)]).cpu().numpy()
    want = oracle.dot_batched_backward(g[0], g[1], offs, *_planes(x.detach()),
                                       *_planes(y.detach()))
    _check(x.grad.cpu().numpy(), want[:2], "dx under torch ops")
    _check(y.grad.cpu().numpy(), want[2:], "dy under torch ops")
    # a single dot scaled by three after joining its planes
    u = fi.gaussian_ff((777,), 5044).cuda().requires_grad_(True)
    v = fi.gaussian_ff((777,), 5045).cuda().requires_grad_(True)
    d = FFDot.apply(u, v)
    (3.0 * (d[0] + d[1])).backward()
    o = np.array([0, 777], np.int64)
    want = oracle.dot_batched_backward(np.float32([3.0]), np.float32([0.0]), o,
                                       *_planes(u.detach()), *_planes(v.detach()))
    _check(u.grad.cpu().numpy(), want[:2], "FFDot du under torch ops")
    _check(v.grad.cpu().numpy(), want[2:], "FFDot dv under torch ops")


def _candidates_hold(d, g, y_h, y_l):
    """Every element of the gradient pair d is Mul22(g_v, y_i) for some v, or
    a zero pair: the property the entry point keeps for offsets that break
    their non-decreasing order (which vector owns an element is then
    unspecified, but only real gradients or zeros are written)."""
    n = y_h.size
    ok = (d[0] == 0) & (d[1] == 0)
    for v in range(g.shape[1]):
        ch, cl = oracle.elementwise("mul", np.full(n, g[0, v], np.float32),
                                    np.full(n, g[1, v], np.float32), y_h, y_l)
        ok |= same_bits_mask(d[0], ch) & same_bits_mask(d[1], cl)
    return ok


def same_bits_mask(a, b):
    return a.view(np.int32) == b.view(np.int32)


@pytest.mark.parametrize("case", ["shuffled_small", "out_of_range", "shuffled_wide"])
def test_offsets_out_of_order_write_only_real_gradients(case):
    _announce(f"[gpu] dot backward with offsets out of order: {case}")
    rng = np.random.default_rng(5011)
    if case == "shuffled_small":
        total, offs = 5000, np.array([100, 3000, 800, 4999, 2, 4000], np.int64)
    elif case == "out_of_range":
        total, offs = 7001, np.array([-9, 7100, -1, 50, 7001, 1 << 40], np.int64)
    else:
        # 600 vectors, starts shuffled: windows wider than the LDS copy
        total = 300007
        offs = np.sort(rng.integers(0, total + 1, 601)).astype(np.int64)
        rng.shuffle(offs[100:500])
    nvec = offs.size - 1
    x = fi.random_ff(total, 5012, -20, 20)
    y = fi.random_f32(total, 5013, -20, 20)
    g = fi.random_ff(nvec, 5014, -4, 4)
    dx, dy = _run(g.cuda(), x.cuda(), y.cuda(), torch.from_numpy(offs).cuda())
    gn = g.numpy()
    yh, yl = _planes(y)
    xh, xl = _planes(x)
    assert _candidates_hold(dx, gn, yh, yl).all()
    assert _candidates_hold(dy, gn, xh, xl).all()
