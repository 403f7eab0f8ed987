"""GPU parity of the float-float matvec, its hand-written backward pass and
the autograd wrappers.

* plain algorithm: bit-exact against the oracle's sequential definition;
* fast algorithm: every output against the exact value (long accumulator),
  normwise error <= 2^-44 of sum |terms|;
* dA = g x^T: bit-exact against the oracle's Mul22 (it is elementwise);
* the full-size case (8192 x 8192) adds FP64 central finite differences of
  the loss L = sum_i w_i (A x)_i in 64 seeded coordinates of x and 64 of A
  as an independent sanity check.
"""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest
import torch

import ff_inputs as fi
import oracle
from fpexact import frac, mismatch_report, same_bits

pytestmark = pytest.mark.gpu

TWO_M44 = Fraction(1, 1 << 44)


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _announce(msg):
    print(msg, file=sys.stderr, flush=True)


def _abs_ff(h, l):
    """(|v|_hi, |v|_lo) of float-float planes (sign of the value = sign of hi)."""
    s = np.where(h < 0, -1.0, 1.0).astype(np.float32)
    return h * s, l * s


def check_rows_exact(A, x, y, label):
    """y_i vs exact sum_j A_ij x_j for every row (normwise 2^-44)."""
    An, xn, yn = A.cpu().numpy(), x.cpu().numpy(), y.cpu().numpy()
    xa = _abs_ff(xn[0], xn[1])
    worst = -math.inf
    for i in range(An.shape[1]):
        exact = oracle.exact_dot_ff(An[0, i], An[1, i], xn[0], xn[1])
        aa = _abs_ff(An[0, i], An[1, i])
        absum = oracle.exact_dot_ff(aa[0], aa[1], xa[0], xa[1])
        err = abs(frac(yn[0, i]) + frac(yn[1, i]) - exact)
        assert err <= TWO_M44 * absum, (label, i, float(err / absum) if absum else err)
        if err:
            worst = max(worst, math.log2(err / absum))
    return worst


def check_cols_exact(A, g, dx, label, cols=None):
    """dx_j vs exact sum_i g_i A_ij."""
    An, gn, dn = A.cpu().numpy(), g.cpu().numpy(), dx.cpu().numpy()
    M, N = An.shape[1], An.shape[2]
    ga = _abs_ff(gn[0], gn[1])
    worst = -math.inf
    for j in (range(N) if cols is None else cols):
        colh = np.ascontiguousarray(An[0, :, j])
        coll = np.ascontiguousarray(An[1, :, j])
        exact = oracle.exact_dot_ff(gn[0], gn[1], colh, coll)
        ca = _abs_ff(colh, coll)
        absum = oracle.exact_dot_ff(ga[0], ga[1], ca[0], ca[1])
        err = abs(frac(dn[0, j]) + frac(dn[1, j]) - exact)
        assert err <= TWO_M44 * absum, (label, j, float(err / absum) if absum else err)
        if err:
            worst = max(worst, math.log2(err / absum))
    return worst


def check_dA_bits(x, g, dA, label, rows=None, block=256):
    """dA[i, j] = Mul22(g_i, x_j) bit for bit, in blocks of `block` rows (the
    oracle runs on one flattened block at a time)."""
    xn, gn, dn = x.cpu().numpy(), g.cpu().numpy(), dA.cpu().numpy()
    M, N = dn.shape[1], dn.shape[2]
    rows = np.arange(M) if rows is None else np.asarray(rows)
    for b0 in range(0, rows.size, block):
        rb = rows[b0:b0 + block]
        gh = np.repeat(gn[0, rb], N)
        gl = np.repeat(gn[1, rb], N)
        rh, rl = oracle.mul22(gh, gl, np.tile(xn[0], rb.size), np.tile(xn[1], rb.size))
        rh, rl = rh.reshape(rb.size, N), rl.reshape(rb.size, N)
        got_h, got_l = dn[0, rb], dn[1, rb]
        if not (same_bits(got_h, rh) and same_bits(got_l, rl)):
            bad = int(rb[np.flatnonzero(((got_h.view(np.uint32) != rh.view(np.uint32)) |
                                         (got_l.view(np.uint32) != rl.view(np.uint32))).any(axis=1))[0]])
            i = int(np.flatnonzero(rb == bad)[0])
            raise AssertionError((label, bad, "hi: " + mismatch_report(got_h[i], rh[i]),
                                  "lo: " + mismatch_report(got_l[i], rl[i])))


SHAPES = [(1, 1), (3, 5), (64, 1024), (300, 517), (129, 4096), (70, 63)]


@pytest.mark.parametrize("M,N", SHAPES)
def test_matvec_forward_fast_and_plain(M, N):
    ff = _ff()
    A = fi.gaussian_ff((M, N), 500 + M).cuda()
    x = fi.gaussian_ff((N,), 600 + N).cuda()
    y = ff.ff_matvec(A, x)
    check_rows_exact(A, x, y, f"fast {M}x{N}")
    yp = ff.ff_matvec(A, x, algo=ff.MATVEC_PLAIN).cpu().numpy()
    An, xn = A.cpu().numpy(), x.cpu().numpy()
    for i in range(M):
        h, l = oracle.dot_ff_seq(An[0, i], An[1, i], xn[0], xn[1])
        assert (np.float32(h), np.float32(l)) == (yp[0, i], yp[1, i]), (i,)


@pytest.mark.parametrize("M,N", SHAPES)
def test_matvec_backward_fast_and_plain(M, N):
    ff = _ff()
    A = fi.gaussian_ff((M, N), 700 + M).cuda()
    x = fi.gaussian_ff((N,), 800 + N).cuda()
    g = fi.gaussian_ff((M,), 900 + M).cuda()
    dA, dx = ff.ff_matvec_backward(A, x, g)
    check_dA_bits(x, g, dA, f"fast {M}x{N}")
    check_cols_exact(A, g, dx, f"fast {M}x{N}")
    dA2, dx2 = ff.ff_matvec_backward(A, x, g)           # reproducible
    assert torch.equal(dx.view(torch.int32), dx2.view(torch.int32))
    dAp, dxp = ff.ff_matvec_backward(A, x, g, algo=ff.MATVEC_PLAIN)
    assert torch.equal(dAp.view(torch.int32), dA.view(torch.int32))
    An, gn, dxn = A.cpu().numpy(), g.cpu().numpy(), dxp.cpu().numpy()
    for j in range(N):
        h, l = oracle.dot_ff_seq(gn[0], gn[1], np.ascontiguousarray(An[0, :, j]),
                                 np.ascontiguousarray(An[1, :, j]))
        assert (np.float32(h), np.float32(l)) == (dxn[0, j], dxn[1, j]), (j,)


def test_backward_partial_requests_and_padded_rows():
    ff = _ff()
    M, N = 100, 260
    base = fi.gaussian_ff((M, N + 12), 31).cuda()
    A = base[:, :, :N]                                   # lda = N + 12 > N
    x = fi.gaussian_ff((N,), 32).cuda()
    g = fi.gaussian_ff((M,), 33).cuda()
    y = ff.ff_matvec(A, x)
    check_rows_exact(A.contiguous(), x, y, "padded")
    dA, dx = ff.ff_matvec_backward(A, x, g, want_dA=False)
    assert dA is None
    check_cols_exact(A.contiguous(), g, dx, "dx only")
    dA, dx = ff.ff_matvec_backward(A, x, g, want_dx=False)
    assert dx is None
    check_dA_bits(x, g, dA, "dA only")


def test_backward_into_preallocated_outputs_and_workspace():
    """dA_out, dx_out and workspace are written in place and give the bits
    of the allocating call; outputs and workspaces of the wrong size are
    refused before any launch."""
    ff = _ff()
    M, N = 300, 517
    A = fi.gaussian_ff((M, N), 34).cuda()
    x = fi.gaussian_ff((N,), 35).cuda()
    g = fi.gaussian_ff((M,), 36).cuda()
    for algo in (ff.MATVEC_FAST, ff.MATVEC_PLAIN):
        want_dA, want_dx = ff.ff_matvec_backward(A, x, g, algo=algo)
        dA = torch.full((2, M, N), float("nan"), device="cuda")
        dx = torch.full((2, N), float("nan"), device="cuda")
        ws = torch.empty(max(ff.ff_matvec_backward_workspace_size(M, N, algo), 16),
                         dtype=torch.uint8, device="cuda")
        for _ in range(2):
            rA, rx = ff.ff_matvec_backward(A, x, g, algo=algo, dA_out=dA, dx_out=dx, workspace=ws)
            assert rA is dA and rx is dx
            assert torch.equal(dA.view(torch.int32), want_dA.view(torch.int32))
            assert torch.equal(dx.view(torch.int32), want_dx.view(torch.int32))
    nbytes = ff.ff_matvec_backward_workspace_size(M, N)
    if nbytes > 16:
        with pytest.raises(ValueError):
            ff.ff_matvec_backward(A, x, g, workspace=torch.empty(nbytes - 1, dtype=torch.uint8,
                                                                  device="cuda"))
    with pytest.raises(ValueError):
        ff.ff_matvec_backward(A, x, g, dA_out=ff.ff_empty((M, N + 1), device="cuda"))
    with pytest.raises(ValueError):
        ff.ff_matvec_backward(A, x, g, dx_out=ff.ff_empty((N - 1,), device="cuda"))


@pytest.mark.parametrize("n", [1, 4095, 4097, 100003])
def test_dot_backward_elementwise(n):
    ff = _ff()
    u = fi.gaussian_ff((n,), 41).cuda()
    v = fi.gaussian_ff((n,), 42).cuda()
    g = fi.gaussian_ff((1,), 43).cuda()
    un, vn, gn = u.cpu().numpy(), v.cpu().numpy(), g.cpu().numpy()
    gh, gl = np.full(n, gn[0, 0], np.float32), np.full(n, gn[1, 0], np.float32)
    for want_dx, want_dy in ((True, True), (True, False), (False, True)):
        du, dv = ff.ff_dot_backward(g, u, v, want_dx=want_dx, want_dy=want_dy)
        for got, other, wanted in ((du, vn, want_dx), (dv, un, want_dy)):
            assert (got is not None) == wanted
            if got is None:
                continue
            rh, rl = oracle.mul22(gh, gl, other[0], other[1])
            got = got.cpu().numpy()
            assert same_bits(got[0], rh) and same_bits(got[1], rl)


def test_dot_backward_at_the_benchmark_size():
    # the benchmark's launch: float-float x and y at N = 2^28 (seeds 115061,
    # 115062), g = 0.75 + 2^-30, into preallocated outputs; every word
    n = 1 << 28
    _announce(f"[gpu] single-dot backward, n {n}")
    ff = _ff()
    x = fi.gaussian_ff((n,), 115061, device="cuda")
    y = fi.gaussian_ff((n,), 115062, device="cuda")
    g = torch.tensor([[0.75], [2.0 ** -30]], dtype=torch.float32, device="cuda")
    dx, dy = ff.ff_empty((n,)), ff.ff_empty((n,))
    ff.ff_dot_backward(g, x, y, dx_out=dx, dy_out=dy)
    torch.cuda.synchronize()
    piece = 1 << 24
    gh, gl = np.full(piece, 0.75, np.float32), np.full(piece, 2.0 ** -30, np.float32)
    for lo in range(0, n, piece):
        sl = slice(lo, lo + piece)
        for got, other in ((dx, y), (dy, x)):
            o = other[:, sl].cpu().numpy()
            rh, rl = oracle.mul22(gh, gl, o[0], o[1])
            gn = got[:, sl].cpu().numpy()
            assert same_bits(gn[0], rh) and same_bits(gn[1], rl), lo
    del x, y, dx, dy
    torch.cuda.empty_cache()


def test_autograd_matvec_then_dot():
    ff = _ff()
    from paper_cs_0603115_amd.autograd import FFDot, FFMatVec, ff_one
    M, N = 192, 320
    A = fi.gaussian_ff((M, N), 51).cuda().requires_grad_()
    x = fi.gaussian_ff((N,), 52).cuda().requires_grad_()
    w = torch.stack([fi.gaussian_f32((M,), 53), torch.zeros(M)]).cuda()
    y = FFMatVec.apply(A, x)
    loss = FFDot.apply(w, y)
    assert loss.shape == (2,)
    loss.backward(ff_one())
    dA, dx = ff.ff_matvec_backward(A.detach(), x.detach(), ff.ff_dot_backward(ff_one().reshape(2, 1), w, y.detach())[1])
    # the upstream gradient of y is 1 * w (Mul22 by one is exact)
    assert torch.equal(ff.ff_dot_backward(ff_one().reshape(2, 1), w, y.detach())[1], w)
    assert torch.equal(A.grad.view(torch.int32), dA.view(torch.int32))
    assert torch.equal(x.grad.view(torch.int32), dx.view(torch.int32))
    check_cols_exact(A.detach(), w, x.grad, "autograd dx")
    # loss value against the exact bilinear form
    An, xn, wn = A.detach().cpu().numpy(), x.detach().cpu().numpy(), w.cpu().numpy()
    exact = sum(frac(wn[0, i]) * oracle.exact_dot_ff(An[0, i], An[1, i], xn[0], xn[1])
                for i in range(M))
    lv = loss.detach().cpu().numpy()
    scale = sum(abs(frac(wn[0, i])) * oracle.exact_dot_ff(*_abs_ff(An[0, i], An[1, i]),
                                                          *_abs_ff(xn[0], xn[1])) for i in range(M))
    assert abs(frac(lv[0]) + frac(lv[1]) - exact) <= 2 * TWO_M44 * scale


def test_autograd_matvec_under_ordinary_torch_ops():
    """A loss built from y's value with ordinary torch operations sends the
    same derivative to both planes; the backward reads it as that value
    (not as the float-float sum of the two planes, which would double it)."""
    _announce("[gpu] FFMatVec under ordinary torch ops")
    from paper_cs_0603115_amd.autograd import FFMatVec
    M, N = 160, 288
    A = fi.gaussian_ff((M, N), 61).cuda().requires_grad_()
    x = fi.gaussian_ff((N,), 62).cuda().requires_grad_()
    w = fi.gaussian_f32((M,), 63).cuda()
    y = FFMatVec.apply(A, x)
    loss = (w * (y[0] + y[1])).sum()
    loss.backward()
    g = torch.stack([w, torch.zeros_like(w)])
    check_dA_bits(x.detach(), g, A.grad, "dA under torch ops")
    check_cols_exact(A.detach(), g, x.grad, "dx under torch ops")
    # FP64 central differences of the same loss in a few coordinates of x
    An = A.detach().cpu().double()
    Av = An[0] + An[1]
    xv = (x.detach().cpu().double())
    xv = xv[0] + xv[1]
    wv = w.cpu().double()
    gx = x.grad.cpu().double()
    for j in (0, 17, 101, N - 1):
        e = torch.zeros(N, dtype=torch.float64)
        e[j] = 1.0
        fd = (wv @ (Av @ (xv + e)) - wv @ (Av @ (xv - e))) / 2
        assert abs(float(gx[0, j] + gx[1, j]) - float(fd)) <= 2.0 ** -30 * float(
            (wv.abs() @ Av.abs())[j]), j
    # y.sum(): every value weighted by one
    A.grad = x.grad = None
    FFMatVec.apply(A, x).sum().backward()
    ones = torch.stack([torch.ones(M), torch.zeros(M)]).cuda()
    check_dA_bits(x.detach(), ones, A.grad, "dA of y.sum()")
    check_cols_exact(A.detach(), ones, x.grad, "dx of y.sum()")


def test_full_size_8192_matvec_and_backward():
    # Differentiable matvec at full size: A 8192 x 8192 float-float, x 8192,
    # w normal(0,1) binary32, loss = sum w * (A x).
    ff = _ff()
    from paper_cs_0603115_amd.autograd import FFDot, FFMatVec, ff_one
    M = N = 8192
    _announce("[gpu] matvec full size 8192^2: generating")
    A = fi.gaussian_ff((M, N), 115005, device="cuda").requires_grad_()
    x = fi.gaussian_ff((N,), 115006, device="cuda").requires_grad_()
    w = torch.stack([fi.gaussian_f32((M,), 115007, device="cuda"),
                     torch.zeros(M, device="cuda")])
    y = FFMatVec.apply(A, x)
    loss = FFDot.apply(w, y)
    loss.backward(ff_one())
    torch.cuda.synchronize()
    _announce("[gpu] matvec full size: checking y (all rows)")
    wy = check_rows_exact(A.detach(), x.detach(), y.detach(), "full y")
    _announce(f"  y worst normwise log2 error {wy:.1f}")
    _announce("[gpu] matvec full size: checking dA bits (all 8192 rows) and dx (all columns)")
    check_dA_bits(x.detach(), w, A.grad, "full dA")
    wx = check_cols_exact(A.detach(), w, x.grad, "full dx")
    _announce(f"  dx worst normwise log2 error {wx:.1f}")
    # FP64 central finite differences of L in 64 seeded coordinates of x and
    # 64 of A.  L = w^T (A x) is evaluated in FP64 at every perturbed point;
    # the unperturbed pieces are cached (w^T A for the x coordinates, A x
    # with only the perturbed row recomputed for the A coordinates).
    An = A.detach().cpu().numpy()
    Ad = An[0].astype(np.float64) + An[1].astype(np.float64)
    xn = x.detach().cpu().numpy()
    xd = xn[0].astype(np.float64) + xn[1].astype(np.float64)
    wd = w[0].cpu().numpy().astype(np.float64)
    gx = x.grad.cpu().numpy()
    gA = A.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    u = wd @ Ad                                    # w^T A
    v = Ad @ xd                                    # A x
    h = 1.0
    for j in rng.integers(0, N, 64):
        e = np.zeros(N)
        e[j] = h
        fd = (u @ (xd + e) - u @ (xd - e)) / (2 * h)
        an = float(gx[0, j]) + float(gx[1, j])
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(an)), (j, fd, an)
    for i, j in zip(rng.integers(0, M, 64), rng.integers(0, N, 64)):
        ends = []
        for step in (h, -h):
            row = Ad[i].copy()
            row[j] = Ad[i, j] + step
            vp = v.copy()
            vp[i] = row @ xd
            ends.append(wd @ vp)
        fd = (ends[0] - ends[1]) / (2 * h)
        an = float(gA[0, i, j]) + float(gA[1, i, j])
        assert abs(fd - an) <= 1e-9 * max(1.0, abs(an)), (i, j, fd, an)
    del A, x, y, loss
    torch.cuda.empty_cache()
