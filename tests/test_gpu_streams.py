"""Work enqueued on a side stream keeps its outputs and workspaces.

The Python wrappers allocate outputs and workspaces with torch.  When a
``stream`` is given, that memory must belong to the stream the kernels run
on; otherwise, once the wrapper returns, torch's caching allocator may hand
the same block to the next allocation on the current stream while the side
stream's kernels still use it.  Each case queues a long operation on the
side stream first (so the side stream's kernels start late), then the
reduction or product under test, then allocates and overwrites memory of
the same size on the current stream before any synchronisation, and finally
compares the side stream's result bit for bit with the same call made on the
current stream alone.  Whether the two streams really run concurrently
depends on how the runtime maps them to hardware queues, so each case also
checks the cause directly: the allocator segment holding the output belongs
to the side stream.
"""
import sys

import numpy as np
import pytest
import torch

import ff_inputs as fi

pytestmark = pytest.mark.gpu


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _busy(ff, stream, n=1 << 26, reps=4):
    """A few milliseconds of elementwise work on `stream`, after everything
    already queued on the current stream (the inputs included)."""
    a, b, _ = fi.mixed_ff_pair(n, seed=99, device="cuda")
    out = ff.ff_empty((n,))
    stream.wait_stream(torch.cuda.current_stream())
    for _ in range(reps):
        ff.ff_mul(a, b, out=out, stream=stream)
    return a, b, out


def _owner_stream(t):
    """The stream of torch's allocator segment holding tensor t."""
    ptr = t.data_ptr()
    for seg in torch.cuda.memory_snapshot():
        if seg["address"] <= ptr < seg["address"] + seg["total_size"]:
            return seg["stream"]
    raise AssertionError("tensor not found in the allocator snapshot")


def _scribble(nbytes, times=4):
    """Allocate and overwrite blocks of nbytes on the current stream."""
    keep = []
    for _ in range(times):
        t = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        t.fill_(0xFF)
        keep.append(t)
    return keep


def test_batched_dot_on_a_side_stream():
    ff = _ff()
    print("[gpu] batched dot on a side stream", file=sys.stderr, flush=True)
    x, y, offs = fi.batched_dot(3301, device="cuda", nvec=600, log2_max=16)
    want = ff.ff_dot_batched(x, y, offs)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    keep = _busy(ff, side)
    got = ff.ff_dot_batched(x, y, offs, stream=side)
    assert _owner_stream(got) == side.cuda_stream
    nbytes = ff.ff_dot_batched_workspace_size(x.numel(), 600)
    junk = _scribble(nbytes) + _scribble(got.numel() * 4)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want.cpu().numpy().view(np.uint32))
    del keep, junk


def test_sliced_gemm_on_a_side_stream():
    ff = _ff()
    print("[gpu] sliced GEMM on a side stream", file=sys.stderr, flush=True)
    A = fi.gaussian_ff((384, 512), 3302).cuda()
    B = fi.gaussian_ff((512, 256), 3303).cuda()
    want = ff.ff_gemm(A, B)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    keep = _busy(ff, side)
    got = ff.ff_gemm(A, B, stream=side)
    assert _owner_stream(got) == side.cuda_stream
    junk = _scribble(ff.ff_gemm_workspace_size(384, 256, 512)) + _scribble(got.numel() * 4)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want.cpu().numpy().view(np.uint32))
    del keep, junk


def test_matvec_backward_on_a_side_stream_by_handle():
    """The stream may also be passed as a raw hipStream_t handle."""
    ff = _ff()
    print("[gpu] matvec backward on a side stream (raw handle)", file=sys.stderr, flush=True)
    A = fi.gaussian_ff((1024, 768), 3304).cuda()
    x = fi.gaussian_ff((768,), 3305).cuda()
    g = fi.gaussian_ff((1024,), 3306).cuda()
    want_dA, want_dx = ff.ff_matvec_backward(A, x, g)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    keep = _busy(ff, side)
    dA, dx = ff.ff_matvec_backward(A, x, g, stream=side.cuda_stream)
    assert _owner_stream(dx) == side.cuda_stream
    nbytes = int(ff.lib.ff_matvec_backward_workspace_size(1024, 768, 0))
    junk = _scribble(nbytes) + _scribble(dx.numel() * 4) + _scribble(dA.numel() * 4, times=1)
    torch.cuda.synchronize()
    assert torch.equal(dA.view(torch.int32), want_dA.view(torch.int32))
    assert torch.equal(dx.view(torch.int32), want_dx.view(torch.int32))
    del keep, junk
