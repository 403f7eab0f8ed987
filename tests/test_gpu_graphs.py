"""HIP graph capture of the entry points.

The library allocates nothing, issues no memset and never waits on the host
inside an entry point (the autotuner aside), so a sequence of calls can be
captured once into a HIP graph (through torch.cuda.graph) and replayed.
Each replay, with eager work and synchronisations between replays, must give
the eager results bit for bit: elementwise operators, the batched dot (with
its plan and combine launches), the sliced GEMM (prepasses included), matvec
and its backward, and compensated Horner.
"""
import sys

import pytest
import torch

import ff_inputs as fi

pytestmark = pytest.mark.gpu


def _ff():
    import paper_cs_0603115_amd as ff
    return ff


def _bits_equal(a, b):
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def test_captured_graph_replays_match_eager():
    print("[gpu] graph capture and replay of the entry points", file=sys.stderr, flush=True)
    ff = _ff()
    dev = "cuda"
    a, b, _ = fi.mixed_ff_pair((1 << 20) + 3, 8101, device=dev)
    x, y, offs = fi.batched_dot(8102, device=dev, nvec=64, log2_max=16.0)
    A = fi.gaussian_ff((256, 320), 8103, device=dev)
    B = fi.gaussian_ff((320, 192), 8104, device=dev)
    Mv = fi.gaussian_ff((300, 200), 8105, device=dev)
    v = fi.gaussian_ff((200,), 8106, device=dev)
    gy = fi.gaussian_ff((300,), 8107, device=dev)
    coef = fi.random_poly(9, 8108).to(dev)
    pts = fi.horner_points(4099, 8109, -1.0, 1.0, device=dev)

    # outputs and workspaces exist before capture
    r_add, r_div = ff.ff_empty(a.shape[1:]), ff.ff_empty(a.shape[1:])
    d_out = ff.ff_empty((offs.numel() - 1,))
    ws_dot = torch.empty(max(ff.ff_dot_batched_workspace_size(x.numel(), offs.numel() - 1), 1),
                         dtype=torch.uint8, device=dev)
    C = ff.ff_empty((256, 192))
    ws_gemm = torch.empty(max(ff.ff_gemm_workspace_size(256, 192, 320), 1), dtype=torch.uint8,
                          device=dev)
    y_mv = ff.ff_empty((300,))
    h_out = torch.empty_like(pts)
    fixed = (r_add, r_div, d_out, C, y_mv, h_out)

    def calls():
        ff.ff_add(a, b, out=r_add)
        ff.ff_div(a, b, out=r_div)
        ff.ff_dot_batched(x, y, offs, out=d_out, workspace=ws_dot)
        ff.ff_gemm(A, B, out=C, workspace=ws_gemm)
        ff.ff_matvec(Mv, v, out=y_mv)
        ff.ff_horner_comp(coef, pts, out=h_out)
        return ff.ff_matvec_backward(Mv, v, gy)          # allocates dA, dx, workspace

    dA0, dx0 = calls()
    torch.cuda.synchronize()
    eager = [t.clone() for t in fixed] + [dA0.clone(), dx0.clone()]

    # warm up on a side stream, as torch recommends before capture
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dA_g, dx_g = calls()
    torch.cuda.synchronize()

    for rep in range(4):
        for t in fixed + (dA_g, dx_g):
            t.zero_()                                  # a fill kernel, outside the graph
        ff.ff_mul(a, b)                                # unrelated eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = list(fixed) + [dA_g, dx_g]
        names = ["add", "div", "dot_batched", "gemm", "matvec", "horner_comp", "dA", "dx"]
        for name, g_, e_ in zip(names, got, eager):
            assert _bits_equal(g_, e_), (rep, name)
