"""Host logic of the benchmark: the CPU baseline runs the unchanged oracle on
disjoint pieces of one sample on several host threads; the pieces must give
the same results as one call over the whole sample, and the piece bounds
must tile the range.  Also: more than one GPU is refused with a message, and
the defaults measure one GPU on the full 2^28-pair workload."""
import subprocess
import sys

import numpy as np
import pytest

import bench
import ff_inputs as fi
import oracle


@pytest.mark.parametrize("n,parts", [(0, 3), (1, 4), (7, 3), (4096, 16), (1000003, 8)])
def test_chunks_tile_the_range(n, parts):
    b = bench._chunks(n, parts)
    assert len(b) == parts and b[0][0] == 0 and b[-1][1] == n
    assert all(b[k][1] == b[k + 1][0] for k in range(parts - 1))
    sizes = [hi - lo for lo, hi in b]
    assert max(sizes) - min(sizes) <= 1


def test_host_threads_bounded():
    assert 1 <= bench._host_threads() <= 16


def test_parallel_elementwise_pieces_match_one_call():
    a, b, _ = fi.mixed_ff_pair(100003, 115002)
    ah, al, bh, bl = (t.numpy() for t in (a[0], a[1], b[0], b[1]))
    n = ah.size
    for op in ("add", "sub", "mul", "div"):
        rh, rl = np.empty(n, np.float32), np.empty(n, np.float32)

        def piece(lo, hi):
            return lambda: oracle.elementwise(op, ah[lo:hi], al[lo:hi], bh[lo:hi], bl[lo:hi],
                                              out=(rh[lo:hi], rl[lo:hi]))

        dt, th = bench._oracle_parallel([piece(lo, hi) for lo, hi in bench._chunks(n, 13)])
        assert dt >= 0 and 1 <= th <= 16
        eh, el = oracle.elementwise(op, ah, al, bh, bl)
        assert np.array_equal(eh.view(np.int32), rh.view(np.int32)), op
        assert np.array_equal(el.view(np.int32), rl.view(np.int32)), op


def test_parallel_dot_pieces_match_one_call():
    x, y, offs = fi.batched_dot(115003, nvec=40)
    xs, ys, oh = x.numpy(), y.numpy(), offs.numpy()
    one = oracle.dot_seq_batched(xs, ys, oh)
    parts = {}

    def piece(v0, v1):
        o0, o1 = int(oh[v0]), int(oh[v1])

        def run():
            parts[v0] = oracle.dot_seq_batched(xs[o0:o1], ys[o0:o1], oh[v0:v1 + 1] - o0)
        return run

    bench._oracle_parallel([piece(v0, v1) for v0, v1 in bench._chunks(40, 7)])
    for k in (0, 1):
        got = np.concatenate([parts[v][k] for v in sorted(parts)])
        assert np.array_equal(got.view(np.int32), one[k].view(np.int32))


def test_parallel_gemm_row_pieces_match_one_call():
    A = fi.gaussian_ff((37, 96), 11)
    B = fi.gaussian_ff((96, 21), 12)
    Ah, Al, Bh, Bl = A[0].numpy(), A[1].numpy(), B[0].numpy(), B[1].numpy()
    full = oracle.gemm_ff_seq(Ah, Al, Bh, Bl)
    res = {}

    def piece(lo, hi):
        def run():
            res[lo] = oracle.gemm_ff_seq(Ah[lo:hi], Al[lo:hi], Bh, Bl)
        return run

    bench._oracle_parallel([piece(lo, hi) for lo, hi in bench._chunks(37, 5)])
    for k in (0, 1):
        got = np.concatenate([res[r][k] for r in sorted(res)])
        assert np.array_equal(got.view(np.int32), full[k].view(np.int32))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_default_arguments_measure_one_gpu_on_the_full_workload():
    a = bench.parse_args([])
    assert a.gpus == 1 and a.steps > 0 and a.warmup >= 0
    assert a.log2n == 28 and a.seed == 115002 and a.dot_cfg is None
    assert not a.no_cpu_baseline and not a.no_secondary
    b = bench.parse_args(["--steps", "5", "--warmup", "2", "--dot-cfg", "256,4096,0,16"])
    assert (b.steps, b.warmup, b.dot_cfg) == (5, 2, "256,4096,0,16")
