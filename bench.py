"""Benchmark of the float-float hot path on one MI355X.

One step = the full elementwise operator set (ff_add, ff_sub, ff_mul, ff_div)
over N = 2^28 float-float pairs of the mixed workload (25 % cancellation and
10 % exponent-gap pairs), inputs resident in HBM.  The metric is float-float
operations per second (4 N per step).

Printed: ONE JSON line on stdout, with
  * ``roofline`` for the dominant kernel (algorithmic bytes / average launch
    time from HIP events recorded on the launch stream, against 8 TB/s),
  * ``cpu_baseline``: the oracle (C) timed on this host on a bounded sample of
    the same inputs, on up to 16 host threads over disjoint pieces of the
    sample (``cores``), with its single-threaded rate beside it.
Progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_FF_OP = 24           # 4 binary32 words in, 2 out
# binary32 VALU rate: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T adds,
# multiplies or fused multiply-adds per second (the published 157.3 TFLOP/s
# counts a fused multiply-add as two).  A wave64 binary32 instruction issues
# in two cycles: the compensated Horner loop, 11 such instructions per point
# and step and no packed ones, averages 2.8 cycles per instruction.
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
OPS = ["add", "sub", "mul", "div"]


PROFILE_SUMMARY = os.path.join(_ROOT, "profiles", "elementwise_ff_ops_2p28.md")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def profiled_traffic(op: str, n: int):
    """HBM bytes per launch of ff_<op> measured by rocprofv3 (FETCH_SIZE and
    WRITE_SIZE, calibrated on the copy probe) and recorded in the profile
    summary -- or None if that summary is missing, was taken at another size,
    or the kernel sources changed since (sha256 of the listed files)."""
    import hashlib

    try:
        text = open(PROFILE_SUMMARY).read()
    except OSError:
        return None
    if n != 1 << 28:
        return None
    fields = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) >= 2 and parts[0] in ("traffic_bytes_per_launch", "sources_sha256", "sources"):
            fields.setdefault(parts[0], []).append(parts[1:])
    try:
        digest = hashlib.sha256()
        for path in fields["sources"][0]:
            with open(os.path.join(_ROOT, path), "rb") as f:
                digest.update(f.read())
        if digest.hexdigest() != fields["sources_sha256"][0][0]:
            return None
        for entry in fields["traffic_bytes_per_launch"]:
            if entry[0] == op:
                return int(entry[1])
    except (KeyError, IndexError, OSError, ValueError):
        return None
    return None


def parse_args(argv=None):
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--log2n", type=int, default=28, help="log2 of the pair count (default 28)")
    p.add_argument("--seed", type=int, default=115002)
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="target duration of the CPU-baseline sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--dot-cfg", default=None,
                   help="block,chunk,grid,unroll of the batched dot (for example 256,4096,0,16); "
                        "skips the autotuner (so that a profile holds only launches of this "
                        "shape)")
    p.add_argument("--no-secondary", action="store_true",
                   help="skip the batched-dot, Horner, GEMM, matvec, conversion and single-dot "
                        "backward measurements")
    return p.parse_args(argv)


def _time_launches(fn, reps: int, stream, warmup: int = 1) -> float:
    """Mean milliseconds per call of fn() over reps calls, HIP events on the
    launch stream (warmup untimed calls first)."""
    import torch

    for _ in range(warmup):
        fn()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def _oracle_timed(fn):
    """Seconds of one call of an oracle function (single-threaded C)."""
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def _host_threads() -> int:
    """Host threads for the CPU baseline: the CPUs this process may run on,
    at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _chunks(n: int, parts: int):
    """[lo, hi) bounds of `parts` near-equal contiguous pieces of range(n)."""
    return [(n * k // parts, n * (k + 1) // parts) for k in range(parts)]


def _oracle_parallel(tasks) -> tuple[float, int]:
    """Wall seconds to run the oracle calls `tasks` (zero-argument callables
    on disjoint pieces of one sample) on _host_threads() threads, and that
    thread count.  The oracle is unchanged: its C entry points release the
    interpreter lock, so the pieces run concurrently, like static chunks of a
    parallel loop."""
    from concurrent.futures import ThreadPoolExecutor

    threads = _host_threads()
    with ThreadPoolExecutor(threads) as pool:
        list(pool.map(lambda f: f(), [lambda: None] * threads))   # threads started
        t0 = time.perf_counter()
        list(pool.map(lambda f: f(), tasks))
        dt = time.perf_counter() - t0
    return dt, threads


def _baseline(value_mt, threads, value_st, unit, sample) -> dict:
    """The cpu_baseline object: the oracle on `threads` host threads, with the
    single-threaded rate of the same sample and the host's total logical CPU
    count beside it."""
    return {"value": value_mt, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": sample, "single_thread_value": value_st, "host_cpu": _host_cpu(),
            "host_cores_total": os.cpu_count()}


def secondary(stream, cpu: bool = True, dot_cfg=None) -> dict:
    """The other float-float workloads, one line each (not part of the step)."""
    import torch

    import ff_inputs as fi
    import paper_cs_0603115_amd as ff
    from paper_cs_0603115_amd import autotune

    dev = torch.device("cuda:0")
    out = {}

    n = 1 << 20
    log("[bench] ff_add / ff_mul on 2^20 base pairs, cache-warm and after a cache flush")
    a = fi.base_ff(n, 115001, device=dev)
    b = fi.base_ff(n, 115011, device=dev)
    r = ff.ff_empty((n,), device=dev)
    # cache-flushed: 1 GiB written between launches evicts the 25 MB working
    # set from L2 and the 256 MB Infinity Cache; events bracket the operator's
    # own launch, queued behind the fill so that no host gap is timed
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    small = {}
    for name, fn in (("add", ff.ff_add), ("mul", ff.ff_mul)):
        # cache-warm: 200 launches captured in one graph and replayed, so that
        # the host's launch rate does not enter the time
        fn(a, b, out=r, stream=stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                cap = torch.cuda.current_stream(dev)
                for _ in range(200):
                    fn(a, b, out=r, stream=cap)
        torch.cuda.synchronize()
        warm_ms = min(_time_launches(graph.replay, 1, stream) for _ in range(3)) / 200
        del graph
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(20)]
        for s_ev, e_ev in evs:
            flush.zero_()
            s_ev.record(stream)
            fn(a, b, out=r, stream=stream)
            e_ev.record(stream)
        torch.cuda.synchronize()
        cold_ms = sum(s_ev.elapsed_time(e_ev) for s_ev, e_ev in evs) / len(evs)
        small[name] = {"warm_us": round(warm_ms * 1e3, 2), "warm_ff_ops/s": n / (warm_ms * 1e-3),
                       "flushed_us": round(cold_ms * 1e3, 2),
                       "flushed_ff_ops/s": n / (cold_ms * 1e-3)}
    out["elementwise_2p20"] = small
    del a, b, r, flush
    torch.cuda.empty_cache()

    n, deg = 1 << 26, 25
    log(f"[bench] polynomial evaluation: (x - 1)^{deg} expanded at 2^26 points")
    coef = fi.binomial_poly(deg).to(dev)
    x = fi.horner_points(n, 115041, 0.75, 1.25, device=dev)
    y = torch.empty_like(x)
    yff = ff.ff_empty((n,), device=dev)
    horner = {"points": n, "degree": deg}
    # floating-point operations per point and degree: mul + add; TwoProd 2 +
    # TwoSum 6 + correction 3; Mul22 12 + Add22 11
    for name, fn, per_step in (
            ("horner_f32", lambda: ff.ff_horner_f32(coef, x, out=y, stream=stream), 2),
            ("horner_comp", lambda: ff.ff_horner_comp(coef, x, out=y, stream=stream), 11),
            ("horner_ff", lambda: ff.ff_horner_ff(coef, x, out=yff, stream=stream,
                                                  ff_points=False), 23)):
        # ALU-bound: ~100 ms of the same launches first, so that the clock
        # has ramped up before the timed ones
        ms = _time_launches(fn, 50, stream, warmup=max(10, int(0.1 / (per_step * deg * n / ALU_PEAK_OPS))))
        ops = per_step * deg * n / (ms * 1e-3)
        horner[name] = {"ms": round(ms, 4), "Gpoints/s": round(n / (ms * 1e-3) / 1e9, 2),
                        "fp32_ops/s": ops, "alu_frac": round(ops / ALU_PEAK_OPS, 4)}
    if cpu:
        import oracle
        m = 1 << 23
        xs, cs = x[:m].cpu().numpy(), coef.cpu().numpy()
        dt = _oracle_timed(lambda: oracle.horner_comp(cs, xs))
        xa = x.cpu().numpy()
        dtp, th = _oracle_parallel([lambda lo=lo, hi=hi: oracle.horner_comp(cs, xa[lo:hi])
                                    for lo, hi in _chunks(n, 4 * _host_threads())])
        horner["cpu_baseline"] = _baseline(
            n / dtp, th, m / dt, "points/s (compensated Horner)",
            f"all {n} points in {4 * th} contiguous pieces, C oracle on {th} host threads, "
            f"{dtp:.2f} s (one thread: first {m} points, {dt:.2f} s)")
    out["horner_2p26"] = horner
    del coef, x, y, yff
    torch.cuda.empty_cache()

    log("[bench] batched dot: 4096 vectors, lengths floor(2^U[6,20])")
    x, y, offs = fi.batched_dot(115003, device=dev)
    total = x.numel()
    cfg = tuple(dot_cfg) if dot_cfg is not None else autotune.dot_cfg(x, y, offs)
    res = ff.ff_empty((offs.numel() - 1,), device=dev)
    # large enough for the tuned shape and for every entry point's default
    ws = torch.empty(max(ff.ff_dot_batched_workspace_size(total, offs.numel() - 1, cfg),
                         ff.ff_dot_batched_workspace_size(total, offs.numel() - 1)),
                     dtype=torch.uint8, device=dev)
    ms = _time_launches(lambda: ff.ff_dot_batched(x, y, offs, cfg=cfg, out=res, workspace=ws,
                                                  stream=stream), 10, stream)
    gbs = 8 * total / (ms * 1e-3) / 1e9
    ms2 = _time_launches(lambda: ff.ff_dot2_batched(x, y, offs, cfg=cfg, out=res, workspace=ws,
                                                    stream=stream), 10, stream)
    gbs2 = 8 * total / (ms2 * 1e-3) / 1e9
    # backward for per-vector gradients: reads x and y (binary32), writes dx
    # and dy (float-float): 24 bytes per element
    gvec = torch.ones((2, offs.numel() - 1), device=dev)
    gvec[1].zero_()
    dxb, dyb = ff.ff_empty((total,), device=dev), ff.ff_empty((total,), device=dev)
    wsb = torch.empty(ff.ff_dot_batched_backward_workspace_size(total), dtype=torch.uint8,
                      device=dev)
    msb = _time_launches(lambda: ff.ff_dot_batched_backward(gvec, x, y, offs, dx_out=dxb, dy_out=dyb,
                                                            workspace=wsb, stream=stream),
                         10, stream)
    gbsb = 24 * total / (msb * 1e-3) / 1e9
    del dxb, dyb, gvec, wsb
    # the other entry points of the family on the same batch, each with its
    # default launch shape: float-float inputs (16 B per element), sums of
    # binary32 (4 B) and of float-float (8 B) terms
    xf = torch.stack([x, torch.zeros_like(x)])
    yf = torch.stack([y, torch.zeros_like(y)])
    family = {}
    for name, fn, bpe in (
            ("dot_ff_inputs", lambda: ff.ff_dot_ff_batched(xf, yf, offs, out=res,
                                                           workspace=ws, stream=stream), 16),
            ("sum_f32", lambda: ff.ff_sum_batched(x, offs, out=res, workspace=ws,
                                                  stream=stream), 4),
            ("sum_ff", lambda: ff.ff_sum_ff_batched(xf, offs, out=res, workspace=ws,
                                                    stream=stream), 8)):
        msf = _time_launches(fn, 10, stream)
        gbf = bpe * total / (msf * 1e-3) / 1e9
        family[name] = {"ms": round(msf, 4), "GB/s": round(gbf, 1),
                        "hbm_frac": round(gbf / HBM_PEAK_GBS, 4), "bytes_per_element": bpe}
    del xf, yf
    out["dot_batched"] = {"elements": total, "ms": round(ms, 4), "elements/s": total / (ms * 1e-3),
                          "GB/s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                          "cfg": list(cfg),
                          "dot2_compensated": {"ms": round(ms2, 4), "GB/s": round(gbs2, 1),
                                               "hbm_frac": round(gbs2 / HBM_PEAK_GBS, 4)},
                          "backward": {"ms": round(msb, 4), "GB/s": round(gbsb, 1),
                                       "hbm_frac": round(gbsb / HBM_PEAK_GBS, 4),
                                       "bytes_per_element": 24},
                          "family": family}
    if cpu:
        import oracle
        offs_h = offs.cpu().numpy()
        nv = int((offs_h <= 150_000_000).sum()) - 1         # whole vectors, ~150 M elements
        e = int(offs_h[nv])
        xs, ys = x[:e].cpu().numpy(), y[:e].cpu().numpy()
        dt = _oracle_timed(lambda: oracle.dot_seq_batched(xs, ys, offs_h[:nv + 1]))
        del xs, ys
        xa, ya = x.cpu().numpy(), y.cpu().numpy()
        nall = offs_h.size - 1

        def piece(v0, v1):
            o0, o1 = int(offs_h[v0]), int(offs_h[v1])
            return lambda: oracle.dot_seq_batched(xa[o0:o1], ya[o0:o1], offs_h[v0:v1 + 1] - o0)

        dtp, th = _oracle_parallel([piece(v0, v1) for v0, v1 in _chunks(nall, 4 * _host_threads())])
        out["dot_batched"]["cpu_baseline"] = _baseline(
            total / dtp, th, e / dt, "elements/s",
            f"all {nall} vectors ({total} elements), sequential Add22 dot per vector, vectors "
            f"in {4 * th} pieces, C oracle on {th} host threads, {dtp:.2f} s (one thread: "
            f"first {nv} vectors, {e} elements, {dt:.2f} s)")
        # the backward on the same batch: per-vector gradients (1, 0), as timed above
        import numpy as np
        g1, g0 = np.ones(nall, np.float32), np.zeros(nall, np.float32)
        zs = np.zeros(e, np.float32)
        dt = _oracle_timed(lambda: oracle.dot_batched_backward(
            g1[:nv], g0[:nv], offs_h[:nv + 1], xa[:e], zs, ya[:e], zs))
        del zs

        def bpiece(v0, v1):
            o0, o1 = int(offs_h[v0]), int(offs_h[v1])
            z = np.zeros(o1 - o0, np.float32)
            return lambda: oracle.dot_batched_backward(g1[v0:v1], g0[v0:v1],
                                                       offs_h[v0:v1 + 1] - o0, xa[o0:o1], z,
                                                       ya[o0:o1], z)

        dtp, th = _oracle_parallel([bpiece(v0, v1) for v0, v1 in _chunks(nall, 4 * _host_threads())])
        out["dot_batched"]["backward"]["cpu_baseline"] = _baseline(
            total / dtp, th, e / dt, "elements/s",
            f"all {nall} vectors ({total} elements), dx and dy by Mul22 per element, vectors "
            f"in {4 * th} pieces, C oracle on {th} host threads, {dtp:.2f} s (one thread: "
            f"first {nv} vectors, {e} elements, {dt:.2f} s)")
        del xa, ya
    del x, y, offs, res, ws
    torch.cuda.empty_cache()

    n = 4096
    log(f"[bench] ff GEMM {n}^3: sliced int8, sliced BF16, FMA loop")
    A = fi.gaussian_ff((n, n), 115004, device=dev)
    B = fi.gaussian_ff((n, n), 115014, device=dev)
    C = ff.ff_empty((n, n), device=dev)
    flops = 2.0 * n * n * n
    gemm = {}
    for name, algo, reps, rough_ms in (("sliced_i8", ff.GEMM_SLICED_I8, 5, 2.0),
                                       ("sliced_bf16", ff.GEMM_SLICED_BF16, 5, 3.5),
                                       ("fma_loop", ff.GEMM_FMA_LOOP, 2, 30.0)):
        wsg = torch.empty(max(ff.ff_gemm_workspace_size(n, n, n, algo), 1), dtype=torch.uint8,
                          device=dev)
        # matrix-core clocks ramp up under load: ~100 ms of the same calls first
        # (the CPU baselines before this line leave the GPU idle for seconds)
        ms = _time_launches(lambda: ff.ff_gemm(A, B, algo=algo, out=C, workspace=wsg,
                                               stream=stream), reps, stream,
                            warmup=max(3, int(0.1 / (rough_ms * 1e-3))))
        gemm[name] = {"ms": round(ms, 3), "ff_TFLOP/s": round(flops / (ms * 1e-3) / 1e12, 2)}
        del wsg
    gemm["speedup_i8_vs_fma_loop"] = round(gemm["fma_loop"]["ms"] / gemm["sliced_i8"]["ms"], 1)
    gemm["speedup_bf16_vs_fma_loop"] = round(gemm["fma_loop"]["ms"] / gemm["sliced_bf16"]["ms"], 1)
    if cpu:
        import oracle
        r = 192
        Ah, Al = A[0, :r].cpu().numpy(), A[1, :r].cpu().numpy()
        Bh, Bl = B[0, :, :r].contiguous().cpu().numpy(), B[1, :, :r].contiguous().cpu().numpy()
        dt = _oracle_timed(lambda: oracle.gemm_ff_seq(Ah, Al, Bh, Bl))
        th = _host_threads()
        rp = r * th                                           # 192 rows of C per thread
        Aph, Apl = A[0, :rp].cpu().numpy(), A[1, :rp].cpu().numpy()
        dtp, th = _oracle_parallel([lambda lo=lo, hi=hi: oracle.gemm_ff_seq(Aph[lo:hi], Apl[lo:hi], Bh, Bl)
                                    for lo, hi in _chunks(rp, th)])
        rate, rate1 = 2.0 * rp * r * n / dtp, 2.0 * r * r * n / dt
        gemm["cpu_baseline"] = _baseline(
            rate / 1e12, th, rate1 / 1e12, "ff_TFLOP/s",
            f"{rp} x {r} block of C at K = {n} (plain Add22/Mul22 loop), rows in {th} pieces, "
            f"C oracle on {th} host threads, {dtp:.2f} s (one thread: {r} x {r}, {dt:.2f} s); "
            f"4096^3 would take {flops / rate:.0f} s")
    out["gemm_4096"] = gemm
    del A, B, C
    torch.cuda.empty_cache()

    m = 8192
    log(f"[bench] ff matvec {m}^2 forward and backward (fast vs plain)")
    A = fi.gaussian_ff((m, m), 115005, device=dev)
    xv = fi.gaussian_ff((m,), 115006, device=dev)
    g = torch.stack([fi.gaussian_f32((m,), 115007, device=dev), torch.zeros(m, device=dev)])
    # outputs and workspace allocated once, outside the timed calls
    yv, dA, dxv = ff.ff_empty((m,), device=dev), ff.ff_empty((m, m), device=dev), ff.ff_empty((m,), device=dev)
    mv = {}
    for name, algo in (("fast", ff.MATVEC_FAST), ("plain", ff.MATVEC_PLAIN)):
        wsm = torch.empty(max(ff.ff_matvec_backward_workspace_size(m, m, algo), 16),
                          dtype=torch.uint8, device=dev)
        fwd = _time_launches(lambda: ff.ff_matvec(A, xv, algo=algo, out=yv, stream=stream), 10, stream)
        bwd = _time_launches(lambda: ff.ff_matvec_backward(A, xv, g, algo=algo, dA_out=dA, dx_out=dxv,
                                                           workspace=wsm, stream=stream),
                             5, stream)
        del wsm
        mv[name] = {"forward_ms": round(fwd, 4), "backward_ms": round(bwd, 4),
                    "forward_GB/s": round(8 * m * m / (fwd * 1e-3) / 1e9, 1),
                    "backward_GB/s": round(16 * m * m / (bwd * 1e-3) / 1e9, 1)}
    mv["backward_speedup_fast_vs_plain"] = round(mv["plain"]["backward_ms"] / mv["fast"]["backward_ms"], 1)
    mv["forward_speedup_fast_vs_plain"] = round(mv["plain"]["forward_ms"] / mv["fast"]["forward_ms"], 1)
    if cpu:
        import oracle
        r = m
        Ah, Al = A[0, :r].cpu().numpy(), A[1, :r].cpu().numpy()
        xh, xl = xv[0].cpu().numpy().reshape(m, 1), xv[1].cpu().numpy().reshape(m, 1)
        dt = _oracle_timed(lambda: oracle.gemm_ff_seq(Ah, Al, xh, xl))
        dtp, th = _oracle_parallel([lambda lo=lo, hi=hi: oracle.gemm_ff_seq(Ah[lo:hi], Al[lo:hi], xh, xl)
                                    for lo, hi in _chunks(r, 4 * _host_threads())])
        mv["cpu_baseline"] = _baseline(
            8 * r * m / dtp / 1e9, th, 8 * r * m / dt / 1e9, "forward GB/s of A",
            f"all {r} rows of y = A x (sequential Add22 of Mul22 terms), rows in {4 * th} "
            f"pieces, C oracle on {th} host threads, {dtp:.2f} s ({dt:.2f} s on one)")
    out["matvec_8192"] = mv
    del A, xv, g, yv, dA, dxv
    torch.cuda.empty_cache()

    n = 1 << 28
    log("[bench] binary64 <-> float-float conversions at N = 2^28")
    xd = fi.gaussian_f32((n,), 115051, device=dev).double()
    pair = ff.ff_empty((n,), device=dev)
    back = torch.empty_like(xd)
    conv = {}
    for name, fn in (("from_f64", lambda: ff.ff_from_f64(xd, out=pair, stream=stream)),
                     ("to_f64", lambda: ff.ff_to_f64(pair, out=back, stream=stream))):
        ms = _time_launches(fn, 10, stream, warmup=2)
        gbs = 16 * n / (ms * 1e-3) / 1e9                # 8 B read + 8 B written per element
        conv[name] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["conversions_2p28"] = conv
    if cpu:
        import oracle
        xh = xd.cpu().numpy()
        m = 1 << 26
        dt = _oracle_timed(lambda: oracle.from_f64(xh[:m]))
        dtp, th = _oracle_parallel([lambda lo=lo, hi=hi: oracle.from_f64(xh[lo:hi])
                                    for lo, hi in _chunks(n, 4 * _host_threads())])
        conv["cpu_baseline"] = _baseline(
            n / dtp, th, m / dt, "elements/s (binary64 to float-float)",
            f"all {n} values in {4 * th} contiguous pieces, C oracle on {th} host threads, "
            f"{dtp:.2f} s (one thread: first {m} values, {dt:.2f} s)")
        del xh
    del xd, pair, back
    torch.cuda.empty_cache()

    log("[bench] single-dot backward at N = 2^28 (float-float x and y)")
    xs = fi.gaussian_ff((n,), 115061, device=dev)
    ys = fi.gaussian_ff((n,), 115062, device=dev)
    gs = torch.tensor([[0.75], [2.0 ** -30]], dtype=torch.float32, device=dev)
    dxs, dys = ff.ff_empty((n,), device=dev), ff.ff_empty((n,), device=dev)
    ms = _time_launches(lambda: ff.ff_dot_backward(gs, xs, ys, dx_out=dxs, dy_out=dys,
                                                   stream=stream), 10, stream, warmup=2)
    gbs = 32 * n / (ms * 1e-3) / 1e9                    # x, y read; dx, dy written: 4 planes each
    out["dot_backward_2p28"] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_element": 32}
    del xs, ys, gs, dxs, dys
    torch.cuda.empty_cache()
    return out


def cpu_baseline(a, b, target_s: float):
    """Oracle throughput (ff ops/s) on a bounded prefix of the same inputs."""
    import numpy as np

    import oracle

    n_total = a.shape[1]
    probe = min(1 << 20, n_total)
    ah, al, bh, bl = (t.cpu().numpy() for t in (a[0, :probe], a[1, :probe], b[0, :probe], b[1, :probe]))
    t0 = time.perf_counter()
    for op in OPS:
        oracle.elementwise(op, ah, al, bh, bl)
    per_elem = (time.perf_counter() - t0) / probe
    n = int(min(n_total, max(probe, target_s / max(per_elem, 1e-12))))
    n -= n % 4
    ah, al, bh, bl = (np.ascontiguousarray(t.cpu().numpy())
                      for t in (a[0, :n], a[1, :n], b[0, :n], b[1, :n]))
    rh, rl = np.empty(n, np.float32), np.empty(n, np.float32)
    t0 = time.perf_counter()
    for op in OPS:
        oracle.elementwise(op, ah, al, bh, bl, out=(rh, rl))
    dt = time.perf_counter() - t0

    def piece(lo, hi):
        def run():
            for op in OPS:
                oracle.elementwise(op, ah[lo:hi], al[lo:hi], bh[lo:hi], bl[lo:hi],
                                   out=(rh[lo:hi], rl[lo:hi]))
        return run

    dtp, th = _oracle_parallel([piece(lo, hi) for lo, hi in _chunks(n, _host_threads())])
    return _baseline(
        4 * n / dtp, th, 4 * n / dt, "ff ops/s",
        f"first {n} of the {n_total} pairs, ops add/sub/mul/div once each ({4 * n} ff ops), "
        f"pairs in {th} contiguous pieces, C oracle on {th} host threads, {dtp:.2f} s "
        f"({dt:.2f} s on one)")


def main(argv=None) -> int:
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the float-float operators need no inter-GPU exchange: run one process per GPU "
              "on independent shards)", file=sys.stderr)
        return 2

    import torch

    import ff_inputs as fi
    import paper_cs_0603115_amd as ff

    if not torch.cuda.is_available():
        log("bench.py needs a HIP device")
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 1 << args.log2n
    log(f"[bench] generating {n} mixed float-float pairs on {torch.cuda.get_device_name(dev)}")
    a, b, _ = fi.mixed_ff_pair(n, args.seed, device=dev)
    r = ff.ff_empty((n,), device=dev)
    torch.cuda.synchronize()
    fns = {"add": ff.ff_add, "sub": ff.ff_sub, "mul": ff.ff_mul, "div": ff.ff_div}
    stream = torch.cuda.current_stream()

    def step(events=None, k=0):
        for op in OPS:
            if events is not None:
                events[op][k][0].record(stream)
            fns[op](a, b, out=r, stream=stream)
            if events is not None:
                events[op][k][1].record(stream)

    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = {op: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)] for op in OPS}
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events, k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps

    kernel_ms = {op: sum(s.elapsed_time(e) for s, e in events[op]) / args.steps for op in OPS}

    # Bandwidth reference: the ff_copy probe (one plane in, one out; 512
    # threads by 4 lane-contiguous elements, non-temporal, the fastest copy
    # pattern measured) over N binary32 words, after the timed region.  It
    # also calibrates the HBM byte counters.
    copy_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    for s_ev, e_ev in copy_ev:
        s_ev.record(stream)
        ff.ff_copy(a[0], r[0], stream=stream)
        e_ev.record(stream)
    torch.cuda.synchronize()
    copy_ms = sum(s.elapsed_time(e) for s, e in copy_ev) / args.steps
    copy_gbs = 8 * n / (copy_ms * 1e-3) / 1e9
    # The tighter-bound operators on the same pairs (not part of the step).
    accurate = {}
    for name, fn in (("add", ff.ff_add_accurate), ("mul", ff.ff_mul_accurate),
                     ("div", ff.ff_div_accurate)):
        acc_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
        for s_ev, e_ev in acc_ev:
            s_ev.record(stream)
            fn(a, b, out=r, stream=stream)
            e_ev.record(stream)
        torch.cuda.synchronize()
        acc_ms = sum(s.elapsed_time(e) for s, e in acc_ev) / args.steps
        accurate[name] = {"ms": round(acc_ms, 5),
                          "GB/s": round(BYTES_PER_FF_OP * n / (acc_ms * 1e-3) / 1e9, 1),
                          "ff ops/s": n / (acc_ms * 1e-3)}
    per_op = {op: {"ms": round(kernel_ms[op], 5),
                   "GB/s": round(BYTES_PER_FF_OP * n / (kernel_ms[op] * 1e-3) / 1e9, 1)}
              for op in OPS}
    dominant = max(OPS, key=lambda op: kernel_ms[op])
    achieved = BYTES_PER_FF_OP * n / (kernel_ms[dominant] * 1e-3) / 1e9
    log(f"[bench] per-op kernel times: {per_op}")

    result = {
        "metric": "ff ops/s (elementwise add/sub/mul/div, mixed workload)",
        "value": 4 * n / (ms_per_step * 1e-3),
        "unit": "ff ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; 65% base +-2^U[-20,20], 25% cancellation, 10% exponent gap)",
        "config": {"workload": f"elementwise ff add/sub/mul/div on N=2^{args.log2n} SoA hi/lo pairs",
                   "format": "float-float: binary32 hi + lo, computed in binary32 arithmetic",
                   "n": n, "ops_per_step": 4, "seed": args.seed},
        "roofline": {
            "bound": "hbm",
            "kernel": f"ff_{dominant}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(dominant, n),
            "traffic_source": os.path.relpath(PROFILE_SUMMARY, _ROOT),
        },
        "per_op": per_op,
        "copy_probe": {"ms": round(copy_ms, 5), "GB/s": round(copy_gbs, 1),
                       "bytes": 8 * n, "dominant_frac_of_copy": round(achieved / copy_gbs, 4)},
        "accurate_ops": accurate,
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle) on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(a, b, args.cpu_seconds)
    if not args.no_secondary:
        del a, b, r
        torch.cuda.empty_cache()
        dot_cfg = None
        if args.dot_cfg:
            dot_cfg = tuple(int(v) for v in args.dot_cfg.split(","))
            if len(dot_cfg) != 4:
                raise SystemExit("--dot-cfg takes four integers: block,chunk,grid,unroll")
        result["secondary"] = secondary(stream, cpu=not args.no_cpu_baseline, dot_cfg=dot_cfg)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
