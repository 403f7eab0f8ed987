"""Benchmark of the float-float hot path on one MI355X.

One step = the full elementwise operator set (ff_add, ff_sub, ff_mul, ff_div)
over N = 2^28 float-float pairs of the mixed workload (25 % cancellation and
10 % exponent-gap pairs), inputs resident in HBM.  The metric is float-float
operations per second (4 N per step).

Printed: ONE JSON line on stdout, with
  * ``roofline`` for the dominant kernel (algorithmic bytes / average launch
    time from HIP events recorded on the launch stream, against 8 TB/s),
  * ``cpu_baseline``: the oracle (single-threaded C) timed on this host on a
    bounded sample of the same inputs.
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
OPS = ["add", "sub", "mul", "div"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


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
    return p.parse_args(argv)


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
    return {
        "value": 4 * n / dt,
        "unit": "ff ops/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {n} of the {n_total} pairs, ops add/sub/mul/div once each "
                  f"({4 * n} ff ops in {dt:.2f} s, single-threaded C oracle)",
    }


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

    # Bandwidth reference: the ff_copy probe (one plane in, one out, same
    # 16-byte non-temporal pattern) over N binary32 words, after the timed
    # region.  It also calibrates the HBM byte counters.
    copy_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    for s_ev, e_ev in copy_ev:
        s_ev.record(stream)
        ff.ff_copy(a[0], r[0], stream=stream)
        e_ev.record(stream)
    torch.cuda.synchronize()
    copy_ms = sum(s.elapsed_time(e) for s, e in copy_ev) / args.steps
    copy_gbs = 8 * n / (copy_ms * 1e-3) / 1e9
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
        "dtype": "f32x2 (float-float: binary32 hi + lo)",
        "data": "synthetic (seeded; 65% base +-2^U[-20,20], 25% cancellation, 10% exponent gap)",
        "config": {"workload": f"elementwise ff add/sub/mul/div on N=2^{args.log2n} SoA hi/lo pairs",
                   "n": n, "ops_per_step": 4, "seed": args.seed},
        "roofline": {
            "bound": "hbm",
            "kernel": f"ff_{dominant}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "per_op": per_op,
        "copy_probe": {"ms": round(copy_ms, 5), "GB/s": round(copy_gbs, 1),
                       "bytes": 8 * n, "dominant_frac_of_copy": round(achieved / copy_gbs, 4)},
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle) on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(a, b, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
