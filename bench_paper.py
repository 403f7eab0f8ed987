"""Timing table of the shape of the paper's Table 3 on one MI355X.

The paper (section 6) times binary32 Add, Mul and Mad next to Add12, Mul12,
Add22 and Mul22 on streams of 2^12 .. 2^20 elements, each normalised to the
time of 4096 binary32 additions on the same device.  This script times the
library's kernels on device-resident data (no host transfers; the paper's
timings included them): R launches of one operator are captured into one HIP
graph, so that the host-side cost of issuing a launch from Python drops out,
and the graph replay is timed with HIP events (best of 3 replays).  It prints
one JSON object per (operator, size) and a table.

  python bench_paper.py [--sizes 12,14,16,18,20,22,24,26] [--reps 200]

Inputs: binary32 x = +-2^t, t ~ U[-20, 20] (the high words of the base
float-float generator, seeds 115031 / 115032 / 115033); float-float operands
from the same generator.  Each launch's algorithmic bytes: Add / Mul 12,
Mad / Add12 / Mul12 16, the float-float operators 24 per element.
"""
from __future__ import annotations

import argparse
import json
import sys

OPS = ["Add", "Mul", "Mad", "Add12", "Mul12 (FMA)", "Mul12 (Dekker)", "Add22", "Mul22",
       "Mul22 (Dekker)", "Div22", "Add22 (accurate)", "Mul22 (accurate)", "Div22 (accurate)"]
BYTES = {"Add": 12, "Mul": 12, "Mad": 16, "Add12": 16, "Mul12 (FMA)": 16, "Mul12 (Dekker)": 16,
         "Add22": 24, "Mul22": 24, "Mul22 (Dekker)": 24, "Div22": 24, "Add22 (accurate)": 24,
         "Mul22 (accurate)": 24, "Div22 (accurate)": 24}


def main(argv=None) -> int:
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--sizes", default="12,14,16,18,20,22,24,26",
                   help="comma-separated log2 stream sizes")
    p.add_argument("--reps", type=int, default=200, help="timed launches per point")
    args = p.parse_args(argv)

    import torch

    import ff_inputs as fi
    import paper_cs_0603115_amd as ff

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sizes = [int(s) for s in args.sizes.split(",")]
    nmax = 1 << max(sizes)
    A = fi.base_ff(nmax, 115031, device=dev)
    B = fi.base_ff(nmax, 115032, device=dev)
    C = fi.base_ff(nmax, 115033, device=dev)[0].contiguous()
    a, b = A[0].contiguous(), B[0].contiguous()
    R = ff.ff_empty((nmax,), device=dev)
    r1 = torch.empty(nmax, dtype=torch.float32, device=dev)

    def launcher(op, n):
        av, bv, cv, rv = a[:n], b[:n], C[:n], r1[:n]
        Av, Bv = A[:, :n], B[:, :n]
        Rv = R[:, :n]
        return {
            "Add": lambda st=stream: ff.f32_add(av, bv, out=rv, stream=st),
            "Mul": lambda st=stream: ff.f32_mul(av, bv, out=rv, stream=st),
            "Mad": lambda st=stream: ff.f32_mad(av, bv, cv, out=rv, stream=st),
            "Add12": lambda st=stream: ff.ff_add12(av, bv, out=Rv, stream=st),
            "Mul12 (FMA)": lambda st=stream: ff.ff_mul12(av, bv, out=Rv, stream=st),
            "Mul12 (Dekker)": lambda st=stream: ff.ff_mul12(av, bv, dekker=True, out=Rv, stream=st),
            "Add22": lambda st=stream: ff.ff_add(Av, Bv, out=Rv, stream=st),
            "Mul22": lambda st=stream: ff.ff_mul(Av, Bv, out=Rv, stream=st),
            "Mul22 (Dekker)": lambda st=stream: ff.ff_mul_dekker(Av, Bv, out=Rv, stream=st),
            "Div22": lambda st=stream: ff.ff_div(Av, Bv, out=Rv, stream=st),
            "Add22 (accurate)": lambda st=stream: ff.ff_add_accurate(Av, Bv, out=Rv, stream=st),
            "Mul22 (accurate)": lambda st=stream: ff.ff_mul_accurate(Av, Bv, out=Rv, stream=st),
            "Div22 (accurate)": lambda st=stream: ff.ff_div_accurate(Av, Bv, out=Rv, stream=st),
        }[op]

    # the first n words of each plane: every plane of A[:, :n] is contiguous
    results = {}
    for lg in sizes:
        n = 1 << lg
        for op in OPS:
            call = launcher(op, n)
            call()
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream(dev)
            side.wait_stream(stream)
            with torch.cuda.stream(side):
                with torch.cuda.graph(graph, stream=side):
                    cap = torch.cuda.current_stream(dev)
                    for _ in range(args.reps):
                        call(cap)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                graph.replay()
                e1.record(stream)
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e3 / args.reps)
            results[(op, lg)] = best
            del graph
        print(f"[paper-table] 2^{lg} done", file=sys.stderr, flush=True)

    ref = results[("Add", 12)] if ("Add", 12) in results else results[("Add", sizes[0])]
    for lg in sizes:
        n = 1 << lg
        for op in OPS:
            us = results[(op, lg)]
            print(json.dumps({"table": "paper_table3_shape", "op": op, "n": n, "us_per_launch": round(us, 3),
                              "normalised_to_add_4096": round(us / ref, 3),
                              "GB/s": round(BYTES[op] * n / (us * 1e-6) / 1e9, 1)}))
    print("\n| size | " + " | ".join(OPS) + " |", file=sys.stderr)
    print("|---|" + "---|" * len(OPS), file=sys.stderr)
    for lg in sizes:
        cells = " | ".join(f"{results[(op, lg)] / ref:.2f}" for op in OPS)
        print(f"| 2^{lg} | {cells} |", file=sys.stderr)
    print(f"\n(1.00 = {ref:.2f} us, one binary32 Add launch over 4096 elements)", file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
