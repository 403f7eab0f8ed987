"""Write ``oracle_regression.txt``: a bit-level lock on the oracle.

Inputs are drawn once from the seeded generators and stored as binary32 hex
bit patterns next to the oracle's outputs, so the file does not depend on
the generator's future behaviour.  Only ``oracle/`` computes the outputs.
Re-run this script only when a change of the oracle's arithmetic is
justified by the paper (the commit must say which passage).

    python tests/golden/make_oracle_regression.py
"""
import os
import sys

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, _ROOT)

import ff_inputs as fi  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.txt")
OPS = ["add", "sub", "mul", "mul_dekker", "div", "add_accurate", "mul_accurate", "div_accurate"]


def main():
    a, b, _ = fi.mixed_ff_pair(96, seed=424242)
    r1, r2 = fi.random_ff(64, 424243, -30, 30), fi.random_ff(64, 424244, -30, 30)
    ah = np.concatenate([a[0].numpy(), r1[0].numpy()])
    al = np.concatenate([a[1].numpy(), r1[1].numpy()])
    bh = np.concatenate([b[0].numpy(), r2[0].numpy()])
    bl = np.concatenate([b[1].numpy(), r2[1].numpy()])
    hx = lambda v: "%08x" % np.float32(v).view(np.uint32)
    lines = ["# op | ah al bh bl | rh rl   (binary32 hex; written by make_oracle_regression.py)"]
    for op in OPS:
        rh, rl = oracle.elementwise(op, ah, al, bh, bl)
        for i in range(ah.size):
            lines.append(f"{op} | {hx(ah[i])} {hx(al[i])} {hx(bh[i])} {hx(bl[i])} | "
                         f"{hx(rh[i])} {hx(rl[i])}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
