"""Golden fixtures for the oracle.

* ``golden/hand_cases.txt``: cases whose outputs were derived by hand from
  the paper's operation sequences (each line carries its derivation).
* ``golden/oracle_regression.txt``: a bit-level lock written by
  ``golden/make_oracle_regression.py`` (oracle only); it catches changes of
  evaluation order, flags or rounding that the mathematical pins tolerate.
"""
import os

import numpy as np
import pytest

import oracle

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f(hexword: str) -> np.float32:
    return np.array([int(hexword, 16)], np.uint32).view(np.float32)[0]


def _rows(name):
    with open(os.path.join(_GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                yield [c.strip() for c in line.split("|")]


def _run(op, ins):
    a = [np.array([v], np.float32) for v in ins]
    if op == "add12":
        return oracle.add12(*a)
    if op == "split":
        return oracle.split(*a)
    if op == "mul12":
        return oracle.mul12(*a)
    if op == "horner_comp":
        # coefficients a0 .. an, then the point x
        return [oracle.horner_comp(np.concatenate(a[:-1]), a[-1])]
    return oracle.elementwise({"add22": "add", "mul22": "mul", "div22": "div"}.get(op, op), *a)


HAND = list(_rows("hand_cases.txt"))


@pytest.mark.parametrize("row", HAND, ids=[f"{r[0]}-{i}" for i, r in enumerate(HAND)])
def test_hand_derived_case(row):
    op, ins, outs, why = row
    got = _run(op, [_f(w) for w in ins.split()])
    want = [_f(w) for w in outs.split()]
    assert len(got) == len(want), (op, why)
    for g, w in zip(got, want):
        assert g[0].view(np.uint32) == w.view(np.uint32), (op, why, g[0], w)


def check_hand_cases(op: str) -> None:
    """Every hand-derived case of one operator (used by the mutation tests)."""
    rows = [r for r in HAND if r[0] == op]
    assert rows, op
    for row in rows:
        test_hand_derived_case(row)


def test_oracle_regression_lock():
    rows = list(_rows("oracle_regression.txt"))
    assert len(rows) == 1280
    by_op = {}
    for op, ins, outs in rows:
        by_op.setdefault(op, []).append(([int(w, 16) for w in ins.split()],
                                         [int(w, 16) for w in outs.split()]))
    for op, items in by_op.items():
        ins = np.array([i for i, _ in items], np.uint32).view(np.float32)
        want = np.array([o for _, o in items], np.uint32)
        rh, rl = oracle.elementwise(op, ins[:, 0], ins[:, 1], ins[:, 2], ins[:, 3])
        got = np.stack([rh.view(np.uint32), rl.view(np.uint32)], axis=1)
        assert np.array_equal(got, want), op
