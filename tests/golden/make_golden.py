"""Writes tests/golden/sweep_small.json from the oracle only (no HIP code).

Run:  python tests/golden/make_golden.py
Stored values: for a few seeded grids, the last row, last column and final
cell of the min and max sweeps in fp64 and fp32 (fp32 values stored as their
bit patterns), plus int32-input sweeps.  The test test_golden.py checks the
oracle still reproduces them, so any later change to the oracle's arithmetic
shows up as a diff here.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import wfgen  # noqa: E402

CASES = [(1, 1, 1), (1, 7, 13), (2, 64, 64), (3, 65, 129), (4, 100, 37), (5, 256, 300)]


def main():
    out = {"generator": "splitmix64, f32 = (x>>40)*2^-24, i32 = x&255", "cases": []}
    for seed, m, n in CASES:
        c = wfgen.cells(seed, m, n, "f32")
        ci = wfgen.cells(seed, m, n, "i32")
        case = {"seed": seed, "m": m, "n": n}
        for rule in ("min", "max"):
            lr, lc = oracle.sweep(c, rule, "f64", full=False)
            lr32, lc32 = oracle.sweep(c, rule, "f32", full=False)
            lri, lci = oracle.sweep(ci, rule, "i64", full=False)
            case[rule] = {
                "f64_last_row": [float(x) for x in lr],
                "f64_last_col": [float(x) for x in lc],
                "f32_last_row_bits": [int(x) for x in lr32.view(np.uint32)],
                "f32_last_col_bits": [int(x) for x in lc32.view(np.uint32)],
                "i64_last_row": [int(x) for x in lri],
                "i64_last_col": [int(x) for x in lci],
            }
        out["cases"].append(case)
    with open(os.path.join(HERE, "sweep_small.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
