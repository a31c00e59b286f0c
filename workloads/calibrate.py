"""Writes ``workloads/calibration.json`` by calling the oracle only.

The 100k-point mixture workload fixes its Wendland radius r0 so that rows
hold about 50 nonzeros on average: bisection on r0 (bump radius fixed at
0.02, 4 x 4 bumps) until the realised mean row length of the oracle's
pattern lies in [49.5, 50.5].

Run:  python -m workloads.calibrate
"""
from __future__ import annotations

import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import kernel  # noqa: E402
from workloads import gmm_problem  # noqa: E402


def mean_row(r0: float) -> float:
    p = gmm_problem(100_000, 2, r0, 0.02)
    indptr, cols, vals = kernel.sparse(p.x, p.theta)
    return float(indptr[-1]) / p.n


def main():
    lo, hi = 0.003, 0.02
    r0 = 0.5 * (lo + hi)
    for it in range(40):
        r0 = 0.5 * (lo + hi)
        m = mean_row(r0)
        print(f"iter {it}: r0 = {r0:.8f}  mean nnz/row = {m:.3f}", flush=True)
        if 49.5 <= m <= 50.5:
            break
        if m < 50.0:
            lo = r0
        else:
            hi = r0
    out = dict(cfg2_r0=round(r0, 8), cfg2_mean_row=round(m, 3),
               note="bisection on r0 with bump radius 0.02; written by workloads/calibrate.py")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "calibration.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
