"""Writes spacetime_n1095000_slq.json: the oracle's stochastic Lanczos
quadrature estimate of log det K for the space-time workload (3000 stations x
365 days, ``workloads.config3``) with the probes the benchmark draws (seed
2411: SplitMix64 Rademacher probes keyed by the original point index), 30
probes x 80 Lanczos steps on the Jacobi-scaled matrix, breakdown below 1e-10
(``oracle.slq.slq_logdet`` on ``oracle.kernel.sparse``): plain Lanczos, then
with full re-orthogonalisation (``reorth``); per-probe quadratures of both.

Calls only oracle/ and the seeded input generator.  About half an hour on one
core.  Usage: python tests/golden/make_spacetime_slq.py"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import kernel, slq  # noqa: E402
from workloads import config3  # noqa: E402

SEED = 2411
PROBES, STEPS = 30, 80


def main():
    p = config3()
    t0 = time.time()
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    t1 = time.time()
    r = slq.slq_logdet(A, SEED, PROBES, STEPS, 1e-10)
    t2 = time.time()
    ro = slq.slq_logdet(A, SEED, PROBES, STEPS, 1e-10, reorth=True)
    out = dict(workload=p.name, n=int(p.n), nnz=int(A.nnz), seed=SEED, probes=PROBES, steps=STEPS,
               method="oracle.slq.slq_logdet", logdet=r["logdet"], se=r["se"], jacobi=r["jacobi"],
               gammas=[float(g) for g in r["gammas"]], probe_steps=[int(k) for k in r["steps"]],
               reorth=dict(logdet=ro["logdet"], se=ro["se"], gammas=[float(g) for g in ro["gammas"]],
                           probe_steps=[int(k) for k in ro["steps"]]),
               seconds=dict(matrix=round(t1 - t0, 1), plain=round(t2 - t1, 1), reorth=round(time.time() - t2, 1)))
    path = os.path.join(HERE, "spacetime_n1095000_slq.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({k: v for k, v in out.items() if k not in ("gammas", "probe_steps", "reorth")}),
          out["reorth"]["logdet"])


if __name__ == "__main__":
    main()
