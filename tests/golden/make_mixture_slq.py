"""Writes mixture_n100000_slq.json: the oracle's stochastic Lanczos quadrature
estimate of log det K for the 100,000-point mixture workload
(``workloads.config2``), with the probes the library draws for the default
seed (SplitMix64 Rademacher probes keyed by the original point index), 30
probes x 50 plain Lanczos steps on the Jacobi-scaled matrix, breakdown below
1e-10 (``oracle.slq.slq_logdet`` on ``oracle.kernel.sparse``), plus the
per-probe quadratures; then the same with full re-orthogonalisation of every
residual against all Lanczos vectors (``reorth``).

Calls only oracle/ and the seeded input generator.  About a minute.
Usage: python tests/golden/make_mixture_slq.py"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import kernel, slq  # noqa: E402
from workloads import config2  # noqa: E402

SEED = 0x5EED     # the library's default probe seed
PROBES, STEPS = 30, 50


def main():
    p = config2()
    t0 = time.time()
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    r = slq.slq_logdet(A, SEED, PROBES, STEPS, 1e-10)
    ro = slq.slq_logdet(A, SEED, PROBES, STEPS, 1e-10, reorth=True)
    out = dict(workload=p.name, n=int(p.n), seed=SEED, probes=PROBES, steps=STEPS, method="oracle.slq.slq_logdet",
               logdet=r["logdet"], se=r["se"], jacobi=r["jacobi"], gammas=[float(g) for g in r["gammas"]],
               probe_steps=[int(k) for k in r["steps"]],
               reorth=dict(logdet=ro["logdet"], se=ro["se"], gammas=[float(g) for g in ro["gammas"]],
                           probe_steps=[int(k) for k in ro["steps"]]),
               seconds=round(time.time() - t0, 1))
    path = os.path.join(HERE, "mixture_n100000_slq.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({k: v for k, v in out.items() if k not in ("gammas", "probe_steps", "reorth")}),
          out["reorth"]["logdet"])


if __name__ == "__main__":
    main()
