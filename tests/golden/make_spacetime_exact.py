"""Writes spacetime_n1095000_exact.json: the exact log det, quadratic form and
log-likelihood of the space-time workload (3000 stations x 365 days with its
hyper-parameters and observations y, ``workloads.config3``), computed by the
oracle's day-blocked split K = A + F F^T (block Cholesky of the local part,
matrix determinant lemma, Woodbury; ``oracle.likelihood.banded_split``).

Calls only oracle/ and the seeded input generator.  About 10 minutes on 8
cores.  Usage: python tests/golden/make_spacetime_exact.py"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import likelihood  # noqa: E402
from workloads import config3  # noqa: E402


def main():
    p = config3()
    t0 = time.time()
    r = likelihood.banded_split(p.x, p.theta, p.y)
    out = dict(workload=p.name, n=int(p.n), method="oracle.likelihood.banded_split",
               logdet=r["logdet"], quad=r["quad"], loglik=r["loglik"], logdet_A=r["logdet_A"],
               blocks=int(r["blocks"]), half_width=int(r["half_width"]), seconds=round(time.time() - t0, 1))
    path = os.path.join(HERE, "spacetime_n1095000_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
