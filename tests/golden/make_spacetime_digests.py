"""Writes spacetime_n1095000_csr_digest.json: digests of the oracle's CSR of
the space-time workload (3000 stations x 365 days with its hyper-parameters,
``workloads.config3``), in original point order with ascending columns
(``oracle.kernel.sparse``: KD-tree candidates re-tested by the pinned float64
support predicate, plus the bump groups' member pairs):

* SHA-256 of row_ptr (int64, little-endian) and of the column ids (int32,
  little-endian): the pattern, bit for bit;
* per block of 1024 consecutive rows, the sum of the values and the sum of
  their magnitudes (float64), so that values can be compared within a
  relative bound per block.

Calls only oracle/ and the seeded input generator.  A few minutes on 8
cores, about 6 GB of memory.  Usage: python tests/golden/make_spacetime_digests.py"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import kernel  # noqa: E402
from workloads import config3  # noqa: E402

BLOCK = 1024


def block_sums(indptr, vals, block=BLOCK):
    n = indptr.shape[0] - 1
    starts = indptr[np.arange(0, n, block)]
    s = np.add.reduceat(vals, starts) if vals.size else np.zeros(starts.size)
    a = np.add.reduceat(np.abs(vals), starts) if vals.size else np.zeros(starts.size)
    return s, a


def main():
    p = config3()
    t0 = time.time()
    ip, ci, vo = kernel.sparse(p.x, p.theta)
    t1 = time.time()
    s, a = block_sums(ip, vo)
    out = dict(workload=p.name, n=int(p.n), nnz=int(ip[-1]), method="oracle.kernel.sparse",
               row_ptr_sha256=hashlib.sha256(np.ascontiguousarray(ip, "<i8").tobytes()).hexdigest(),
               col_sha256=hashlib.sha256(np.ascontiguousarray(ci, "<i4").tobytes()).hexdigest(),
               block=BLOCK, block_value_sums=[float(v) for v in s], block_abs_sums=[float(v) for v in a],
               seconds=round(t1 - t0, 1))
    path = os.path.join(HERE, "spacetime_n1095000_csr_digest.json")
    with open(path, "w") as f:
        json.dump(out, f)
        f.write("\n")
    print(json.dumps({k: v for k, v in out.items() if not k.startswith("block_")}))


if __name__ == "__main__":
    main()
