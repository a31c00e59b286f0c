"""The products over stale memory: the CSR column and value arrays carry 64
entries of padding that the products' four-wide loads can reach past the last
row, multiplied by a zero weight.  The padding must be zeroed at assembly, since
0 x NaN is NaN.

Set-up: PyTorch's cache of small blocks is first filled with NaN and released,
so the matrix arrays of a fresh context are carved from NaN-filled memory.  One
bump covers every point, so every row holds n = 301 group entries (301 is not
a multiple of four: the last row's loads run three entries past its end).  The
one- and multi-column products and a log-likelihood are checked against the
oracle's matrix, to the bounds of the product tests."""
import numpy as np
import pytest

from oracle import kernel, likelihood
from workloads import Problem, Theta
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _dirty_small_pool():
    import torch
    # 64 blocks of 1 MiB (the largest size PyTorch serves from its small
    # pool): 32 segments of 2 MiB full of NaN, then returned to the cache
    blocks = [torch.full((1 << 17,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(64)]
    torch.cuda.synchronize()
    del blocks


@pytest.mark.parametrize("prec", [0, 1])
def test_products_over_stale_padding(prec):
    from paper_2411_05869_amd import Context, LOGDET_EXACT
    rng = np.random.default_rng(3)
    n = 301
    x = rng.random((n, 2))
    th = Theta(1.0, np.array([0.3, 0.3]), np.array([[[0.5, 0.5]]]), np.array([[[0.9, 0.9]]]), np.ones((1, 1)),
               np.ones((1, 1)), 0.1)
    p = Problem("all rows in one group", x, th, cell=None)
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    assert np.all(np.diff(A.indptr) == n)
    _dirty_small_pool()
    ctx = Context()
    ds = ctx.dataset(dev(p.x))
    K = ctx.assemble(ds, p.theta, prec)
    tol = 1e-13 if prec == 0 else 2.0 ** -24 + 1e-13
    for k in (1, 2, 32):
        X = rng.standard_normal((n, k)) if k > 1 else rng.standard_normal(n)
        Y = host(ctx.matvec(K, dev(X)))
        bound = abs(A) @ np.abs(X)
        worst = float(np.max(np.abs(Y - A @ X) / bound)) if np.all(np.isfinite(Y)) else np.inf
        print(f"[stale padding prec={prec} k={k}] worst |dy| / (|K||x|) {worst:.2e}")
        assert np.all(np.isfinite(Y)), (prec, k)
        assert np.all(np.abs(Y - A @ X) <= tol * bound), (prec, k)
    if prec == 0:
        y = rng.standard_normal(n)
        ref = likelihood.dense_cholesky(A.toarray(), y)
        r = ctx.loglik(K, dev(y), logdet_mode=LOGDET_EXACT)
        print(f"[stale padding] loglik {r['loglik']:.12g} ref {ref['loglik']:.12g}")
        assert abs(r["loglik"] - ref["loglik"]) <= 1e-10 * abs(ref["loglik"])
