"""gp_matvec_noalloc (the allocation-free one-column product) gives bitwise
the result of gp_matvec with one right-hand side, called through the C ABI:
two calls in a row on one GPU, the second on a smaller matrix, so the shared
scratch array holds the first call's data when the second runs.  The first
call runs before any cached int16 column offsets exist (int32 columns), the
second after gp_matvec built them, and the FP64 and mixed forms are both
checked.  A matrix above the scratch limit is refused."""
import ctypes as C

import numpy as np
import pytest

from workloads import config1, uniform_problem
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _noalloc(ctx, K, x, y):
    st = ctx._L.gp_matvec_noalloc(ctx._h, K._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert st == 0, ctx._L.gp_last_error(ctx._h)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_matvec(prec):
    import torch
    from paper_2411_05869_amd import Context
    ctx = Context()
    big = config1()
    small = uniform_problem(777, 2, 5, r0=0.07, n1=2, n2=2, bump_radius=0.2)
    rng = np.random.default_rng(31 + prec)
    cases = []
    for p in (big, small):
        ds = ctx.dataset(dev(p.x), cell=p.cell)
        K = ctx.assemble(ds, p.theta, prec)
        cases.append((ds, K, dev(rng.standard_normal(p.n))))
    # first call on the larger matrix before any product built a cache
    ds1, K1, x1 = cases[0]
    y1 = torch.full((K1.n,), float("nan"), dtype=torch.float64, device="cuda")
    _noalloc(ctx, K1, x1, y1)
    torch.cuda.synchronize()
    ref1 = ctx.matvec(K1, x1)   # builds the int16 offsets of K1
    assert np.array_equal(host(y1), host(ref1)), "first call differs from gp_matvec"
    # second call on the smaller matrix (scratch still holds the first call's vectors)
    ds2, K2, x2 = cases[1]
    ref2 = ctx.matvec(K2, x2)
    y2 = torch.full((K2.n,), float("nan"), dtype=torch.float64, device="cuda")
    _noalloc(ctx, K2, x2, y2)
    torch.cuda.synchronize()
    assert np.array_equal(host(y2), host(ref2)), "second (smaller) call differs from gp_matvec"
    # and once more on the first matrix, now with its cached offsets
    y3 = torch.empty_like(y1)
    _noalloc(ctx, K1, x1, y3)
    torch.cuda.synchronize()
    assert np.array_equal(host(y3), host(ref1)), "call after the cache was built differs"
    ctx.close()


def test_noalloc_refuses_n_above_the_scratch():
    import torch
    from paper_2411_05869_amd import Context
    ctx = Context()
    n = 4_194_305   # one point more than 64 MiB holds for two float64 n-vectors
    p = uniform_problem(n, 1, 7, r0=1e-9, n1=1, n2=1, bump_radius=1e-9)
    ds = ctx.dataset(dev(p.x), cell=[1e-5])
    K = ctx.assemble(ds, p.theta, 1)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    st = ctx._L.gp_matvec_noalloc(ctx._h, K._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert st == 1, st   # GP_EINVAL
    assert b"exceeds" in ctx._L.gp_last_error(ctx._h)
    ctx.close()
