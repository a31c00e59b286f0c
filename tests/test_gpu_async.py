"""gp_loglik_async: the likelihood with every solver decision taken on the
device, written by the device into pinned memory and signalled by an event.
It enqueues the same kernels in the same order as gp_loglik with the
conjugate-gradient solver (the iterations after convergence return at
once), so every result equals gp_loglik's bitwise; checked on
config 1 (n = 2000) and a 20,000-point mixture set, both precisions, SLQ,
re-orthogonalised SLQ and no log det, with alpha.  Two evaluations on two
streams are in flight together.  An iteration cap that is too small gives
GP_ENOTCONV in the result, y = 0 gives alpha = 0, a non-finite y gives
GP_EINVAL in the result; bad arguments are refused before any device work."""
import math

import numpy as np
import pytest

from workloads import config1, gmm_problem
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

KEYS = ("loglik", "logdet", "quad", "logdet_se", "cg_iters", "refreshes", "lanczos_steps", "status")


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


def _problems():
    p1 = config1()
    y1 = np.random.default_rng(5).standard_normal(p1.n)
    s = math.sqrt(1e5 / 20000)
    p2 = gmm_problem(20000, 911, 0.0078 * s, 0.02 * s)
    return [(p1, y1), (p2, p2.y)]


def _same(a, b, what):
    for k in KEYS + ("relres",):
        assert a[k] == b[k], (what, k, a[k], b[k])


@pytest.mark.parametrize("prec", [0, 1])
def test_async_equals_sync(ctx, prec):
    import torch
    from paper_2411_05869_amd import LOGDET_NONE, LOGDET_SLQ, LOGDET_SLQ_REORTH, SOLVER_CG
    for p, y in _problems():
        ds = ctx.dataset(dev(p.x), cell=p.cell)
        K = ctx.assemble(ds, p.theta, prec)
        yd = dev(y)
        for mode in (LOGDET_SLQ, LOGDET_SLQ_REORTH, LOGDET_NONE):
            opts = dict(solver=SOLVER_CG, logdet_mode=mode, n_lanczos=30, seed=77)
            a_sync = torch.empty(p.n, dtype=torch.float64, device="cuda")
            r_sync = ctx.loglik(K, yd, alpha_out=a_sync, **opts)
            a_async = torch.full((p.n,), float("nan"), dtype=torch.float64, device="cuda")
            pend, ev = ctx.loglik_async(K, yd, alpha_out=a_async, max_iter=2 * r_sync["cg_iters"] + 16, **opts)
            r_async = pend.result()
            what = f"{p.name} prec={prec} mode={mode}"
            _same(r_async, r_sync, what)
            assert np.array_equal(host(a_async), host(a_sync)), what
            print(f"[async {what}] loglik {r_async['loglik']:.12g} iters {r_async['cg_iters']} equal to gp_loglik")


def test_two_streams_in_flight():
    import torch
    from paper_2411_05869_amd import Context, SOLVER_CG
    (p1, y1), (p2, y2) = _problems()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c1, c2 = Context(stream=s1), Context(stream=s2)
    K1 = c1.assemble(c1.dataset(dev(p1.x), cell=p1.cell), p1.theta, 1)
    K2 = c2.assemble(c2.dataset(dev(p2.x), cell=p2.cell), p2.theta, 1)
    torch.cuda.synchronize()
    ref1 = c1.loglik(K1, dev(y1), solver=SOLVER_CG)
    ref2 = c2.loglik(K2, dev(y2), solver=SOLVER_CG)
    torch.cuda.synchronize()
    y1d, y2d = dev(y1), dev(y2)
    torch.cuda.synchronize()
    pa, _ = c1.loglik_async(K1, y1d, solver=SOLVER_CG, max_iter=2 * ref1["cg_iters"] + 16)
    pb, _ = c2.loglik_async(K2, y2d, solver=SOLVER_CG, max_iter=2 * ref2["cg_iters"] + 16)
    _same(pb.result(), ref2, "stream 2")
    _same(pa.result(), ref1, "stream 1")


def test_async_status_cases(ctx):
    import ctypes as C

    import torch
    from paper_2411_05869_amd import GPError, LOGDET_EXACT, SOLVER_CG, SOLVER_MINRES
    from paper_2411_05869_amd._lib import CLoglikResult
    p, y = _problems()[0]
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, 0)
    # an iteration cap that is too small
    r = ctx.loglik_async(K, dev(y), solver=SOLVER_CG, max_iter=8)[0].result()
    assert r["status"] == 3 and r["cg_iters"] == 8 and r["relres"] > 1e-10
    # y = 0: alpha = 0 exactly, quadratic form 0
    a = torch.full((p.n,), 7.0, dtype=torch.float64, device="cuda")
    r = ctx.loglik_async(K, torch.zeros(p.n, dtype=torch.float64, device="cuda"), alpha_out=a, solver=SOLVER_CG,
                         max_iter=64)[0].result()
    assert r["status"] == 0 and r["quad"] == 0.0 and r["cg_iters"] == 0 and float(a.abs().max()) == 0.0
    # a non-finite y is reported in the result
    yb = y.copy()
    yb[17] = np.nan
    r = ctx.loglik_async(K, dev(yb), solver=SOLVER_CG, max_iter=64)[0].result()
    assert r["status"] == 1
    # refused before any device work
    for kw in (dict(solver=SOLVER_MINRES), dict(logdet_mode=LOGDET_EXACT)):
        with pytest.raises(GPError) as e:
            ctx.loglik_async(K, dev(y), max_iter=64, **kw)
        assert e.value.name == "GP_EINVAL"
    pageable = CLoglikResult()
    o = ctx.opts(solver=SOLVER_CG, max_iter=64)
    st = ctx._L.gp_loglik_async(ctx._h, K._h, C.c_void_p(dev(y).data_ptr()), C.byref(o), None,
                                C.c_void_p(C.addressof(pageable)), None)
    assert st == 1   # out must be memory the device can write
