"""The log det on the context's second stream (gp_ctx_set_concurrency): with
it on (the default) the SLQ launches run beside the solver's; with it off they
follow the solve on one stream.  The kernels and their order within each task
are the same, so every result is bitwise the same: gp_loglik, gp_loglik_async
and gp_loglik_batch, both precisions."""
import math

import numpy as np
import pytest

from workloads import config1, gmm_problem
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

KEYS = ("loglik", "logdet", "quad", "logdet_se", "relres", "cg_iters", "refreshes", "lanczos_steps", "status")


def _same(a, b, what):
    for k in KEYS:
        assert a[k] == b[k], (what, k, a[k], b[k])


@pytest.mark.parametrize("prec", [0, 1])
def test_concurrency_on_off_equal(prec):
    import torch
    from paper_2411_05869_amd import LOGDET_SLQ_REORTH, SOLVER_CG, Context
    ctx = Context()
    p1 = config1()
    y1 = np.random.default_rng(5).standard_normal(p1.n)
    s = math.sqrt(1e5 / 20000)
    p2 = gmm_problem(20000, 911, 0.0078 * s, 0.02 * s)
    Ks, ys = [], []
    for p, y in ((p1, y1), (p2, p2.y)):
        Ks.append(ctx.assemble(ctx.dataset(dev(p.x), cell=p.cell), p.theta, prec))
        ys.append(dev(y))
    res = {}
    for on in (True, False):
        ctx.set_concurrency(on)
        out = []
        for K, y in zip(Ks, ys):
            a = torch.empty(K.n, dtype=torch.float64, device="cuda")
            r = ctx.loglik(K, y, alpha_out=a, n_lanczos=40)
            rr = ctx.loglik(K, y, logdet_mode=LOGDET_SLQ_REORTH, n_lanczos=20)
            ra = ctx.loglik_async(K, y, solver=SOLVER_CG, max_iter=2 * r["cg_iters"] + 16, n_lanczos=40)[0].result()
            out.append((r, host(a), rr, ra))
        out.append(ctx.loglik_batch(Ks, ys, solver=SOLVER_CG, n_lanczos=40))
        res[on] = out
    for i in range(2):
        (r1, a1, rr1, ra1), (r0, a0, rr0, ra0) = res[True][i], res[False][i]
        _same(r1, r0, f"gp_loglik problem {i}")
        assert np.array_equal(a1, a0)
        _same(rr1, rr0, f"gp_loglik re-orthogonalised problem {i}")
        _same(ra1, ra0, f"gp_loglik_async problem {i}")
    for i, (b1, b0) in enumerate(zip(res[True][2], res[False][2])):
        _same(b1, b0, f"gp_loglik_batch problem {i}")
    print(f"[concurrency prec={prec}] on and off equal: loglik {res[True][0][0]['loglik']:.12g}, "
          f"{res[True][1][0]['loglik']:.12g}")


def test_profile_only_times_the_named_groups():
    """gp_profile_only: with a list of names only those launch groups are timed
    (two events each on their stream); what is timed does not change a result."""
    from paper_2411_05869_amd import Context, GPError
    ctx = Context()
    p = config1()
    y = dev(np.random.default_rng(5).standard_normal(p.n))
    K = ctx.assemble(ctx.dataset(dev(p.x), cell=p.cell), p.theta, 1)
    ctx.profile(True, only=["spmm", "spmv_f32val_f64"])
    r1 = ctx.loglik(K, y, n_lanczos=20)
    some = ctx.profile_read()
    ctx.profile(True)
    r2 = ctx.loglik(K, y, n_lanczos=20)
    every = ctx.profile_read()
    ctx.profile(False)
    assert set(some) == {"spmm", "spmv_f32val_f64"}
    assert some["spmm"][0] == 20 and some["spmv_f32val_f64"][0] >= r1["cg_iters"]
    assert {"spmm", "spmv_f32val_f64", "pcg_vector_ops", "lanczos_vector_ops"} <= set(every)
    _same(r1, r2, "timed subsets")
    with pytest.raises(GPError):
        ctx.profile(True, only=["x" * 32])


@pytest.mark.parametrize("prec", [0, 1])
def test_side_work_after_an_error_and_across_probe_blocks(prec):
    """The log det is handed to the side stream a Lanczos step at a time.  A
    likelihood that fails inside the solve (y holds a NaN: GP_EINVAL after the
    log det has started) drops the steps not yet enqueued; the next call on the
    same context is unaffected.  With 40 probes (two blocks of at most 32: the
    first block's quadrature and the second block's start fall between units)
    the estimate is bitwise the same beside the solve, after it, and on a fresh
    context."""
    import torch
    from paper_2411_05869_amd import Context, GPError
    p = config1()
    y = np.random.default_rng(8).standard_normal(p.n)
    bad = y.copy()
    bad[17] = np.nan
    ctx = Context()
    K = ctx.assemble(ctx.dataset(dev(p.x), cell=p.cell), p.theta, prec)
    opts = dict(n_probes=40, n_lanczos=30)
    with pytest.raises(GPError) as e:
        ctx.loglik(K, dev(bad), **opts)
    assert e.value.name == "GP_EINVAL"
    r_on = ctx.loglik(K, dev(y), **opts)
    ctx.set_concurrency(False)
    r_off = ctx.loglik(K, dev(y), **opts)
    fresh = Context()
    Kf = fresh.assemble(fresh.dataset(dev(p.x), cell=p.cell), p.theta, prec)
    r_fresh = fresh.loglik(Kf, dev(y), **opts)
    assert r_on["status"] == 0 and r_on["lanczos_steps"] > 0
    _same(r_on, r_off, "beside vs after the solve")
    _same(r_on, r_fresh, "after an error vs a fresh context")
    print(f"[side work prec={prec}] loglik {r_on['loglik']:.12g} logdet {r_on['logdet']:.12g} "
          f"+- {r_on['logdet_se']:.3g} (40 probes)")


@pytest.mark.parametrize("prec", [0, 1])
def test_side_work_through_the_minres_fallback(prec):
    """CG capped below convergence hands over to MINRES (GP_SOLVER_AUTO) while
    the log det's Lanczos steps are handed to the side stream from both
    solvers' loops: every result is bitwise the same with the log det beside
    the solve and after it."""
    from paper_2411_05869_amd import LOGDET_NONE, SOLVER_AUTO, SOLVER_CG, Context
    ctx = Context()
    p = config1()
    y = dev(np.random.default_rng(9).standard_normal(p.n))
    K = ctx.assemble(ctx.dataset(dev(p.x), cell=p.cell), p.theta, prec)
    full = ctx.loglik(K, y, logdet_mode=LOGDET_NONE, solver=SOLVER_CG)
    cap = max(8, int(0.75 * full["cg_iters"]))
    res = {}
    for on in (True, False):
        ctx.set_concurrency(on)
        res[on] = ctx.loglik(K, y, solver=SOLVER_AUTO, max_iter=cap, n_lanczos=40)
    r = res[True]
    print(f"[side work, MINRES fallback prec={prec}] cg {r['cg_iters']} + minres {r['minres_iters']}, "
          f"loglik {r['loglik']:.12g}")
    assert r["status"] == 0 and r["cg_iters"] == cap and r["minres_iters"] > 0
    _same(res[True], res[False], "MINRES fallback beside vs after the solve")
    assert res[True]["minres_iters"] == res[False]["minres_iters"]
