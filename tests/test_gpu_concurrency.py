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
