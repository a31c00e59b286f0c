"""gp_loglik_batch: the likelihoods of several small problems in shared launches
(the sampler of Appendix C evaluates many proposals of a few thousand to tens
of thousands of points, Sec. 3.3).  The matrices are stacked block-diagonally
and every problem keeps its own scalars, stopping test and probes, so each
result equals gp_loglik's for that problem alone, bitwise: checked on a mix of
dimensions, sizes, core kernels and bump groups (and several proposals of one
data set), both precisions, SLQ and no log det, block and point Jacobi, with
alpha.  A failing problem does not disturb the others; GP_SOLVER_AUTO hands a
problem that did not converge to gp_loglik; bad arguments are refused."""
import math

import numpy as np
import pytest

from workloads import config1, core_problem, gmm_problem, perturb_theta, uniform_problem
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

KEYS = ("loglik", "logdet", "quad", "logdet_se", "relres", "cg_iters", "refreshes", "lanczos_steps", "status",
        "minres_iters")


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


def _problems():
    out = []
    p = config1()
    out.append((p, np.random.default_rng(5).standard_normal(p.n)))
    s = math.sqrt(1e5 / 12000)
    g = gmm_problem(12000, 913, 0.0078 * s, 0.02 * s)
    out.append((g, g.y))
    # three proposals on one data set (same points, perturbed theta)
    rng = np.random.default_rng(17)
    for _ in range(2):
        q = gmm_problem(12000, 913, 0.0078 * s, 0.02 * s)
        q.theta = perturb_theta(rng, g.theta)
        out.append((q, g.y))
    c1 = core_problem(1, 1, n=1500, seed=21)
    out.append((c1, np.random.default_rng(6).standard_normal(c1.n)))
    u3 = uniform_problem(3000, 3, 23, r0=0.12, n1=2, n2=2, bump_radius=0.3, name="uniform-3d-n3000")
    out.append((u3, np.random.default_rng(7).standard_normal(u3.n)))
    return out


def _same(a, b, what):
    for k in KEYS:
        assert a[k] == b[k], (what, k, a[k], b[k])


def _setup(ctx, prec):
    probs = _problems()
    Ks, ys = [], []
    for p, y in probs:
        ds = ctx.dataset(dev(p.x), cell=p.cell)
        Ks.append(ctx.assemble(ds, p.theta, prec))
        ys.append(dev(y))
    return probs, Ks, ys


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_alone(ctx, prec):
    import torch
    from paper_2411_05869_amd import LOGDET_NONE, LOGDET_SLQ, PRECOND_BLOCK_JACOBI, PRECOND_JACOBI, SOLVER_CG
    probs, Ks, ys = _setup(ctx, prec)
    for mode, pre in ((LOGDET_SLQ, PRECOND_BLOCK_JACOBI), (LOGDET_NONE, PRECOND_JACOBI)):
        opts = dict(solver=SOLVER_CG, logdet_mode=mode, precond=pre, n_lanczos=40, seed=91)
        alone, a_alone = [], []
        for K, y in zip(Ks, ys):
            a = torch.empty(K.n, dtype=torch.float64, device="cuda")
            alone.append(ctx.loglik(K, y, alpha_out=a, **opts))
            a_alone.append(a)
        a_batch = [torch.full((K.n,), float("nan"), dtype=torch.float64, device="cuda") for K in Ks]
        res = ctx.loglik_batch(Ks, ys, alpha_outs=a_batch, **opts)
        for (p, _), r, ra, a, b in zip(probs, res, alone, a_batch, a_alone):
            what = f"{p.name} prec={prec} mode={mode} precond={pre}"
            _same(r, ra, what)
            assert np.array_equal(host(a), host(b)), what
            print(f"[batch {what}] loglik {r['loglik']:.12g} iters {r['cg_iters']} equal to gp_loglik alone")


def test_batch_order_and_subsets(ctx):
    """A problem's result does not depend on its neighbours in the stack."""
    from paper_2411_05869_amd import SOLVER_CG
    probs, Ks, ys = _setup(ctx, 1)
    opts = dict(solver=SOLVER_CG, n_lanczos=30, seed=5)
    full = ctx.loglik_batch(Ks, ys, **opts)
    order = [4, 1, 5, 0, 3, 2]
    rev = ctx.loglik_batch([Ks[i] for i in order], [ys[i] for i in order], **opts)
    for j, i in enumerate(order):
        _same(rev[j], full[i], f"reordered {probs[i][0].name}")
    one = ctx.loglik_batch([Ks[3]], [ys[3]], **opts)
    _same(one[0], full[3], "batch of one")


def test_batch_status_cases(ctx):
    import torch
    from paper_2411_05869_amd import (GPError, LOGDET_EXACT, LOGDET_SLQ_REORTH, SOLVER_AUTO, SOLVER_CG,
                                      SOLVER_MINRES)
    probs, Ks, ys = _setup(ctx, 0)
    Ks, ys = Ks[:3], ys[:3]
    # a non-finite y fails its own problem only
    bad = ys[1].clone()
    bad[11] = float("nan")
    ref = ctx.loglik_batch(Ks, ys, solver=SOLVER_CG)
    res = ctx.loglik_batch(Ks, [ys[0], bad, ys[2]], solver=SOLVER_CG, raise_on_error=False)
    assert res[1]["status"] == 1
    _same(res[0], ref[0], "neighbour of a failed problem")
    _same(res[2], ref[2], "neighbour of a failed problem")
    # y = 0: alpha = 0, quadratic form 0, no iterations
    z = torch.zeros_like(ys[2])
    a = torch.full_like(ys[2], 3.0)
    res = ctx.loglik_batch([Ks[0], Ks[2]], [ys[0], z], alpha_outs=[None, a], solver=SOLVER_CG)
    assert res[1]["quad"] == 0.0 and res[1]["cg_iters"] == 0 and float(a.abs().max()) == 0.0
    _same(res[0], ref[0], "neighbour of y = 0")
    # an iteration cap too small: GP_ENOTCONV with CG; AUTO hands it to gp_loglik (MINRES)
    res = ctx.loglik_batch(Ks, ys, solver=SOLVER_CG, max_iter=8, raise_on_error=False)
    assert all(r["status"] == 3 and r["cg_iters"] == 8 for r in res)
    res = ctx.loglik_batch(Ks, ys, solver=SOLVER_AUTO, max_iter=8, raise_on_error=False)
    for K, y, r in zip(Ks, ys, res):
        _same(r, ctx.loglik(K, y, solver=SOLVER_AUTO, max_iter=8, raise_on_error=False), "AUTO fallback")
        assert r["minres_iters"] > 0
    # refused before any device work
    for kw in (dict(solver=SOLVER_MINRES), dict(logdet_mode=LOGDET_EXACT), dict(logdet_mode=LOGDET_SLQ_REORTH)):
        with pytest.raises(GPError) as e:
            ctx.loglik_batch(Ks, ys, **kw)
        assert e.value.name == "GP_EINVAL"
    p0 = probs[0][0]
    K32 = ctx.assemble(ctx.dataset(dev(p0.x), cell=p0.cell), p0.theta, 1)
    with pytest.raises(GPError) as e:
        ctx.loglik_batch([Ks[0], K32], [ys[0], ys[0]])
    assert e.value.name == "GP_EINVAL"
