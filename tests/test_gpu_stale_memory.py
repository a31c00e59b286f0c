"""Results must not depend on what device memory held before.  Several kernels
read past the data they use (four-wide loads past a row's end, whole 32-column
blocks when fewer columns are live) and give those values a zero weight; that is
only sound where the memory read holds finite numbers (0 x NaN = NaN).

The same calls run twice, each on a fresh context: first on memory PyTorch
has just obtained, then after both of its block pools have been filled with
NaN and released, so the library's arrays and work spaces are carved from
NaN-filled memory.  The library is deterministic (fixed reduction grids, cells
sorted after binning, counter-based probes), so every result must agree
bitwise: log-likelihoods (SLQ and exact log det) in both precisions, 1-, 7- and
32-column products, the solve (conjugate gradients and MINRES), the kriging mean
(float64 and float32 evaluation), and posterior variances for
a ragged number of test points (37: one full and one partial block of 32);
and, for a Matern core, the nonstationary core and per-point error variances,
the products, an SLQ log-likelihood and the kriging mean."""
import numpy as np
import pytest

from workloads import config1
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _fill_pools_with_nan():
    import torch
    # 64 blocks of 1 MiB from the small pool, 12 blocks of 32 MiB from the large one
    small = [torch.full((1 << 17,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(64)]
    large = [torch.full((1 << 22,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(12)]
    torch.cuda.synchronize()
    del small, large


def _run(p, y, X, xs):
    import torch
    from paper_2411_05869_amd import Context, LOGDET_EXACT, MIXED, SOLVER_MINRES
    ctx = Context()
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    out = {}
    for prec in (0, 1):
        K = ctx.assemble(ds, p.theta, prec)
        r = ctx.loglik(K, dev(y))
        out[f"slq{prec}"] = (r["loglik"], r["quad"], r["logdet"], r["logdet_se"], r["cg_iters"])
        if prec == 0:
            r = ctx.loglik(K, dev(y), logdet_mode=LOGDET_EXACT)
            out["exact"] = (r["loglik"], r["quad"], r["logdet"])
        for k in (1, 7, 32):
            out[f"mv{prec}_{k}"] = host(ctx.matvec(K, dev(X[:, 0] if k == 1 else X[:, :k])))
        alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
        r = ctx.solve(K, dev(y), alpha, solver=SOLVER_MINRES)
        out[f"minres{prec}"] = np.append(host(alpha), r["minres_iters"])
        ctx.solve(K, dev(y), alpha)
        out[f"alpha{prec}"] = host(alpha)
        pred = ctx.predictor(ds, p.theta, alpha)
        out[f"mean{prec}"] = host(ctx.predict(pred, dev(xs)))
        out[f"mean32_{prec}"] = host(ctx.predict(pred, dev(xs), precision=MIXED))
        pred.close()
        var, res = ctx.predict_var(K, p.theta, dev(xs))
        out[f"var{prec}"] = np.append(host(var), res["iters"])
        K.close()
    return out


def _run_light(problems):
    import torch
    from paper_2411_05869_amd import Context, MIXED
    ctx = Context()
    out = {}
    for name, p in problems:
        rng = np.random.default_rng(5)
        y = rng.standard_normal(p.n)
        X = rng.standard_normal((p.n, 32))
        xs = rng.random((37, p.x.shape[1]))
        ds = ctx.dataset(dev(p.x), cell=p.cell)
        for prec in (0, 1):
            K = ctx.assemble(ds, p.theta, prec)
            out[f"{name} mv{prec}_1"] = host(ctx.matvec(K, dev(X[:, 0])))
            out[f"{name} mv{prec}_32"] = host(ctx.matvec(K, dev(X)))
            alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
            r = ctx.loglik(K, dev(y), alpha_out=alpha)
            out[f"{name} slq{prec}"] = (r["loglik"], r["quad"], r["logdet"], r["cg_iters"])
            pred = ctx.predictor(ds, p.theta, alpha)
            out[f"{name} mean{prec}"] = host(ctx.predict(pred, dev(xs)))
            out[f"{name} mean32_{prec}"] = host(ctx.predict(pred, dev(xs), precision=MIXED))
            pred.close()
            K.close()
    return out


def _compare(clean, dirty):
    for key in clean:
        a, b = np.asarray(clean[key], dtype=float), np.asarray(dirty[key], dtype=float)
        print(f"[stale memory] {key}: finite {bool(np.all(np.isfinite(b)))}, "
              f"max |diff| {float(np.max(np.abs(a - b))) if np.all(np.isfinite(b)) else np.inf:.3g}")
        assert np.all(np.isfinite(a)), key
        assert np.array_equal(a, b), key


def test_core_kernels_and_noise_do_not_depend_on_stale_memory():
    # the fills and predictions with a core kernel (Matern, nonstationary) and
    # with per-point error variances have code paths of their own
    from paper_2411_05869_amd import CORE_MATERN, CORE_PACIOREK
    from workloads import core_problem, noise_variances
    pn = config1()
    pn.theta.tau2 = noise_variances(pn.n, 3, 0.0, 0.05)
    problems = [("matern", core_problem(CORE_MATERN, 2)), ("nonstationary", core_problem(CORE_PACIOREK, 2)),
                ("tau2", pn)]
    clean = _run_light(problems)
    _fill_pools_with_nan()
    dirty = _run_light(problems)
    _compare(clean, dirty)


def test_results_do_not_depend_on_stale_memory():
    p = config1()
    rng = np.random.default_rng(21)
    y = rng.standard_normal(p.n)
    X = rng.standard_normal((p.n, 32))
    xs = rng.random((37, p.x.shape[1]))
    clean = _run(p, y, X, xs)
    _fill_pools_with_nan()
    dirty = _run(p, y, X, xs)
    _compare(clean, dirty)
