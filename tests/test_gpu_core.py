"""GPU parity of the core kernel C_y = C_core x C_sparse (Eq. sparseCov;
stationary Matern and the nonstationary kernel of Eq. PScov) against the FP64
oracle.

* Assembly: pattern bit-exact (the core never changes it), FP64 values
  within 1e-12 relative (floor 1e-14 max|K|; exp, sqrt and the prefactor's
  powers are formed differently on the two sides), float32 values within one
  float32 rounding (1.2e-7), bitwise symmetry.
* Log-likelihood in exact mode against dense Cholesky: 1e-8 (FP64) / 1e-5
  (mixed) for quad, alpha and log det.
* Kriging mean against the oracle's brute-force sum: 1e-10 (FP64) / 2e-7
  (mixed) of sum_q |C(x*, x_q)| |alpha_q|.
"""
import numpy as np
import pytest

from oracle import kernel, likelihood, predict
from workloads import Core, core_problem
from gpu_util import assert_pattern_equal, dev, export, host, rel, to_scipy, value_errors

pytestmark = pytest.mark.gpu

MATERN, PACIOREK = 1, 2


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


CASES = [(MATERN, 1, 1), (MATERN, 2, 3), (MATERN, 3, 5), (MATERN, 2, 0),
         (PACIOREK, 1, 5), (PACIOREK, 2, 5), (PACIOREK, 3, 3), (PACIOREK, 2, 0), (PACIOREK, 2, 1)]


@pytest.mark.parametrize("kind,d,nu2", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_with_core(ctx, kind, d, nu2, prec):
    p = core_problem(kind, d, n=1200, seed=30 + d, nu2=nu2)
    what = f"core kind={kind} d={d} nu2={nu2} prec={prec}"
    print(f"[case] {what}", flush=True)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, prec)
    rp, col, val = export(ctx, K)
    ip, ci, vo = kernel.sparse(p.x, p.theta)
    assert_pattern_equal(rp, col, ip, ci, what)
    err = value_errors(val, vo)
    print(f"[{what}] nnz {K.nnz} value error {err:.2e}")
    assert err <= (1e-12 if prec == 0 else 1.2e-7)
    A = to_scipy(rp, col, val, p.n)
    assert (A != A.T).nnz == 0, "not bitwise symmetric"


@pytest.mark.parametrize("kind,nu2", [(MATERN, 3), (PACIOREK, 5)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-5)])
def test_loglik_with_core(ctx, kind, nu2, prec, tol):
    import torch
    from paper_2411_05869_amd import LOGDET_EXACT
    p = core_problem(kind, 2, n=1500, seed=5, nu2=nu2)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    ref = likelihood.dense_cholesky(K, y)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    Kg = ctx.assemble(ds, p.theta, prec)
    alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
    r = ctx.loglik(Kg, dev(y), alpha_out=alpha, logdet_mode=LOGDET_EXACT)
    errs = dict(loglik=rel(r["loglik"], ref["loglik"]), logdet=rel(r["logdet"], ref["logdet"]),
                quad=rel(r["quad"], ref["quad"]),
                alpha=float(np.abs(host(alpha) - ref["alpha"]).max() / np.abs(ref["alpha"]).max()))
    print(f"[core loglik kind={kind} prec={prec}] iters {r['cg_iters']} errors {errs}")
    assert r["status"] == 0
    for k, v in errs.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("kind,d,nu2", [(MATERN, 1, 5), (MATERN, 2, 0), (PACIOREK, 2, 5), (PACIOREK, 3, 3)])
def test_predict_with_core(ctx, kind, d, nu2):
    p = core_problem(kind, d, n=700, seed=60 + d, nu2=nu2)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    alpha = likelihood.dense_cholesky(K, y)["alpha"]
    rng = np.random.default_rng(d)
    xs = rng.uniform(-0.2, 1.2, (250, d))
    ref = predict.mean(xs, p.x, p.theta, alpha)
    rp, cols, vals = kernel.cross_entries(xs, p.x, p.theta)
    sc = np.array([np.abs(vals[rp[i]:rp[i + 1]]) @ np.abs(alpha[cols[rp[i]:rp[i + 1]]])
                   for i in range(xs.shape[0])]) + 1e-300
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    pred = ctx.predictor(ds, p.theta, dev(alpha))
    for prec, tol in ((0, 1e-10), (1, 2e-7)):
        m = host(ctx.predict(pred, dev(xs), precision=prec))
        err = float(np.max(np.abs(m - ref) / sc))
        print(f"[core predict kind={kind} d={d} nu2={nu2} prec={prec}] max scaled error {err:.2e}")
        assert err <= tol


def test_core_none_matches_no_core(ctx):
    p = core_problem(MATERN, 2, n=600, seed=8)
    p.theta.core = Core(0)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    a = export(ctx, ctx.assemble(ds, p.theta, 0))
    p.theta.core = None
    b = export(ctx, ctx.assemble(ds, p.theta, 0))
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("field,value", [("nu2", 2), ("sigma0", 0.0), ("ell", np.array([1.0, -1.0, 1.0])),
                                         ("Sigma0", -1.0), ("width", np.array([0.0, 1.0, 1.0])),
                                         ("kind", 7)])
def test_invalid_core_is_einval(ctx, field, value):
    from paper_2411_05869_amd import GPError
    p = core_problem(PACIOREK, 2, n=200, seed=9)
    setattr(p.theta.core, field, value)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    with pytest.raises(GPError) as e:
        ctx.assemble(ds, p.theta, 0)
    assert e.value.status == 1
