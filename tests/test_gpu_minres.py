"""GPU parity of the MINRES solver (Sec. 3.3; Paige and Saunders) and of the
automatic fallback from conjugate gradients.

* MINRES alone on config 1: alpha and y^T K^-1 y against dense Cholesky,
  1e-8 (float64) / 1e-5 (mixed: products on the float32 values).
* The same system against the oracle's MINRES with the same (Jacobi)
  preconditioner: the same solution, and step counts within the host-check
  granularity (8 steps) plus a few steps of rounding.
* Fallback: with an iteration cap below what conjugate gradients need, CG alone
  reports GP_ENOTCONV while GP_SOLVER_AUTO continues with MINRES from the last
  CG iterate and converges to the oracle's answer.
"""
import numpy as np
import pytest

from oracle import kernel, likelihood
from oracle.minres import minres
from workloads import config1
from gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


@pytest.fixture(scope="module")
def cfg1():
    p = config1()
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    return p, K, y, likelihood.dense_cholesky(K, y)


def _solve(ctx, p, y, prec, **opts):
    import torch
    from paper_2411_05869_amd import LOGDET_NONE
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, prec)
    alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
    r = ctx.loglik(K, dev(y), alpha_out=alpha, logdet_mode=LOGDET_NONE, raise_on_error=False, **opts)
    return r, host(alpha)


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-5)])
def test_minres_matches_cholesky(ctx, cfg1, prec, tol, precond):
    from paper_2411_05869_amd import SOLVER_MINRES
    p, K, y, ref = cfg1
    r, a = _solve(ctx, p, y, prec, solver=SOLVER_MINRES, precond=precond)
    e_q = rel(r["quad"], ref["quad"])
    e_a = float(np.abs(a - ref["alpha"]).max() / np.abs(ref["alpha"]).max())
    print(f"[minres prec={prec} precond={precond}] iters {r['minres_iters']} relres {r['relres']:.2e} "
          f"quad {e_q:.2e} alpha {e_a:.2e}")
    assert r["status"] == 0 and r["cg_iters"] == 0 and r["minres_iters"] > 0
    assert r["relres"] <= 1e-10
    assert e_q <= tol and e_a <= (tol if prec == 0 else 1e-3)


def test_minres_matches_oracle_minres(ctx, cfg1):
    from paper_2411_05869_amd import PRECOND_JACOBI, SOLVER_MINRES
    p, K, y, ref = cfg1
    r, a = _solve(ctx, p, y, 0, solver=SOLVER_MINRES, precond=PRECOND_JACOBI)
    d = np.diag(K).copy()
    o = minres(K, y, lambda v: v / d, rtol=1e-10)
    e = float(np.abs(a - o["x"]).max() / np.abs(o["x"]).max())
    print(f"[minres vs oracle] gpu iters {r['minres_iters']} oracle iters {o['iters']} solution diff {e:.2e}")
    assert o["converged"]
    assert e <= 1e-8
    assert abs(r["minres_iters"] - o["iters"]) <= 8 + 4


def test_auto_falls_back_to_minres(ctx, cfg1):
    from paper_2411_05869_amd import SOLVER_AUTO, SOLVER_CG
    p, K, y, ref = cfg1
    full, _ = _solve(ctx, p, y, 0, solver=SOLVER_CG)
    cap = max(8, int(0.75 * full["cg_iters"]))
    cg_only, _ = _solve(ctx, p, y, 0, solver=SOLVER_CG, max_iter=cap)
    auto, a = _solve(ctx, p, y, 0, solver=SOLVER_AUTO, max_iter=cap)
    e_q = rel(auto["quad"], ref["quad"])
    print(f"[auto] CG needs {full['cg_iters']}; cap {cap}: CG alone status {cg_only['status']}; "
          f"auto status {auto['status']} cg {auto['cg_iters']} + minres {auto['minres_iters']} quad {e_q:.2e}")
    assert cg_only["status"] == 3
    assert auto["status"] == 0 and auto["cg_iters"] == cap and auto["minres_iters"] > 0
    assert e_q <= 1e-8
    assert float(np.abs(a - ref["alpha"]).max() / np.abs(ref["alpha"]).max()) <= 1e-8
