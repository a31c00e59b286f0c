"""GPU parity of the log-likelihood against the FP64 oracle.

Tolerances (per component; the error is printed for every result):
  * quadratic form y^T K^-1 y and alpha: 1e-8 relative (FP64), 1e-5 (mixed);
  * log det in exact mode vs dense Cholesky: 1e-8 (FP64), 1e-5 (mixed);
  * SLQ log det vs the oracle's SLQ with identical probes: 1e-8 (FP64),
    1e-5 (mixed); SLQ vs the exact log det: within 3 standard errors;
  * full log-likelihood in exact mode: 1e-8 (FP64), 1e-5 (mixed)."""
import math

import numpy as np
import pytest

from oracle import kernel, likelihood, slq
from workloads import config1, uniform_problem
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
    ref = likelihood.dense_cholesky(K, y)
    return p, K, y, ref


def _setup(ctx, p, prec):
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    return ds, ctx.assemble(ds, p.theta, prec)


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-5)])
def test_exact_mode_config1(ctx, cfg1, prec, tol):
    from paper_2411_05869_amd import LOGDET_EXACT
    import torch
    p, K, y, ref = cfg1
    ds, Kg = _setup(ctx, p, prec)
    alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
    r = ctx.loglik(Kg, dev(y), alpha_out=alpha, logdet_mode=LOGDET_EXACT)
    errs = dict(loglik=rel(r["loglik"], ref["loglik"]), logdet=rel(r["logdet"], ref["logdet"]),
                quad=rel(r["quad"], ref["quad"]),
                alpha=float(np.abs(host(alpha) - ref["alpha"]).max() / np.abs(ref["alpha"]).max()))
    print(f"[cfg1 exact prec={prec}] iters={r['cg_iters']} refresh={r['refreshes']} relres={r['relres']:.2e} errors={errs}")
    assert r["status"] == 0
    for k, v in errs.items():
        assert v <= tol, (k, v)


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-5)])
def test_slq_matches_oracle_slq(ctx, cfg1, prec, tol):
    p, K, y, ref = cfg1
    ds, Kg = _setup(ctx, p, prec)
    seed = 20241108
    r = ctx.loglik(Kg, dev(y), seed=seed, n_probes=30, n_lanczos=50)
    o = slq.slq_logdet(K, seed=seed, n_probes=30, n_steps=50)
    e_slq = rel(r["logdet"], o["logdet"])
    e_exact = abs(r["logdet"] - ref["logdet"])
    print(f"[cfg1 slq prec={prec}] gpu {r['logdet']:.12g} oracle-slq {o['logdet']:.12g} rel {e_slq:.2e}; "
          f"exact {ref['logdet']:.12g} |err| {e_exact:.3g} se {r['logdet_se']:.3g} (oracle se {o['se']:.3g})")
    assert e_slq <= tol
    assert e_exact <= 3 * r["logdet_se"]
    assert rel(r["logdet_se"], o["se"]) < (1e-4 if prec == 0 else 1e-2)


def test_mixed_vs_fp64_same_gpu(ctx, cfg1):
    from paper_2411_05869_amd import LOGDET_EXACT
    p, K, y, ref = cfg1
    out = {}
    for prec in (0, 1):
        ds, Kg = _setup(ctx, p, prec)
        out[prec] = ctx.loglik(Kg, dev(y), seed=7)
    e = rel(out[1]["loglik"], out[0]["loglik"])
    print(f"[cfg1 mixed vs fp64, same probes] rel {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("d", [1, 2, 3])
def test_random_theta_small(ctx, d):
    from paper_2411_05869_amd import LOGDET_EXACT
    for seed, n in [(31, 100), (32, 500)]:
        p = uniform_problem(n, d, seed + d, r0=0.15 if d > 1 else 0.02, n1=2, n2=3, bump_radius=0.25)
        K, _ = kernel.dense(p.x, p.theta)
        y = np.linalg.cholesky(K) @ p.z_std
        ref = likelihood.dense_cholesky(K, y)
        ds, Kg = _setup(ctx, p, 0)
        r = ctx.loglik(Kg, dev(y), logdet_mode=LOGDET_EXACT)
        e = rel(r["loglik"], ref["loglik"])
        print(f"[random d={d} n={n}] loglik rel err {e:.2e} iters {r['cg_iters']}")
        assert e <= 1e-8


def test_diagonal_closed_form(ctx):
    from paper_2411_05869_amd import LOGDET_EXACT
    p = uniform_problem(300, 2, 9, r0=1e-7, n1=1, n2=1, bump_radius=1e-4)
    p.theta.a[:] = 0.0
    p.theta.s0 = 1.7
    y = p.z_std
    c = p.theta.s0 + p.theta.nugget
    expect = -0.5 * p.n * math.log(c) - 0.5 * float(y @ y) / c - 0.5 * p.n * math.log(2 * math.pi)
    ds, Kg = _setup(ctx, p, 0)
    for mode in (0, LOGDET_EXACT):
        r = ctx.loglik(Kg, dev(y), logdet_mode=mode)
        print(f"[diagonal mode={mode}] rel {rel(r['loglik'], expect):.2e} steps {r['lanczos_steps']}")
        assert rel(r["loglik"], expect) <= 1e-12


def test_not_converged_reports_enotconv(ctx, cfg1):
    p, K, y, ref = cfg1
    ds, Kg = _setup(ctx, p, 0)
    r = ctx.loglik(Kg, dev(y), raise_on_error=False, max_iter=1)
    assert r["status"] == 3 and r["cg_iters"] == 1 and r["relres"] > 1e-10


def test_deterministic(ctx, cfg1):
    p, K, y, ref = cfg1
    a = []
    for _ in range(2):
        ds, Kg = _setup(ctx, p, 1)
        a.append(ctx.loglik(Kg, dev(y), seed=3))
    assert a[0] == a[1]


@pytest.mark.parametrize("prec", [0, 1])
def test_block_jacobi_matches_jacobi(ctx, cfg1, prec):
    from paper_2411_05869_amd import LOGDET_NONE, PRECOND_BLOCK_JACOBI, PRECOND_JACOBI
    p, K, y, ref = cfg1
    ds, Kg = _setup(ctx, p, prec)
    out = {}
    for pc in (PRECOND_JACOBI, PRECOND_BLOCK_JACOBI):
        out[pc] = ctx.loglik(Kg, dev(y), precond=pc, logdet_mode=LOGDET_NONE)
    e = {pc: rel(out[pc]["quad"], ref["quad"]) for pc in out}
    print(f"[precond prec={prec}] iters jacobi {out[0]['cg_iters']} block {out[1]['cg_iters']}; quad errors {e}")
    tol = 1e-8 if prec == 0 else 1e-5
    assert e[0] <= tol and e[1] <= tol
    assert out[1]["cg_iters"] < out[0]["cg_iters"]
