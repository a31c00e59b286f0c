"""GPU parity of the kriging mean (Sec. 3.2) against the FP64 oracle.

FP64: relative error <= 1e-10 of the scale sum_q |C(x*, x_q)| |alpha_q|
(the sum is formed in a different order and grouping).  Mixed (float32
cross-covariance values and alpha): <= 2e-7 of the same scale, a few
float32 roundings per term."""
import numpy as np
import pytest

from oracle import kernel, likelihood, predict
from workloads import uniform_problem
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


def _scale(xs, p, alpha):
    rp, cols, vals = kernel.cross_entries(xs, p.x, p.theta)
    s = np.zeros(xs.shape[0])
    for i in range(xs.shape[0]):
        s[i] = np.abs(vals[rp[i]:rp[i + 1]]) @ np.abs(alpha[cols[rp[i]:rp[i + 1]]])
    return s


@pytest.mark.parametrize("d", [1, 2, 3])
def test_predict_matches_oracle(ctx, d):
    p = uniform_problem(500, d, 70 + d, r0=0.12 if d > 1 else 0.01, n1=3, n2=2, bump_radius=0.25)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    alpha = likelihood.dense_cholesky(K, y)["alpha"]
    rng = np.random.default_rng(d)
    xs = rng.uniform(-0.2, 1.2, (300, d))     # some test points outside the training box
    ref = predict.mean(xs, p.x, p.theta, alpha)
    sc = _scale(xs, p, alpha) + 1e-300
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    pred = ctx.predictor(ds, p.theta, dev(alpha))
    for prec, tol in ((0, 1e-10), (1, 2e-7)):
        m = host(ctx.predict(pred, dev(xs), precision=prec))
        err = float(np.max(np.abs(m - ref) / sc))
        print(f"[predict d={d} prec={prec}] max scaled error {err:.2e}")
        assert err <= tol


def test_identity_at_training_inputs(ctx):
    import torch
    p = uniform_problem(800, 2, 5, r0=0.08, n1=2, n2=3, bump_radius=0.2)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    Kg = ctx.assemble(ds, p.theta, 0)
    alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
    ctx.solve(Kg, dev(y), alpha, rtol=1e-12)
    pred = ctx.predictor(ds, p.theta, alpha)
    m = host(ctx.predict(pred, dev(p.x)))
    a = host(alpha)
    err = np.abs(m - (y - p.theta.nugget * a)).max() / np.abs(y).max()
    print(f"[identity] max error {err:.2e}")
    assert err <= 1e-9


def test_empty_request(ctx):
    import torch
    p = uniform_problem(50, 2, 5)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    pred = ctx.predictor(ds, p.theta, dev(np.ones(p.n)))
    out = ctx.predict(pred, torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert out.shape == (0,)
