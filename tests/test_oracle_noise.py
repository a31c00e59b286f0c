"""Pins of the oracle's per-point error variances (Sec. 3.1, Eq. Zcov:
Delta = diag[tau^2(x_1), ..., tau^2(x_N)] added to Omega), here a constant
nugget sigma^2 plus tau2[p] on the diagonal.

Checks: the closed form of a diagonal K; K(tau2) - K(0) is zero off the
diagonal and tau2 on it; a constant tau2 equals a larger nugget; the
KD-tree route equals brute force; the log-likelihood equals SciPy's
multivariate normal density; the predictor at the training inputs is
y - (sigma^2 + tau2) alpha (the error variances belong to the observations,
not to the cross-covariance); the variance at a training input is
(sigma^2 + tau2_p) - (sigma^2 + tau2_p)^2 (K^-1)_pp; bad inputs are refused."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import kernel, likelihood, predict
from workloads import noise_variances, uniform_problem


def _with_tau2(p, seed=5, lo=0.0, hi=0.05):
    th = p.theta.copy()
    th.tau2 = noise_variances(p.n, seed, lo, hi)
    return th


def test_diagonal_closed_form_per_point():
    # r0 below the minimum pair distance, all a = 0: K = diag(s0 + sigma^2 + tau2_p)
    p = uniform_problem(400, 2, 3, r0=1e-6, n1=2, n2=2)
    p.theta.a[:] = 0.0
    th = _with_tau2(p, hi=2.0)
    K, P = kernel.dense(p.x, th)
    assert P.sum() == p.n
    k = (th.s0 + th.nugget) + th.tau2
    y = p.z_std
    expect = -0.5 * float(np.sum(np.log(k))) - 0.5 * float(np.sum(y * y / k)) - 0.5 * p.n * math.log(2 * math.pi)
    for r in (likelihood.dense_cholesky(K, y),
              likelihood.sparse_lu(kernel.to_scipy(*kernel.sparse(p.x, th), p.n), y)):
        assert abs(r["loglik"] - expect) <= 1e-12 * abs(expect)


def test_tau2_only_on_the_diagonal():
    p = uniform_problem(300, 2, 8, r0=0.12, n1=2, n2=2, bump_radius=0.25)
    th = _with_tau2(p)
    K0, P0 = kernel.dense(p.x, p.theta)
    K1, P1 = kernel.dense(p.x, th)
    assert np.array_equal(P0, P1)
    off = ~np.eye(p.n, dtype=bool)
    assert np.array_equal(K0[off], K1[off])
    dd = np.diag(K1) - np.diag(K0)
    assert np.all(np.abs(dd - th.tau2) <= 4 * np.spacing(np.diag(K1)))


def test_constant_tau2_is_a_larger_nugget():
    p = uniform_problem(300, 3, 9, r0=0.2, n1=2, n2=2, bump_radius=0.3)
    th = p.theta.copy()
    th.tau2 = np.full(p.n, 0.03)
    th_n = p.theta.copy()
    th_n.nugget = p.theta.nugget + 0.03
    K1, _ = kernel.dense(p.x, th)
    K2, _ = kernel.dense(p.x, th_n)
    assert np.allclose(K1, K2, rtol=1e-15, atol=0)
    y = p.z_std
    a, b = likelihood.dense_cholesky(K1, y)["loglik"], likelihood.dense_cholesky(K2, y)["loglik"]
    assert abs(a - b) <= 1e-13 * abs(b)


def test_kdtree_route_equals_brute_force_with_tau2():
    p = uniform_problem(500, 2, 10, r0=0.08, n1=3, n2=2, bump_radius=0.2)
    th = _with_tau2(p)
    K, P = kernel.dense(p.x, th)
    ip, ci, vv = kernel.sparse(p.x, th)
    for r in range(p.n):
        cols = ci[ip[r]:ip[r + 1]]
        assert np.array_equal(cols, np.nonzero(P[r])[0])
        assert np.array_equal(vv[ip[r]:ip[r + 1]], K[r, cols])
    c, v = kernel.row(p.x, th, 123)
    assert np.array_equal(v, K[123, c])


def test_loglik_is_the_multivariate_normal_density():
    p = uniform_problem(250, 2, 11, r0=0.15, n1=2, n2=2, bump_radius=0.3)
    th = _with_tau2(p, hi=0.5)
    K, _ = kernel.dense(p.x, th)
    y = np.random.default_rng(4).standard_normal(p.n)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(p.n), cov=K).logpdf(y)
    assert abs(likelihood.dense_cholesky(K, y)["loglik"] - ref) <= 1e-10 * abs(ref)


def test_predictor_and_variance_at_training_inputs():
    p = uniform_problem(300, 2, 12, r0=0.12, n1=2, n2=2, bump_radius=0.25)
    th = _with_tau2(p, hi=0.2)
    K, _ = kernel.dense(p.x, th)
    y = np.linalg.cholesky(K) @ p.z_std
    alpha = likelihood.dense_cholesky(K, y)["alpha"]
    delta = th.nugget + th.tau2
    m = predict.mean(p.x, p.x, th, alpha)
    assert np.allclose(m, y - delta * alpha, rtol=0, atol=1e-10 * np.abs(y).max())
    idx = np.arange(0, p.n, 11)
    v = predict.variance(p.x[idx], p.x, th)
    Kinv = np.linalg.inv(K)
    assert np.allclose(v, delta[idx] - delta[idx] ** 2 * np.diag(Kinv)[idx], rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("bad", ["negative", "nan", "length"])
def test_bad_tau2_is_refused(bad):
    p = uniform_problem(50, 2, 13)
    th = p.theta.copy()
    t = np.full(p.n, 0.1)
    if bad == "negative":
        t[7] = -1e-3
    elif bad == "nan":
        t[7] = np.nan
    else:
        t = t[:-1]
    th.tau2 = t
    with pytest.raises(ValueError):
        kernel.dense(p.x, th)
