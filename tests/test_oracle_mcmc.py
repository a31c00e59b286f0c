"""Pins of the MCMC oracle (``oracle.mcmc``, Appendix C).

* The beta block alone, with the kernel fixed, targets the conjugate
  Gaussian posterior N(m, V), V = (W K^-1 W^T + I / k)^-1,
  m = V W K^-1 z: the chain's mean and variance match it.
* The Gibbs step alone draws pi_ij from Beta(1 + a_ij, 2 - a_ij)
  (Kolmogorov-Smirnov against scipy's Beta).
* With every bump away from the data the likelihood does not depend on the
  amplitudes, so the amplitude block accepts every proposal and, together
  with the Gibbs step, leaves the prior invariant: P(a_ij = 1) = 1/2.
* The recorded log-likelihood equals a fresh evaluation at the recorded
  state.
"""
import math

import numpy as np
import scipy.stats

from oracle import kernel, likelihood
from oracle import mcmc as om
from workloads import McmcPriors, mcmc_draws, mean_covariates, uniform_problem


def _problem(n=60, seed=21, beta_true=(0.7, -1.2)):
    p = uniform_problem(n, 1, seed, r0=0.15, n1=2, n2=2, bump_radius=0.3)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    W = mean_covariates(p.x)
    z = np.asarray(beta_true) @ W + y
    pri = McmcPriors(lo=np.zeros(3), hi=np.ones(3), r0_max=np.full(3, 1.0), r_max=np.full(3, 1.0), sd_beta=0.3)
    return p, K, W, z, pri


def test_beta_block_targets_the_conjugate_posterior():
    p, K, W, z, pri = _problem()
    Ki = np.linalg.inv(K)
    V = np.linalg.inv(W @ Ki @ W.T + np.eye(2) / pri.beta_var)
    m = V @ W @ Ki @ z
    n_it = 4000
    draws = mcmc_draws(5, n_it, 2, 3, 8, 4)
    chain = om.run(p.x, z, W, p.theta, np.zeros(2), np.full((2, 2), 0.5), pri, draws, blocks=(1,))
    B = np.array([r["beta"] for r in chain[500:]])
    sd = np.sqrt(np.diag(V))
    rate = np.mean([r["acc"][0] for r in chain[500:]])
    print("chain mean", B.mean(0), "posterior mean", m, "sd", sd, "var ratio", B.var(0) / np.diag(V), "acc", rate)
    assert np.all(np.abs(B.mean(0) - m) < 0.3 * sd)
    assert np.all((B.var(0) / np.diag(V) > 0.6) & (B.var(0) / np.diag(V) < 1.5))
    assert 0.1 < rate < 0.6


def test_gibbs_step_draws_beta():
    p, K, W, z, pri = _problem()
    a = np.array([[1.0, 0.0], [0.0, 1.0]])
    th = p.theta.copy()
    th.a = a
    draws = mcmc_draws(6, 1500, 2, 3, 8, 4)
    chain = om.run(p.x, z, W, th, np.zeros(2), np.full((2, 2), 0.5), pri, draws, blocks=(5,))
    P = np.array([r["pi"] for r in chain])
    on = P[:, a == 1.0].ravel()
    off = P[:, a == 0.0].ravel()
    assert scipy.stats.kstest(on, scipy.stats.beta(2, 1).cdf).pvalue > 1e-3
    assert scipy.stats.kstest(off, scipy.stats.beta(1, 2).cdf).pvalue > 1e-3


def test_amplitudes_keep_the_prior_when_the_likelihood_is_flat():
    p, K, W, z, pri = _problem()
    th = p.theta.copy()
    th.h = th.h + 50.0      # every bump far from the data: no point is in a group
    th.a = np.ones_like(th.a)
    draws = mcmc_draws(7, 3000, 2, 3, 8, 4)
    chain = om.run(p.x, z, W, th, np.zeros(2), np.full((2, 2), 0.5), pri, draws, blocks=(4, 5))
    assert all(r["acc"][3] for r in chain)
    A = np.array([r["a"] for r in chain[100:]])
    freq = A.mean()
    print("P(a = 1)", freq)
    assert abs(freq - 0.5) < 0.05


def test_recorded_loglik_matches_the_state():
    p, K, W, z, pri = _problem(n=50)
    draws = mcmc_draws(8, 30, 2, 3, 8, 4)
    chain = om.run(p.x, z, W, p.theta, np.zeros(2), np.full((2, 2), 0.5), pri, draws)
    r = chain[-1]
    th = om.put_v3(om.put_v2(p.theta, r["v2"]), r["v3"])
    th.a = r["a"]
    y = z - r["beta"] @ W
    Kr, _ = kernel.dense(p.x, th)
    assert math.isclose(r["loglik"], likelihood.dense_cholesky(Kr, y)["loglik"], rel_tol=1e-12)
    assert any(any(rr["acc"][:3]) for rr in chain)
