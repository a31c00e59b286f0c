"""Oracle: the Markov chain Monte Carlo training of Appendix C (float64).

Test infrastructure only: never imported by the HIP product path.

The posterior (Eq. posteriorZ) of the mean coefficients beta and the kernel
hyper-parameters is sampled by four Metropolis-Hastings blocks and a Gibbs
step per iteration (Appendix C):

1. beta, by an adaptive random walk;
2. s0, r0, the nugget and (with a stationary Matern core) sigma0 and ell,
   by an adaptive random walk;
3. the bump centres h_ij and radii r_ij, by an adaptive random walk;
4. all amplitudes a_ij at once, proposed from their prior Bernoulli(pi_ij),
   so the acceptance ratio is the likelihood ratio;
5. pi_ij from its full conditional Beta(1 + a_ij, 2 - a_ij).

Priors (Sec. 3.1): beta ~ N(0, k I); s0, r0, the nugget, r_ij and the core's
sigma0 and ell uniform on (0, upper bound); h_ij uniform on the domain box;
a_ij ~ Bernoulli(pi_ij); pi_ij ~ U(0, 1); the shapes b_ij stay 1.  The
likelihood is the Gaussian one of Eq. Zmarg with residual z - W beta.

Readings (the appendix names the samplers, not their constants):

* the random walk of a block of dimension m proposes v* = v + exp(ls / 2) L e
  with L the lower Cholesky factor of the block's proposal covariance Sigma
  and e the block's standard normals;
* adaptation (after Haario et al. and Shaby and Wells): every A = 20
  iterations, with k = t / A and gamma = (k + 1)^-0.8, the log scale moves
  by gamma (acceptance rate of the last A iterations - target), target 0.44
  for m = 1 and 0.234 otherwise, and Sigma <- Sigma + gamma (S - Sigma) with
  S the sample covariance (divisor A - 1) of the block's states after each
  of those A iterations; ls starts at log(2.38^2 / m), Sigma at
  diag(initial standard deviations^2);
* a proposal outside the prior support, or one whose matrix is not
  positive definite, is rejected (its uniform is still used up);
* an amplitude proposal equal to the current amplitudes is accepted without
  a new likelihood;
* the Beta(1 + a, 2 - a) draw is the inverse distribution function at a
  uniform: sqrt(u) for a = 1 (Beta(2, 1)), 1 - sqrt(1 - u) for a = 0
  (Beta(1, 2)).

Every random number comes from ``workloads.mcmc_draws`` (an input).
"""
from __future__ import annotations

import copy
import math

import numpy as np

from . import kernel, likelihood

ADAPT_EVERY = 20


def loglik(x, th, y):
    """log p(z | beta, theta) for the residual y, by dense Cholesky; -inf when
    the matrix is not positive definite."""
    K, _ = kernel.dense(x, th)
    try:
        return likelihood.dense_cholesky(K, y)["loglik"]
    except np.linalg.LinAlgError:
        return -math.inf


def _matern(th):
    c = getattr(th, "core", None)
    return c is not None and c.kind == 1


def get_v2(th):
    d = len(th.r0)
    v = [th.s0, *np.asarray(th.r0, float)[:d], th.nugget]
    if _matern(th):
        v += [th.core.sigma0, *np.asarray(th.core.ell, float)[:d]]
    return np.array(v, float)


def put_v2(th, v):
    d = len(th.r0)
    t = copy.deepcopy(th)
    t.s0 = float(v[0])
    t.r0 = np.array(v[1:1 + d], float)
    t.nugget = float(v[1 + d])
    if _matern(th):
        t.core.sigma0 = float(v[2 + d])
        ell = np.ones(3)
        ell[:d] = v[3 + d:3 + 2 * d]
        t.core.ell = ell
    return t


def logprior_v2(th, v, pri):
    d = len(th.r0)
    ok = 0.0 < v[0] < pri.s0_max and all(0.0 < v[1 + k] < pri.r0_max[k] for k in range(d)) \
        and 0.0 < v[1 + d] < pri.nugget_max
    if _matern(th):
        ok = ok and 0.0 < v[2 + d] < pri.sigma0_max and all(0.0 < v[3 + d + k] < pri.ell_max[k] for k in range(d))
    return 0.0 if ok else -math.inf


def get_v3(th):
    return np.concatenate([np.asarray(th.h, float).ravel(), np.asarray(th.r, float).ravel()])


def put_v3(th, v):
    t = copy.deepcopy(th)
    nh = np.asarray(th.h).size
    t.h = np.array(v[:nh], float).reshape(np.asarray(th.h).shape)
    t.r = np.array(v[nh:], float).reshape(np.asarray(th.r).shape)
    return t


def logprior_v3(th, v, pri):
    d = len(th.r0)
    nh = np.asarray(th.h).size
    h = v[:nh].reshape(-1, d)
    r = v[nh:].reshape(-1, d)
    ok = np.all(h > pri.lo[:d]) and np.all(h < pri.hi[:d]) and np.all(r > 0.0) and np.all(r < pri.r_max[:d])
    return 0.0 if ok else -math.inf


class _Walk:
    """Adaptive random-walk state of one block."""

    def __init__(self, sd):
        sd = np.asarray(sd, float)
        self.m = sd.size
        self.ls = math.log(2.38 ** 2 / self.m) if self.m else 0.0
        self.Sig = np.diag(sd * sd)
        self.hist = []
        self.acc = 0

    def propose(self, v, e):
        L = np.linalg.cholesky(self.Sig)
        return v + math.exp(0.5 * self.ls) * (L @ e)

    def record(self, v, accepted, t):
        self.hist.append(np.array(v, float))
        self.acc += int(accepted)
        if t % ADAPT_EVERY == 0:
            k = t // ADAPT_EVERY
            gamma = (k + 1.0) ** -0.8
            rate = self.acc / ADAPT_EVERY
            target = 0.44 if self.m == 1 else 0.234
            self.ls += gamma * (rate - target)
            S = np.atleast_2d(np.cov(np.array(self.hist), rowvar=False))
            self.Sig = self.Sig + gamma * (S - self.Sig)
            self.hist = []
            self.acc = 0


def run(x, z, W, th0, beta0, pi0, pri, draws, blocks=(1, 2, 3, 4, 5)):
    """Runs len(draws) iterations from (beta0, th0, pi0).  W: (p, n) covariates.
    ``blocks`` lists the updates that run (1-4 as above, 5 the Gibbs step); the
    others keep their values (their random numbers are still used up).
    Returns one record per iteration: loglik after the iteration, the four
    acceptance flags, and the state (beta, v2, v3, a, pi)."""
    x = np.asarray(x, float)
    z = np.asarray(z, float)
    W = np.asarray(W, float).reshape(-1, x.shape[0])
    beta = np.array(beta0, float)
    th = copy.deepcopy(th0)
    pi = np.array(pi0, float)
    d = x.shape[1]
    sd2 = [pri.sd_s0, *[pri.sd_r0] * d, pri.sd_nugget]
    if _matern(th):
        sd2 += [pri.sd_core] * (1 + d)
    nh = np.asarray(th.h).size
    w1 = _Walk(np.full(beta.size, pri.sd_beta))
    w2 = _Walk(np.array(sd2))
    w3 = _Walk(np.concatenate([np.full(nh, pri.sd_h), np.full(nh, pri.sd_r)]))
    y = z - beta @ W
    ll = loglik(x, th, y)
    out = []
    for t, dr in enumerate(draws, start=1):
        acc = [False] * 4
        # block 1: beta (the matrix is unchanged)
        if 1 in blocks and beta.size:
            bs = w1.propose(beta, dr["z1"])
            ys = z - bs @ W
            lls = loglik(x, th, ys)
            lpr = -0.5 * float(bs @ bs) / pri.beta_var + 0.5 * float(beta @ beta) / pri.beta_var
            if math.log(dr["u1"]) < lls - ll + lpr:
                beta, y, ll, acc[0] = bs, ys, lls, True
            w1.record(beta, acc[0], t)
        # block 2: s0, r0, nugget (and the Matern core's sigma0, ell)
        if 2 in blocks:
            v = get_v2(th)
            vs = w2.propose(v, dr["z2"])
            if logprior_v2(th, vs, pri) == 0.0:
                ths = put_v2(th, vs)
                lls = loglik(x, ths, y)
                if math.log(dr["u2"]) < lls - ll:
                    th, ll, acc[1] = ths, lls, True
            w2.record(get_v2(th), acc[1], t)
        # block 3: bump centres and radii
        if 3 in blocks and nh:
            v = get_v3(th)
            vs = w3.propose(v, dr["z3"])
            if logprior_v3(th, vs, pri) == 0.0:
                ths = put_v3(th, vs)
                lls = loglik(x, ths, y)
                if math.log(dr["u3"]) < lls - ll:
                    th, ll, acc[2] = ths, lls, True
            w3.record(get_v3(th), acc[2], t)
        # block 4: amplitudes from their prior
        if 4 in blocks and nh:
            a = np.asarray(th.a, float)
            a_s = (dr["ua"].reshape(a.shape) < pi).astype(float)
            if np.array_equal(a_s, a):
                acc[3] = True
            else:
                ths = copy.deepcopy(th)
                ths.a = a_s
                lls = loglik(x, ths, y)
                if math.log(dr["u4"]) < lls - ll:
                    th, ll, acc[3] = ths, lls, True
        # Gibbs: pi_ij ~ Beta(1 + a_ij, 2 - a_ij)
        if 5 in blocks and nh:
            ub = dr["ub"].reshape(pi.shape)
            a = np.asarray(th.a, float)
            pi = np.where(a == 1.0, np.sqrt(ub), 1.0 - np.sqrt(1.0 - ub))
        out.append(dict(loglik=ll, acc=acc, beta=beta.copy(), v2=get_v2(th), v3=get_v3(th),
                        a=np.array(th.a, float),
                        pi=pi.copy()))
    return out
