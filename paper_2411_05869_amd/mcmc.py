"""Bayesian training of the GP by Markov chain Monte Carlo (Appendix C) over
the library's likelihood.

One iteration runs four Metropolis-Hastings blocks and a Gibbs step:

1. the mean coefficients beta (adaptive random walk).  The covariance does
   not change, so only the quadratic form is solved again (gp_loglik with
   GP_LOGDET_NONE on the current matrix; log det is kept);
2. s0, r0, the nugget and, with a stationary Matern core, sigma0 and ell;
3. the bump centres h_ij and radii r_ij;
4. all amplitudes a_ij in {0, 1} at once, proposed from Bernoulli(pi_ij)
   (the prior, so the acceptance ratio is the likelihood ratio);
5. pi_ij ~ Beta(1 + a_ij, 2 - a_ij), the closed-form full conditional.

Blocks 2-4 assemble the proposed covariance and evaluate the full
log-likelihood on the GPU.  Priors follow Sec. 3.1: beta ~ N(0, k I), uniform
priors on (0, bound) for the positive scalars and radii, the domain box for
the centres, Bernoulli(pi) amplitudes with pi ~ U(0, 1); the shapes b_ij
stay 1.

The random walk of a block with m coordinates proposes
v* = v + exp(ls / 2) L e (L L^T = Sigma, e standard normal).  Every 20
iterations it adapts (Haario et al.; Shaby and Wells): with
gamma = (k + 1)^-0.8 at the k-th adaptation, ls += gamma (rate - target)
(target 0.44 for m = 1, else 0.234) and Sigma += gamma (S - Sigma), S the
sample covariance of the block's last 20 states.  Proposals outside the prior
support, and proposals whose likelihood fails (non-positive curvature, no
convergence), are rejected.  With stochastic Lanczos quadrature the log
determinant uses the same probes at every evaluation, so the chain targets
one fixed (deterministic) approximation of the posterior.

All random numbers are inputs: one dict per iteration (z1, u1, z2, u2, z3,
u3, ua, u4, ub), as drawn by ``workloads.mcmc_draws``.
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass, field

import numpy as np

from ._lib import LOGDET_NONE, LOGDET_SLQ, MIXED

_LOG_2PI = math.log(2.0 * math.pi)
_ADAPT = 20


class _RandomWalk:
    def __init__(self, sd):
        sd = np.asarray(sd, np.float64).reshape(-1)
        self.dim = int(sd.size)
        self.log_scale = math.log(2.38 * 2.38 / self.dim) if self.dim else 0.0
        self.cov = np.diag(sd ** 2)
        self._states = []
        self._accepted = 0

    def proposal(self, v, e):
        step = np.linalg.cholesky(self.cov) @ np.asarray(e, np.float64)
        return v + math.exp(self.log_scale / 2.0) * step

    def after(self, t, v, accepted):
        self._states.append(np.array(v, np.float64))
        self._accepted += 1 if accepted else 0
        if t % _ADAPT:
            return
        g = (t // _ADAPT + 1.0) ** -0.8
        target = 0.44 if self.dim == 1 else 0.234
        self.log_scale += g * (self._accepted / _ADAPT - target)
        sample_cov = np.atleast_2d(np.cov(np.stack(self._states), rowvar=False))
        self.cov = self.cov + g * (sample_cov - self.cov)
        self._states.clear()
        self._accepted = 0


@dataclass
class _Layout:
    """Where the coordinates of blocks 2 and 3 live in the hyper-parameters."""
    d: int
    matern: bool
    hshape: tuple = field(default=())

    def scalars(self, th):
        out = [th.s0, *np.asarray(th.r0, np.float64)[: self.d], th.nugget]
        if self.matern:
            out += [th.core.sigma0, *np.asarray(th.core.ell, np.float64)[: self.d]]
        return np.asarray(out, np.float64)

    def with_scalars(self, th, v):
        d = self.d
        th = copy.deepcopy(th)
        th.s0, th.r0, th.nugget = float(v[0]), np.array(v[1:d + 1], np.float64), float(v[d + 1])
        if self.matern:
            th.core.sigma0 = float(v[d + 2])
            ell = np.ones(3)
            ell[:d] = v[d + 3:2 * d + 3]
            th.core.ell = ell
        return th

    def scalars_in_support(self, v, pri):
        d = self.d
        bounds = [pri.s0_max, *np.asarray(pri.r0_max)[:d], pri.nugget_max]
        if self.matern:
            bounds += [pri.sigma0_max, *np.asarray(pri.ell_max)[:d]]
        return bool(np.all(v > 0.0) and np.all(v < np.asarray(bounds, np.float64)))

    def bumps(self, th):
        return np.concatenate([np.asarray(th.h, np.float64).reshape(-1), np.asarray(th.r, np.float64).reshape(-1)])

    def with_bumps(self, th, v):
        th = copy.deepcopy(th)
        k = int(np.prod(self.hshape))
        th.h = np.array(v[:k], np.float64).reshape(self.hshape)
        th.r = np.array(v[k:], np.float64).reshape(self.hshape)
        return th

    def bumps_in_support(self, v, pri):
        k = int(np.prod(self.hshape))
        h = v[:k].reshape(-1, self.d)
        r = v[k:].reshape(-1, self.d)
        lo, hi, rmax = (np.asarray(a, np.float64)[: self.d] for a in (pri.lo, pri.hi, pri.r_max))
        return bool(np.all(h > lo) and np.all(h < hi) and np.all(r > 0.0) and np.all(r < rmax))


class Chain:
    """A chain over (beta, theta, pi) for one data set resident on the GPU.

    ctx, ds: library context and binned training inputs; z: observations
    (device, n float64, original order); W: covariates (device, (p, n)
    float64) or None; theta, beta, pi: the starting state (pi: (n1, n2)).
    """

    def __init__(self, ctx, ds, z, W, theta, beta, pi, priors, precision=MIXED, logdet_mode=LOGDET_SLQ,
                 probe_seed=2411, **solve_opts):
        self.ctx, self.ds, self.z = ctx, ds, z.contiguous()
        self.W = None if W is None else W.contiguous()
        self.pri = priors
        self.prec, self.logdet_mode = precision, logdet_mode
        self.opts = dict(solve_opts, seed=probe_seed)
        self.n = int(z.shape[0])
        self.theta = copy.deepcopy(theta)
        self.beta = np.array(beta, np.float64).reshape(-1)
        self.pi = np.array(pi, np.float64)
        d = len(theta.r0)
        core = getattr(theta, "core", None)
        self.layout = _Layout(d, core is not None and core.kind == 1, tuple(np.asarray(theta.h).shape))
        sd2 = [priors.sd_s0] + [priors.sd_r0] * d + [priors.sd_nugget]
        if self.layout.matern:
            sd2 += [priors.sd_core] * (d + 1)
        nbump = int(np.asarray(theta.h).size)
        self.walks = (_RandomWalk(np.full(self.beta.size, priors.sd_beta)), _RandomWalk(sd2),
                      _RandomWalk([priors.sd_h] * nbump + [priors.sd_r] * nbump))
        self.y = self._residual(self.beta)
        self.K = None
        ll, logdet, K = self._evaluate(self.theta)
        if not math.isfinite(ll):
            raise RuntimeError("the starting state has no finite likelihood")
        self._replace(ll, logdet, K)
        self.t = 0

    # ------------------------------------------------------------ likelihood
    def _residual(self, beta):
        if self.W is None or beta.size == 0:
            return self.z.clone()
        return self.ctx.mean_residual(self.W, beta, self.z)

    def _evaluate(self, theta, y=None):
        """(log-likelihood, log det, matrix) at theta, or -inf when the solve fails."""
        K = self.ctx.assemble(self.ds, theta, self.prec)
        r = self.ctx.loglik(K, self.y if y is None else y, logdet_mode=self.logdet_mode, raise_on_error=False,
                            **self.opts)
        if r["status"] != 0 or not math.isfinite(r["loglik"]):
            K.close()
            return -math.inf, None, None
        return r["loglik"], r["logdet"], K

    def _replace(self, ll, logdet, K):
        if self.K is not None:
            self.K.close()
        self.loglik, self.logdet, self.K = ll, logdet, K

    def _loglik_same_matrix(self, y):
        r = self.ctx.loglik(self.K, y, logdet_mode=LOGDET_NONE, raise_on_error=False, **self.opts)
        if r["status"] != 0:
            return -math.inf
        return -0.5 * self.logdet - 0.5 * r["quad"] - 0.5 * self.n * _LOG_2PI

    def _mh_theta(self, th_new, u):
        """Accept th_new with probability min(1, L(th_new) / L(theta))."""
        ll, logdet, K = self._evaluate(th_new)
        if math.log(u) < ll - self.loglik:
            self.theta = th_new
            self._replace(ll, logdet, K)
            return True
        if K is not None:
            K.close()
        return False

    # ------------------------------------------------------------ iteration
    def step(self, dr, blocks=(1, 2, 3, 4, 5)) -> dict:
        self.t += 1
        t, lay, pri = self.t, self.layout, self.pri
        acc = [False, False, False, False]
        w1, w2, w3 = self.walks
        if 1 in blocks and self.beta.size:
            b_new = w1.proposal(self.beta, dr["z1"])
            y_new = self._residual(b_new)
            ll = self._loglik_same_matrix(y_new)
            log_prior = 0.5 * (float(self.beta @ self.beta) - float(b_new @ b_new)) / pri.beta_var
            if math.log(dr["u1"]) < ll - self.loglik + log_prior:
                self.beta, self.y, self.loglik, acc[0] = b_new, y_new, ll, True
            w1.after(t, self.beta, acc[0])
        if 2 in blocks:
            v_new = w2.proposal(lay.scalars(self.theta), dr["z2"])
            if lay.scalars_in_support(v_new, pri):
                acc[1] = self._mh_theta(lay.with_scalars(self.theta, v_new), dr["u2"])
            w2.after(t, lay.scalars(self.theta), acc[1])
        has_bumps = w3.dim > 0
        if 3 in blocks and has_bumps:
            v_new = w3.proposal(lay.bumps(self.theta), dr["z3"])
            if lay.bumps_in_support(v_new, pri):
                acc[2] = self._mh_theta(lay.with_bumps(self.theta, v_new), dr["u3"])
            w3.after(t, lay.bumps(self.theta), acc[2])
        if 4 in blocks and has_bumps:
            a_now = np.asarray(self.theta.a, np.float64)
            a_new = np.where(np.asarray(dr["ua"]).reshape(a_now.shape) < self.pi, 1.0, 0.0)
            if np.array_equal(a_new, a_now):
                acc[3] = True
            else:
                th_new = copy.deepcopy(self.theta)
                th_new.a = a_new
                acc[3] = self._mh_theta(th_new, dr["u4"])
        if 5 in blocks and has_bumps:
            u = np.asarray(dr["ub"]).reshape(self.pi.shape)
            on = np.asarray(self.theta.a, np.float64) == 1.0
            # inverse distribution functions of Beta(2, 1) and Beta(1, 2)
            self.pi = np.where(on, np.sqrt(u), 1.0 - np.sqrt(1.0 - u))
        return dict(loglik=self.loglik, acc=acc, beta=self.beta.copy(), v2=lay.scalars(self.theta),
                    v3=lay.bumps(self.theta), a=np.array(self.theta.a, np.float64), pi=self.pi.copy())

    def run(self, draws, blocks=(1, 2, 3, 4, 5)) -> list:
        return [self.step(dr, blocks) for dr in draws]

    def close(self):
        if self.K is not None:
            self.K.close()
            self.K = None
