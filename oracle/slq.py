"""Oracle: stochastic Lanczos quadrature for log det K (float64).

Test infrastructure only.

The paper estimates the log-determinant with a Lanczos method (Sec. 3.3; it
used a Lanczos-quadrature package with default settings and reports about
0.1 % error; Sec. 6 names Lanczos quadrature).  The estimator written out
here is the standard stochastic Lanczos quadrature:

  log det K = sum_p log D_pp + log det Ahat,   Ahat = D^{-1/2} K D^{-1/2}
  log det Ahat = tr log Ahat ~ (1/m) sum_l z_l^T log(Ahat) z_l
  z_l^T log(Ahat) z_l ~ |z_l|^2 sum_t tau_t^2 log theta_t

where D = diag K (Jacobi scaling), z_l are Rademacher probes, and
(theta_t, tau_t) are the eigenvalues and first eigenvector components of the
k x k Lanczos tridiagonal matrix started at v_1 = z_l / |z_l| (Gauss
quadrature).  Plain three-term Lanczos, no re-orthogonalisation.

Readings (the paper gives none of these details): m = 30 probes, k = 50
steps by default; a probe's recurrence stops early (breakdown) when
beta_j <= tol (Ahat has unit diagonal, so the threshold is scale-free;
1e-10 for float64 vectors); the estimate is the probe mean and its
standard error sd / sqrt(m).

Probe entries come from a counter-indexed SplitMix64 sequence (Steele, Lea
and Flood, 2014): for seed s, probe l and ORIGINAL point index i, the
counter k = (l << 40 | i) + 1 selects the k-th output of the generator
started at state s, i.e. mix(s + k * 0x9E3779B97F4A7C15 mod 2^64) with the
SplitMix64 output function mix; the entry is -1 when bit 63 is set, else +1.
Keying on the original index makes the probes independent of any reordering.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import eigh_tridiagonal

GAMMA = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
    return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed: int, count: int):
    """First ``count`` outputs of SplitMix64 started at state ``seed``."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = np.uint64(seed) + k * GAMMA
    return splitmix64_mix(st)


def rademacher(seed: int, probe: int, orig_index):
    """Probe entries (+-1.0) for the given original indices."""
    i = np.asarray(orig_index, np.uint64)
    with np.errstate(over="ignore"):
        k = ((np.uint64(probe) << np.uint64(40)) | i) + np.uint64(1)
        st = np.uint64(seed) + k * GAMMA
    out = splitmix64_mix(st)
    return np.where((out >> np.uint64(63)) != 0, -1.0, 1.0)


def lanczos(matvec, v1, k: int, tol: float, reorth: bool = False):
    """Three-term Lanczos from unit v1; returns (alpha[0:j], beta[0:j-1]).

    Plain by default.  With ``reorth`` every new residual is made orthogonal
    to all Lanczos vectors so far by classical Gram-Schmidt applied twice
    (w -= Q (Q^T w), twice) after the alpha step, so the basis stays
    orthonormal to rounding and the recurrence does not amplify rounding."""
    alphas, betas = [], []
    v_prev = np.zeros_like(v1)
    v = v1
    beta_prev = 0.0
    basis = [v1]
    for j in range(k):
        w = matvec(v) - beta_prev * v_prev
        a = float(v @ w)
        w = w - a * v
        if reorth:
            Q = np.array(basis)
            for _ in range(2):
                w = w - Q.T @ (Q @ w)
        alphas.append(a)
        if j == k - 1:
            break
        b = float(math.sqrt(w @ w))
        if b <= tol:
            break
        betas.append(b)
        v_prev, v = v, w / b
        beta_prev = b
        if reorth:
            basis.append(v)
    return np.array(alphas), np.array(betas)


def gauss_quadrature_log(alphas, betas, znorm2: float) -> float:
    """|z|^2 sum_t tau_t^2 log theta_t from the Lanczos tridiagonal."""
    if len(alphas) == 1:
        return znorm2 * math.log(alphas[0])
    theta, Q = eigh_tridiagonal(alphas, betas)
    tau2 = Q[0, :] ** 2
    return znorm2 * float(np.sum(tau2 * np.log(theta)))


def slq_logdet(A, seed: int, n_probes: int = 30, n_steps: int = 50, tol: float = 1e-10,
               orig_index=None, reorth: bool = False):
    """SLQ estimate of log det A for sparse or dense SPD A (rows in the order
    of ``orig_index``; identity order if None); plain Lanczos, or with full
    re-orthogonalisation (``reorth``).  Returns dict with the estimate, its
    standard error, per-probe quadratures and the Jacobi part."""
    n = A.shape[0]
    diag = np.asarray(A.diagonal(), np.float64)
    s = 1.0 / np.sqrt(diag)
    if orig_index is None:
        orig_index = np.arange(n)

    def matvec(v):
        return s * (A @ (s * v))

    gam = np.empty(n_probes)
    steps = np.empty(n_probes, np.int64)
    for l in range(n_probes):
        z = rademacher(seed, l, orig_index)
        znorm2 = float(z @ z)
        al, be = lanczos(matvec, z / math.sqrt(znorm2), n_steps, tol, reorth)
        gam[l] = gauss_quadrature_log(al, be, znorm2)
        steps[l] = len(al)
    jac = float(np.sum(np.log(diag)))
    est = jac + float(np.mean(gam))
    se = float(np.std(gam, ddof=1) / math.sqrt(n_probes)) if n_probes > 1 else float("nan")
    return dict(logdet=est, se=se, gammas=gam, jacobi=jac, steps=steps)
