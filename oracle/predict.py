"""Oracle: posterior (kriging) mean at test points (float64).

Test infrastructure only.

Sec. 3.2 gives m_{y|z} = W_P beta + C_{y,z} C_z^{-1} (z - W beta).  With the
residual y = z - W beta passed in and a zero prior mean at the test points
(the mean term is the caller's), this is

    m(x*) = sum_q C_y(x*, x_q) alpha_q,   alpha = C_z^{-1} y,

where C_y = C_core C_sparse (Eq. sparseCov) carries no nugget (the
nugget belongs to the observations z, Eq. Zcov).  At the training inputs
m(X) = (C_z - sigma^2 I) alpha = y - sigma^2 alpha.

The same passage gives the conditional covariance
C_{y|z} = C_y - C_{y,z} C_z^{-1} C_{z,y}; its diagonal at the test points is

    v(x*) = C_y(x*, x*) - c^T C_z^{-1} c,   c = C_{z,y}(., x*),

the posterior variance of the latent process (no nugget: a new observation
would add sigma^2).
"""

from __future__ import annotations

import numpy as np

from . import kernel


def mean(xs, x, th, alpha, block: int = 256):
    """m(x*) for every row of xs, by brute force over all training points."""
    xs = np.asarray(xs, np.float64)
    x = np.asarray(x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    M, F = kernel.features(x, th)
    Ms, Fs = kernel.features(xs, th)
    out = np.empty(xs.shape[0])
    for s in range(0, xs.shape[0], block):
        e = min(xs.shape[0], s + block)
        xp = xs[s:e, None, :]
        xq = x[None, :, :]
        same = np.zeros((e - s, x.shape[0]), bool)
        P = kernel.pattern_pred(xp, xq, Ms[s:e, None, :], M[None, :, :], same, th)
        v = kernel.entries(xp, xq, Ms[s:e, None, :], M[None, :, :], Fs[s:e, None, :], F[None, :, :],
                           same, th)
        out[s:e] = np.where(P, v, 0.0) @ alpha
    return out


def mean_rows(xs, x, th, alpha):
    """Same as ``mean`` but through the sparse cross-covariance rows."""
    rp, cols, vals = kernel.cross_entries(xs, x, th)
    alpha = np.asarray(alpha, np.float64)
    out = np.empty(xs.shape[0])
    for s in range(xs.shape[0]):
        out[s] = vals[rp[s]:rp[s + 1]] @ alpha[cols[rp[s]:rp[s + 1]]]
    return out


def prior_variance(xs, th):
    """C_y(x*, x*) for every test point (Eq. sparseCov at x = x'; no nugget)."""
    xs = np.asarray(xs, np.float64)
    Ms, Fs = kernel.features(xs, th)
    return kernel.entries(xs, xs, Ms, Ms, Fs, Fs, np.zeros(xs.shape[0], bool), th)


def variance(xs, x, th):
    """diag C_{y|z} at the test points: C_y(x*, x*) - c^T C_z^{-1} c, with the
    dense Cholesky factor L of C_z (c^T C_z^{-1} c = |L^{-1} c|^2)."""
    import scipy.linalg as sla
    xs = np.asarray(xs, np.float64)
    x = np.asarray(x, np.float64)
    K, _ = kernel.dense(x, th)
    L = np.linalg.cholesky(K)
    rp, cols, vals = kernel.cross_entries(xs, x, th)
    C = np.zeros((x.shape[0], xs.shape[0]))
    for s in range(xs.shape[0]):
        C[cols[rp[s]:rp[s + 1]], s] = vals[rp[s]:rp[s + 1]]
    V = sla.solve_triangular(L, C, lower=True)
    return prior_variance(xs, th) - np.sum(V * V, axis=0)


def variance_split(xs, x, th):
    """The same diagonal through the split K = A + F F^T of Proposition 1's
    proof (A: the local Wendland part plus the nugget, F: the bump sums of the
    masked points), for larger n without a core kernel: c^T K^{-1} c with
    K^{-1} C from one sparse factorisation (``likelihood.split_solve``)."""
    import copy

    from . import likelihood
    xs = np.asarray(xs, np.float64)
    x = np.asarray(x, np.float64)
    if getattr(th, "core", None) is not None and th.core.kind != 0:
        raise ValueError("the split K = A + F F^T needs a unit core kernel")
    th_local = copy.deepcopy(th)
    th_local.a = np.zeros_like(np.asarray(th_local.a, np.float64))
    ip, ci, vv = kernel.sparse(x, th_local)
    A = kernel.to_scipy(ip, ci, vv, x.shape[0])
    M, F = kernel.features(x, th)
    rp, cols, vals = kernel.cross_entries(xs, x, th, M=M, F=F)
    C = np.zeros((x.shape[0], xs.shape[0]))
    for s in range(xs.shape[0]):
        C[cols[rp[s]:rp[s + 1]], s] = vals[rp[s]:rp[s + 1]]
    W = likelihood.split_solve(A, np.where(M, F, 0.0), C)
    return prior_variance(xs, th) - np.sum(C * W, axis=0)
