"""Oracle: the core kernel of C_y = C_core x C_sparse (float64).

Test infrastructure only: never imported by the HIP product path.

Definitions followed:

* the kernel is the product C_y(x, x') = C_core(x, x') C_sparse(x, x')
  (Sec. 2, Eq. sparseCov); the nugget of Eq. Zcov is added afterwards, on the
  index diagonal, and is not multiplied by the core;
* Matern correlation with smoothness nu (Sec. 2.2 names the Matern class; the
  paper's experiments use nu = 5/2, Sec. 4.1):
      M_nu(t) = 2^(1-nu) / Gamma(nu) (sqrt(2 nu) t)^nu K_nu(sqrt(2 nu) t),
  used here through its closed forms at the half-integers nu = 1/2, 3/2, 5/2
  and its limit nu -> infinity, exp(-t^2 / 2);
* stationary core: C_core(x, x') = sigma0^2 M_nu(|(x - x') / ell|);
* parametric nonstationary core (Appendix B, Eq. PScov):
      C_core = sigma(x) sigma(x') (Sigma(x) Sigma(x'))^(d/4)
               / ((Sigma(x) + Sigma(x')) / 2)^(d/2)  M_nu(sqrt(Q)),
      Q = |(x - x') / ell|^2 / ((Sigma(x) + Sigma(x')) / 2),
  with log-linear fields
      log sigma(x) = log sigma0 + sum_m s_m(x) phi_sigma_m,
      log Sigma(x) = log Sigma0 + sum_m s_m(x) phi_Sigma_m.

Readings where the paper is silent or garbled:

* Eq. PScov prints Sigma(x') + Sigma(x') in the denominator of the prefactor;
  it is read as Sigma(x) + Sigma(x') (the form of Q beside it and of the
  cited Paciorek construction; the printed form is not symmetric).
* The Matern scaling sqrt(2 nu) t (the paper does not state one).
* The basis functions s_m, left generic in the paper ("polynomials, splines"),
  are Gaussian radial functions s_m(x) = exp(-|(x - c_m) / w|^2 / 2) with
  centres c_m and per-coordinate widths w.
* Distances inside Q are taken on (x_k - x'_k) / ell_k: ell = 1 is the printed,
  locally isotropic form; other ell let space-time coordinates carry their
  own units (Appendix B notes the anisotropic generalisation).
* sigma0 is the signal standard deviation of the stationary core too.

The core is strictly positive, so it never changes the sparsity pattern,
which stays that of C_sparse.
"""
from __future__ import annotations

import math

import numpy as np

NONE, MATERN, PACIOREK = 0, 1, 2


def matern(t, nu2: int):
    """M_nu(t) for 2 nu = nu2 in {1, 3, 5}, or nu = infinity for nu2 = 0."""
    t = np.asarray(t, np.float64)
    if nu2 == 0:
        return np.exp(-0.5 * t * t)
    if nu2 == 1:
        return np.exp(-t)
    if nu2 == 3:
        a = math.sqrt(3.0) * t
        return (1.0 + a) * np.exp(-a)
    if nu2 == 5:
        a = math.sqrt(5.0) * t
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError("nu2 must be 0, 1, 3 or 5")


# Sums below run over coordinates and basis functions in increasing order with
# elementwise operations, so a point's value does not depend on the shape of
# the array it is evaluated in.

def basis(x, core, m: int):
    """s_m(x) over the leading axes of x."""
    x = np.asarray(x, np.float64)
    d = x.shape[-1]
    c = np.asarray(core.centers, np.float64).reshape(-1, d)[m]
    w = np.asarray(core.width, np.float64)
    acc = 0.0
    for k in range(d):
        z = (x[..., k] - c[k]) / w[k]
        acc = acc + z * z
    return np.exp(-0.5 * acc)


def fields(x, core):
    """(sigma(x), Sigma(x)) over the leading axes of x."""
    x = np.asarray(x, np.float64)
    shape = x.shape[:-1]
    if core.kind != PACIOREK or int(core.n_basis) == 0:
        sig = np.full(shape, float(core.sigma0))
        Sig = np.full(shape, float(core.Sigma0) if core.kind == PACIOREK else 1.0)
        return sig, Sig
    ls = np.full(shape, math.log(core.sigma0))
    lS = np.full(shape, math.log(core.Sigma0))
    for m in range(int(core.n_basis)):
        s = basis(x, core, m)
        ls = ls + s * float(core.phi_sigma[m])
        lS = lS + s * float(core.phi_Sigma[m])
    return np.exp(ls), np.exp(lS)


def scaled_dist2(xp, xq, core):
    """|(x - x') / ell|^2 (broadcasting over the leading axes)."""
    d = xp.shape[-1]
    acc = 0.0
    for k in range(d):
        z = (xp[..., k] - xq[..., k]) / float(core.ell[k])
        acc = acc + z * z
    return acc


def value(xp, xq, core):
    """C_core(x_p, x_q) for broadcast arrays of points (last axis d)."""
    xp = np.asarray(xp, np.float64)
    xq = np.asarray(xq, np.float64)
    if core is None or core.kind == NONE:
        return np.ones(np.broadcast_shapes(xp.shape[:-1], xq.shape[:-1]))
    r2 = scaled_dist2(xp, xq, core)
    if core.kind == MATERN:
        return float(core.sigma0) ** 2 * matern(np.sqrt(r2), int(core.nu2))
    d = xp.shape[-1]
    sp, Sp = fields(xp, core)
    sq, Sq = fields(xq, core)
    avg = 0.5 * (Sp + Sq)
    pre = sp * sq * (Sp * Sq) ** (d / 4.0) / avg ** (d / 2.0)
    return pre * matern(np.sqrt(r2 / avg), int(core.nu2))
