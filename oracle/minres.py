"""Preconditioned MINRES oracle (test infrastructure only).

The paper solves its linear systems with MINRES (Sec. 3.3: plain conjugate
gradients often failed for its kernels).  This is the method of Paige and
Saunders (1975) for symmetric, possibly indefinite, A with a symmetric
positive-definite preconditioner M:

* the preconditioned Lanczos process builds v_1 = M^{-1} r_0 / beta_1 and,
  step by step, alpha_k = v_k^T A v_k and beta_{k+1} from
  y = A v_k - alpha_k r_k / beta_k - beta_k r_{k-1} / beta_{k-1} (in the
  M-inner product; r_k holds the unpreconditioned vectors);
* the tridiagonal matrix of the process is reduced by Givens rotations
  (cs, sn), one per step, which gives the step length phi_k and the new
  residual-norm estimate phibar_k = |sn_k| phibar_{k-1};
* the solution is updated through search directions w_k = (v_k -
  eps_k w_{k-2} - delta_k w_{k-1}) / gamma_k, x_k = x_{k-1} + phi_k w_k.

MINRES minimises ||b - A x_k||_{M^{-1}} over x_0 + K_k(M^{-1} A, M^{-1} r_0), so
phibar_k is non-increasing.  Plain float64 NumPy, one operation at a time.
"""
from __future__ import annotations

import numpy as np


def minres(A, b, minv, x0=None, rtol: float = 1e-10, max_iter: int = 10_000):
    """Solve A x = b.  `A` is a dense array or a scipy sparse matrix; `minv(r)`
    applies M^{-1}.  Stops when the true residual ||b - A x||_2 <= rtol ||b||_2;
    the true residual is formed once the estimate phibar (an M^{-1}-norm) has
    fallen below 100 rtol ||b||_{M^{-1}}, since the two norms differ by a
    factor of at most sqrt(cond M).  Returns dict(x, iters, phibar (estimates per step),
    relres (true, final), converged)."""
    b = np.asarray(b, np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return dict(x=np.zeros(n), iters=0, phibar=[], relres=0.0, converged=True)
    bm = float(np.sqrt(b @ minv(b)))
    r1 = b - A @ x
    if float(np.linalg.norm(r1)) <= rtol * bnorm:
        return dict(x=x, iters=0, phibar=[], relres=float(np.linalg.norm(r1)) / bnorm, converged=True)
    y = minv(r1)
    beta1 = float(np.sqrt(r1 @ y))
    phibars = [beta1]
    if beta1 == 0.0:
        return dict(x=x, iters=0, phibar=phibars, relres=float(np.linalg.norm(r1)) / bnorm, converged=True)
    oldb, beta = 0.0, beta1
    dbar, epsln = 0.0, 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    w = np.zeros(n)
    w2 = np.zeros(n)
    r2 = r1.copy()
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        s = 1.0 / beta
        v = s * y
        y = A @ v
        if it >= 2:
            y = y - (beta / oldb) * r1
        alfa = float(v @ y)
        y = y - (alfa / beta) * r2
        r1 = r2
        r2 = y
        y = minv(r2)
        oldb = beta
        beta = float(np.sqrt(r2 @ y))
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = float(np.hypot(gbar, beta))
        gamma = max(gamma, np.finfo(float).tiny)
        cs = gbar / gamma
        sn = beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        phibars.append(phibar)
        w1 = w2
        w2 = w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        if phibar <= 100.0 * rtol * bm or beta == 0.0:
            rn = float(np.linalg.norm(b - A @ x))
            if rn <= rtol * bnorm or beta == 0.0:
                converged = rn <= rtol * bnorm
                break
    relres = float(np.linalg.norm(b - A @ x)) / bnorm
    return dict(x=x, iters=it, phibar=phibars, relres=relres, converged=converged or relres <= rtol)
