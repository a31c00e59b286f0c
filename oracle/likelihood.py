"""Oracle: exact Gaussian log-likelihood of the residual y (float64).

Test infrastructure only.

Definition (Sec. 3.1 Eq. Zmarg with the residual y = z - W beta; Sec. 3.3):

    l(theta) = -1/2 log det K - 1/2 y^T K^{-1} y - (n/2) log(2 pi)

The paper writes the log-likelihood up to an additive constant; the constant
-(n/2) log 2 pi is kept here and log det and the quadratic form are also
returned on their own so that a relative error cannot hide in the constant.

Three independent routes (Sec. 3.3 names LU/Cholesky for smaller problems):

* ``dense_cholesky``   - LAPACK Cholesky of the dense K;
* ``sparse_lu``        - SuperLU with symmetric mode and diagonal pivots;
* ``split_woodbury``   - K = A + F F^T with A = s0 W + sigma^2 I (the local,
                         bump-free part) and F the n x n1 matrix of f_i(x_p)
                         (the rank-n1 bump term of Proposition 1's proof);
                         log det by the matrix determinant lemma and the
                         quadratic form by the Woodbury identity;
* ``banded_split``     - the same split when A is block-banded along an
                         integer coordinate (the days of a space-time data
                         set): a dense block Cholesky of A over the day
                         blocks, forward-substituting y and F as it goes, so
                         n ~ 10^6 fits in memory (no factor is kept).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

LOG2PI = math.log(2.0 * math.pi)


def assemble(logdet: float, quad: float, n: int) -> float:
    return -0.5 * logdet - 0.5 * quad - 0.5 * n * LOG2PI


def dense_cholesky(K, y):
    """logdet = 2 sum log L_pp, quad = |L^{-1} y|^2, alpha = K^{-1} y."""
    K = np.asarray(K, np.float64)
    y = np.asarray(y, np.float64)
    L = np.linalg.cholesky(K)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    w = sla.solve_triangular(L, y, lower=True)
    quad = float(w @ w)
    alpha = sla.cho_solve((L, True), y)
    return dict(logdet=logdet, quad=quad, loglik=assemble(logdet, quad, y.shape[0]), alpha=alpha)


class SparseLU:
    """SuperLU factorisation K = P^T L U P with symmetric ordering and
    diagonal pivots, so det K = prod diag U (all positive for SPD K)."""

    def __init__(self, A):
        A = sp.csc_matrix(A)
        self.lu = spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))
        if not np.array_equal(self.lu.perm_r, self.lu.perm_c):
            raise RuntimeError("SuperLU left the symmetric ordering")
        du = self.lu.U.diagonal()
        if not np.all(du > 0):
            raise np.linalg.LinAlgError("non-positive pivot: matrix is not positive definite")
        self.logdet = float(np.sum(np.log(du)))

    def solve(self, b):
        return self.lu.solve(np.asarray(b, np.float64))


def sparse_lu(A, y):
    f = SparseLU(A)
    alpha = f.solve(y)
    quad = float(np.asarray(y, np.float64) @ alpha)
    return dict(logdet=f.logdet, quad=quad, loglik=assemble(f.logdet, quad, len(y)), alpha=alpha)


def split_woodbury(A, F, y, dense_A: bool = False):
    """K = A + F F^T:  log det K = log det A + log det(I + F^T A^{-1} F);
    y^T K^{-1} y = y^T A^{-1} y - c^T S^{-1} c with S = I + F^T A^{-1} F and
    c = F^T A^{-1} y;  alpha = A^{-1} y - A^{-1} F S^{-1} c."""
    y = np.asarray(y, np.float64)
    F = np.asarray(F, np.float64)
    if dense_A:
        A = np.asarray(A.todense() if sp.issparse(A) else A, np.float64)
        L = np.linalg.cholesky(A)
        logdetA = 2.0 * float(np.sum(np.log(np.diag(L))))
        solve = lambda b: sla.cho_solve((L, True), b)  # noqa: E731
    else:
        f = SparseLU(A)
        logdetA = f.logdet
        solve = f.solve
    Ay = solve(y)
    AF = np.column_stack([solve(F[:, i]) for i in range(F.shape[1])]) if F.shape[1] else np.zeros((len(y), 0))
    S = np.eye(F.shape[1]) + F.T @ AF
    Ls = np.linalg.cholesky(S) if F.shape[1] else np.zeros((0, 0))
    logdetS = 2.0 * float(np.sum(np.log(np.diag(Ls)))) if F.shape[1] else 0.0
    c = F.T @ Ay
    Sc = sla.cho_solve((Ls, True), c) if F.shape[1] else c
    quad = float(y @ Ay - c @ Sc)
    alpha = Ay - AF @ Sc
    logdet = logdetA + logdetS
    return dict(logdet=logdet, quad=quad, loglik=assemble(logdet, quad, len(y)), alpha=alpha)


def split_solve(A, F, B):
    """K^{-1} B for K = A + F F^T (A sparse SPD, F n x n1, B n x k) by the
    Woodbury identity: A^{-1} B - A^{-1} F S^{-1} F^T A^{-1} B with
    S = I + F^T A^{-1} F; one SuperLU factorisation of A."""
    F = np.asarray(F, np.float64)
    B = np.asarray(B, np.float64)
    f = SparseLU(A)
    AB = f.solve(B)
    if F.shape[1] == 0:
        return AB
    AF = f.solve(F)
    S = np.eye(F.shape[1]) + F.T @ AF
    return AB - AF @ np.linalg.solve(S, F.T @ AB)


def banded_split(x, th, y, axis: int = -1):
    """Exact log det K and y^T K^{-1} y for K = A + F F^T (the split of
    ``split_woodbury``) when coordinate ``axis`` of the points takes integer
    values (days) and A couples only points whose values differ by at most w.

    The points are grouped by that coordinate (blocks B_0 < B_1 < ...), so A
    in this order is block-banded with half-width w blocks, w read off A's
    pattern.  Block row k of the Cholesky factor L of A follows from the w
    block rows before it:
        L_kj = (A_kj - sum_{i<j} L_ki L_ji^T) L_jj^{-T}   (k - w <= j < k),
        L_kk = chol(A_kk - sum_{j<k} L_kj L_kj^T),
    and y, F are forward-substituted at the same time (z = L^{-1} y,
    G = L^{-1} F), so only the last w block rows of L are held.  Then
        log det K = 2 sum log diag L + log det(I + G^T G),
        y^T K^{-1} y = z^T z - c^T (I + G^T G)^{-1} c,   c = G^T z
    (determinant lemma and Woodbury, as in ``split_woodbury``).  Needs
    C_core = 1 (the group term is then the rank-n1 product F F^T).
    Returns logdet, quad, loglik and the block count and half-width."""
    from . import kernel
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = x.shape[0]
    if getattr(th, "core", None) is not None and th.core.kind != 0:
        raise ValueError("the split K = A + F F^T needs a unit core kernel")
    t = x[:, axis]
    if not np.array_equal(t, np.round(t)):
        raise ValueError("the blocking coordinate must take integer values")
    th_local = th.copy()
    th_local.a = np.zeros_like(np.asarray(th_local.a, np.float64))
    A = kernel.to_scipy(*kernel.sparse(x, th_local), n)
    M, F = kernel.features(x, th)
    F = np.where(M, F, 0.0)
    order = np.argsort(t, kind="stable")
    A = A[order][:, order].tocsr()
    y, F, t = y[order], F[order], t[order]
    starts = np.concatenate([[0], np.nonzero(np.diff(t))[0] + 1, [n]])
    nb = starts.size - 1
    blk = np.repeat(np.arange(nb), np.diff(starts))
    Ac = A.tocoo()
    w = int(np.max(np.abs(blk[Ac.row] - blk[Ac.col]))) if Ac.nnz else 0
    del Ac

    def block(k, j):
        return A[starts[k]:starts[k + 1], starts[j]:starts[j + 1]].toarray()

    L = {}        # (k, j) -> block of L, for the last w + 1 block rows
    zs, Gs = {}, {}
    logdetA = 0.0
    z_all = np.empty(n)
    G_all = np.empty((n, F.shape[1]))
    for k in range(nb):
        lo = max(0, k - w)
        for j in range(lo, k):
            B = block(k, j)
            for i in range(max(lo, j - w), j):
                B -= L[(k, i)] @ L[(j, i)].T
            L[(k, j)] = sla.solve_triangular(L[(j, j)], B.T, lower=True).T
        D = block(k, k)
        rz = y[starts[k]:starts[k + 1]].copy()
        rG = F[starts[k]:starts[k + 1]].copy()
        for j in range(lo, k):
            D -= L[(k, j)] @ L[(k, j)].T
            rz -= L[(k, j)] @ zs[j]
            rG -= L[(k, j)] @ Gs[j]
        Lkk = np.linalg.cholesky(D)
        L[(k, k)] = Lkk
        logdetA += 2.0 * float(np.sum(np.log(np.diag(Lkk))))
        zs[k] = sla.solve_triangular(Lkk, rz, lower=True)
        Gs[k] = sla.solve_triangular(Lkk, rG, lower=True)
        z_all[starts[k]:starts[k + 1]] = zs[k]
        G_all[starts[k]:starts[k + 1]] = Gs[k]
        # keep only what the next block rows need
        for key in [key for key in L if key[0] <= k - w or key[1] < k - w]:
            del L[key]
        for d in (zs, Gs):
            for key in [key for key in d if key < k - w + 1]:
                del d[key]
    m = F.shape[1]
    S = np.eye(m) + G_all.T @ G_all
    Ls = np.linalg.cholesky(S) if m else np.zeros((0, 0))
    logdetS = 2.0 * float(np.sum(np.log(np.diag(Ls)))) if m else 0.0
    c = G_all.T @ z_all
    quad = float(z_all @ z_all - (c @ sla.cho_solve((Ls, True), c) if m else 0.0))
    logdet = logdetA + logdetS
    return dict(logdet=logdet, quad=quad, loglik=assemble(logdet, quad, n), logdet_A=logdetA,
                blocks=nb, half_width=w)
