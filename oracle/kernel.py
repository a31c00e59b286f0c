"""Oracle: the covariance C_z = C_core C_sparse + sigma^2 I of the paper, in float64.

Test infrastructure only (see the package docstring): never imported by the
HIP product path.

Definitions followed (Sec. 2.1 and 3.1):

* bump function (Eq. bumpFcn): g(x) = a exp{b [1 - (1 - |x-h|^2/r^2)^-1]}
  when |x - h| < r, else 0;
* sum of bumps (Eq. sumOfBumps): f_i(x) = sum_j g_ij(x), i = 1..n1;
* Wendland part (Eq. compSupp): f0 = (1-u)^8 (35 u^3 + 25 u^2 + 8 u + 1)
  for u = |x - x'| / r0 < 1, else 0;
* sparse kernel (Eq. C_sparse): C_sparse = s0 f0 + sum_i f_i(x) f_i(x');
* times the core kernel (Eq. sparseCov; ``oracle.core``, C_core = 1 unless
  the hyper-parameters carry one) plus the error variances of Eq. Zcov on the
  index diagonal, Delta = diag[tau^2(x_1), ..., tau^2(x_N)], here a constant
  nugget sigma^2 plus optional per-point values tau2[p] (``th.tau2``, original
  point order):
  K_pq = C_core(x_p, x_q) C_sparse(x_p, x_q) + (sigma^2 + tau2[p]) [p = q],
  the two diagonal terms added in that order.

Readings where the paper is silent or ambiguous:

* Support decisions ("|x - h| < r", "|x - x'| < r0") are taken on the
  pinned float64 expression  u^2 = sum_k ((x_k - x'_k) * (1/r_k))^2,
  each operation rounded on its own, summed over k in increasing order, no
  fused multiply-add, then compared with ``< 1.0``.  The same expression,
  with x' = h, decides bump membership.  An entry whose support test passes
  belongs to the pattern even if its value underflows to zero.
* Coordinate-specific radii (Appendix E, the anisotropic Wendland with
  per-coordinate truncation) use the same scaled norm inside the same
  polynomial; a bump radius of +inf drops that coordinate from the test.
* The Wendland cubic coefficient is 35 as printed (variant 0); variant 1
  uses the textbook phi_{3,3} coefficient 32.
* The bump group term only exists where both points lie in the support of
  some bump of group i:  [M_i(p) and M_i(q)] f_i(p) f_i(q).  Because
  f_i = 0 wherever M_i is false this equals f_i(p) f_i(q), the rank-one
  term of Proposition 1's proof.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import core


def _theta_arrays(th):
    d = int(np.asarray(th.r0).shape[0])
    return (float(th.s0), np.asarray(th.r0, np.float64), np.asarray(th.h, np.float64).reshape(-1, d),
            np.asarray(th.r, np.float64).reshape(-1, d), np.asarray(th.a, np.float64).reshape(-1),
            np.asarray(th.b, np.float64).reshape(-1), float(th.nugget), int(th.wendland_variant),
            int(np.asarray(th.a).shape[0]), int(np.asarray(th.a).shape[1]))


def scaled_sq(diffs, inv_r):
    """Pinned support expression: sum_k (diff_k * inv_r_k)^2, left to right.

    ``diffs`` is a sequence of d arrays (the coordinate differences).  NumPy
    rounds every elementwise multiply and add on its own (no contraction), so
    this is exactly the float64 expression the support test is defined on.
    """
    acc = None
    for k, dk in enumerate(diffs):
        t = dk * inv_r[k]
        t2 = t * t
        acc = t2 if acc is None else acc + t2
    return acc


def wendland(u, variant: int = 0):
    """f0 as a function of u = |x - x'| / r0 (Eq. compSupp), u < 1 assumed."""
    c3 = 35.0 if variant == 0 else 32.0
    return (1.0 - u) ** 8 * (c3 * u ** 3 + 25.0 * u ** 2 + 8.0 * u + 1.0)


def bump_value(ub2, a, b):
    """g = a exp{b [1 - 1/(1 - |x-h|^2/r^2)]} given ub2 = |x-h|^2/r^2 < 1 (Eq. bumpFcn)."""
    return a * np.exp(b * (1.0 - 1.0 / (1.0 - ub2)))


def features(x, th):
    """Bump-group membership M (n, n1) bool and f_i values F (n, n1) float64.

    M_i(p) is true when p lies strictly inside the support of at least one
    bump j of group i with a_ij > 0; F[p, i] = sum_j g_ij(x_p) summed in j
    order (Eq. sumOfBumps).
    """
    x = np.asarray(x, np.float64)
    n, d = x.shape
    s0, r0, h, r, a, b, nug, var, n1, n2 = _theta_arrays(th)
    M = np.zeros((n, n1), bool)
    F = np.zeros((n, n1))
    for i in range(n1):
        for j in range(n2):
            bj = i * n2 + j
            inv = 1.0 / r[bj]
            ub2 = scaled_sq([x[:, k] - h[bj, k] for k in range(d)], inv)
            inside = (a[bj] > 0.0) & (ub2 < 1.0)
            g = np.zeros(n)
            g[inside] = bump_value(ub2[inside], a[bj], b[bj])
            F[:, i] = F[:, i] + g
            M[:, i] |= inside
    return M, F


def local_sq(xp, xq, th):
    """Pinned u0^2 between point sets (broadcasting over the leading axes)."""
    r0 = np.asarray(th.r0, np.float64)
    inv = 1.0 / r0
    d = r0.shape[0]
    return scaled_sq([xp[..., k] - xq[..., k] for k in range(d)], inv)


def tau2_of(th, n=None):
    """The per-point error variances th.tau2 (float64, original order) or None;
    checks length n, finiteness and tau2 >= 0."""
    t = getattr(th, "tau2", None)
    if t is None:
        return None
    t = np.asarray(t, np.float64).reshape(-1)
    if n is not None and t.shape[0] != n:
        raise ValueError("tau2 must hold one value per point")
    if not (np.all(np.isfinite(t)) and np.all(t >= 0.0)):
        raise ValueError("tau2 must be finite and >= 0")
    return t


def entries(xp, xq, Mp, Mq, Fp, Fq, same, th, tau=None):
    """K_pq for aligned arrays of pairs (Eq. sparseCov, Eq. C_sparse, Eq. Zcov).

    K = C_core(p, q) (s0 f0(u) [u0^2 < 1] + sum_i [M_i(p) and M_i(q)] f_i(p) f_i(q))
        + sigma^2 [p = q] + tau [p = q],
    the group sum taken in increasing i; C_core = 1 unless th.core is set
    (``oracle.core``); ``tau`` holds tau2 of each pair's row point (aligned
    with the pairs), or None for no per-point term.
    """
    u2 = local_sq(xp, xq, th)
    L = u2 < 1.0
    val = np.zeros(u2.shape)
    val[L] = float(th.s0) * wendland(np.sqrt(u2[L]), int(th.wendland_variant))
    n1 = Mp.shape[-1]
    for i in range(n1):
        both = Mp[..., i] & Mq[..., i]
        val = val + np.where(both, Fp[..., i] * Fq[..., i], 0.0)
    cr = getattr(th, "core", None)
    if cr is not None and cr.kind != core.NONE:
        val = core.value(xp, xq, cr) * val
    val = val + np.where(same, float(th.nugget), 0.0)
    if tau is not None:
        val = val + np.where(same, tau, 0.0)
    return val


def pattern_pred(xp, xq, Mp, Mq, same, th):
    """Pattern membership: [u0^2 < 1] or (M(p) and M(q) share a group) or p = q."""
    u2 = local_sq(xp, xq, th)
    share = (Mp & Mq).any(axis=-1)
    return (u2 < 1.0) | share | same


def dense(x, th, nugget: bool = True, block: int = 512):
    """Brute force over all pairs: dense K (n, n) and its pattern (n, n) bool."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    M, F = features(x, th)
    t2 = tau2_of(th, n) if nugget else None
    K = np.zeros((n, n))
    P = np.zeros((n, n), bool)
    idx = np.arange(n)
    for s in range(0, n, block):
        e = min(n, s + block)
        xp = x[s:e, None, :]
        xq = x[None, :, :]
        same = idx[s:e, None] == idx[None, :]
        if not nugget:
            same_n = np.zeros_like(same)
        else:
            same_n = same
        P[s:e] = pattern_pred(xp, xq, M[s:e, None, :], M[None, :, :], same, th)
        v = entries(xp, xq, M[s:e, None, :], M[None, :, :], F[s:e, None, :], F[None, :, :], same_n, th,
                    None if t2 is None else t2[s:e, None])
        K[s:e] = np.where(P[s:e], v, 0.0)
    return K, P


def row(x, th, p: int, M=None, F=None):
    """Row p of K by testing every point: (ascending columns int64, values)."""
    x = np.asarray(x, np.float64)
    if M is None:
        M, F = features(x, th)
    n = x.shape[0]
    same = np.arange(n) == p
    P = pattern_pred(x[p][None, :], x, M[p][None, :], M, same, th)
    cols = np.nonzero(P)[0]
    t2 = tau2_of(th, n)
    vals = entries(x[p][None, :], x[cols], M[p][None, :], M[cols], F[p][None, :], F[cols], cols == p, th,
                   None if t2 is None else t2[p])
    return cols, vals


def sparse(x, th, return_features: bool = False):
    """CSR of K in original order with ascending columns (O4 route).

    Local candidates come from a KD-tree over the coordinates scaled by
    1/r0 with radius 1 + 1e-9 (a superset of the support), re-filtered by
    the pinned predicate; the bump part adds every pair of each group's
    member set S_i x S_i.  Entries whose value underflows stay stored.
    Returns (indptr int64, indices int64, data float64[, (M, F)]).
    """
    x = np.asarray(x, np.float64)
    n, d = x.shape
    r0 = np.asarray(th.r0, np.float64)
    M, F = features(x, th)
    tree = cKDTree(x * (1.0 / r0))
    pairs = tree.query_pairs(1.0 + 1e-9, output_type="ndarray")
    if pairs.size:
        u2 = local_sq(x[pairs[:, 0]], x[pairs[:, 1]], th)
        pairs = pairs[u2 < 1.0]
    keys = [np.arange(n, dtype=np.int64) * (n + 1)]  # diagonal
    if pairs.size:
        pi = pairs[:, 0].astype(np.int64)
        pj = pairs[:, 1].astype(np.int64)
        keys.append(pi * n + pj)
        keys.append(pj * n + pi)
    for i in range(M.shape[1]):
        S = np.nonzero(M[:, i])[0].astype(np.int64)
        if S.size:
            keys.append((S[:, None] * n + S[None, :]).reshape(-1))
    keys = np.unique(np.concatenate(keys))
    rows = keys // n
    cols = keys % n
    del keys
    vals = np.empty(rows.shape[0])
    t2 = tau2_of(th, n)
    chunk = 1 << 22
    for s in range(0, rows.shape[0], chunk):
        e = min(rows.shape[0], s + chunk)
        rp, cq = rows[s:e], cols[s:e]
        vals[s:e] = entries(x[rp], x[cq], M[rp], M[cq], F[rp], F[cq], rp == cq, th,
                            None if t2 is None else t2[rp])
    indptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    if return_features:
        return indptr, cols, vals, (M, F)
    return indptr, cols, vals


def to_scipy(indptr, indices, data, n):
    import scipy.sparse as sp
    A = sp.csr_matrix((data, indices.astype(np.int64), indptr), shape=(n, n))
    return A


def cross_entries(xs, x, th, Ms=None, Fs=None, M=None, F=None):
    """Cross-covariance rows C_y(x*_s, x_q) (no nugget) for test points xs,
    as (row_ptr, cols, vals) with ascending columns, by brute force."""
    xs = np.asarray(xs, np.float64)
    if M is None:
        M, F = features(x, th)
    if Ms is None:
        Ms, Fs = features(xs, th)
    rp = [0]
    cs, vs = [], []
    for s in range(xs.shape[0]):
        same = np.zeros(x.shape[0], bool)
        P = pattern_pred(xs[s][None, :], x, Ms[s][None, :], M, same, th)
        cols = np.nonzero(P)[0]
        vals = entries(xs[s][None, :], x[cols], Ms[s][None, :], M[cols], Fs[s][None, :], F[cols],
                       np.zeros(cols.shape[0], bool), th)
        cs.append(cols)
        vs.append(vals)
        rp.append(rp[-1] + cols.shape[0])
    return np.array(rp, np.int64), np.concatenate(cs) if cs else np.zeros(0, np.int64), \
        np.concatenate(vs) if vs else np.zeros(0)
