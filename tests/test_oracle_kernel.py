"""Pins of the oracle's covariance against closed forms, invariants and
brute force (Sec. 2.1 Eq. bumpFcn / sumOfBumps / C_sparse / compSupp,
Proposition 1, Sec. 2.3 special case (1), Sec. 3.1 Eq. Zcov)."""
import os

import numpy as np
import pytest

from oracle import kernel
from workloads import Theta, uniform_problem, config1

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold():
    out = {}
    with open(os.path.join(GOLD, "closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def theta_1d(r0, centres=(), radii=(), amps=(), s0=1.0, nugget=0.0, b=1.0, variant=0):
    n2 = max(1, len(centres))
    h = np.zeros((1, n2, 1))
    r = np.ones((1, n2, 1))
    a = np.zeros((1, n2))
    for j, (c, rr, aa) in enumerate(zip(centres, radii, amps)):
        h[0, j, 0] = c
        r[0, j, 0] = rr
        a[0, j] = aa
    return Theta(s0, np.array([r0]), h, r, a, np.full((1, n2), b), nugget, variant)


def test_wendland_closed_forms():
    g = gold()
    assert kernel.wendland(np.array(0.5), 0) == g["wendland35_half"]
    assert kernel.wendland(np.array(0.5), 1) == g["wendland32_half"]
    assert kernel.wendland(np.array(0.0), 0) == g["wendland_zero"]
    assert kernel.wendland(np.array(1.0), 0) == 0.0


def test_bump_closed_forms():
    g = gold()
    # centre: g(h) = a (the exponent vanishes)
    assert kernel.bump_value(np.array(0.0), 0.7, 1.3) == 0.7
    assert abs(kernel.bump_value(np.array(0.25), 1.0, 1.0) - g["bump_half_radius"]) < 1e-16


def test_support_boundary_is_strict():
    # r0 = 0.5 so 1/r0 = 2 is exact: distance exactly r0 gives u0^2 = 1 -> outside;
    # one ulp-scale step inside gives u0^2 < 1 -> inside (Eq. compSupp uses strict <).
    th = theta_1d(0.5, nugget=0.1)
    x = np.array([[0.0], [0.5], [1.0 - 0.5 * (1 - 2.0 ** -30)]])
    K, P = kernel.dense(x, th)
    assert not P[0, 1] and K[0, 1] == 0.0
    assert P[1, 2] and K[1, 2] > 0.0
    # bump: a point exactly at distance r from the centre is outside the support
    th2 = theta_1d(0.01, centres=[0.0], radii=[0.5], amps=[1.0])
    M, F = kernel.features(np.array([[0.5], [0.25], [-0.5 + 2.0 ** -40]]), th2)
    assert M[:, 0].tolist() == [False, True, True]
    assert F[0, 0] == 0.0


def test_equispaced_1d_closed_form_matrix():
    # Sec. 2.3 special case (1) (no bumps): spacing r0/2 -> neighbours at u = 1/2,
    # second neighbours at u = 1 (outside).  K = s0 W + sigma^2 I exactly known.
    g = gold()
    s0, nug = 2.0, 0.25
    th = theta_1d(1.0, s0=s0, nugget=nug)
    x = np.arange(5, dtype=float)[:, None] * 0.5
    K, P = kernel.dense(x, th)
    expect = np.diag(np.full(5, s0 + nug))
    for i in range(4):
        expect[i, i + 1] = expect[i + 1, i] = s0 * g["wendland35_half"]
    assert np.array_equal(K, expect)
    assert P.sum() == 5 + 8


def test_bump_pair_closed_form():
    # two points at r/2 on either side of one bump centre, far apart relative to r0:
    # K_12 = f(x1) f(x2) = (a e^{-b/3})^2, and only the bump term links them.
    g = gold()
    th = theta_1d(1e-3, centres=[0.3], radii=[0.2], amps=[1.0])
    x = np.array([[0.2], [0.4], [0.9]])
    K, P = kernel.dense(x, th)
    assert P[0, 1] and not P[0, 2] and not P[1, 2]
    assert abs(K[0, 1] - g["bump_half_radius"] ** 2) < 1e-15
    assert abs(K[0, 0] - (1.0 + K[0, 1])) < 1e-15   # s0 f0(0) + f(x)^2


def test_bumps_link_distant_points_fig_example():
    # The 1-D illustration (Sec. 2.1): N = 100 equispaced points on [0,1],
    # n1 = 2, n2 = 3, r0 = 0.15.  Points sharing a group are linked regardless
    # of distance; points in different groups only locally.
    h = np.array([[[0.17], [0.7], [0.45]], [[0.17], [0.9], [0.3]]])
    r = np.full((2, 3, 1), 0.06)
    a = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0]])
    th = Theta(1.0, np.array([0.15]), h, r, a, np.ones((2, 3)), 0.0, 0)
    x = np.linspace(0, 1, 100)[:, None]
    K, P = kernel.dense(x, th)
    i17, i70, i90 = 17, 69, 89   # x = 0.1717, 0.697, 0.899
    assert P[i17, i70] and K[i17, i70] > 0      # share group 1
    assert P[i17, i90] and K[i17, i90] > 0      # share group 2
    assert not P[i70, i90] and K[i70, i90] == 0  # no shared group, far apart


def test_bump_term_has_rank_n1():
    # Proposition 1's proof: the bump term is sum_i Phi_i Phi_i^T, rank <= n1.
    p = uniform_problem(300, 2, 11, r0=1e-4, n1=3, n2=4, bump_radius=0.3)
    K, P = kernel.dense(p.x, p.theta)
    B = K - np.diag(np.diag(K))            # off-diagonal: bump term only (r0 tiny)
    M, F = kernel.features(p.x, p.theta)
    B = B + np.diag((F * F).sum(1))        # restore its diagonal
    s = np.linalg.svd(B, compute_uv=False)
    assert (s > 1e-10 * s[0]).sum() <= 3


def test_brute_force_equals_kdtree_pattern():
    for seed, d in [(21, 1), (22, 2), (23, 3)]:
        p = uniform_problem(450, d, seed, r0=0.12, n1=3, n2=2, bump_radius=0.25)
        K, P = kernel.dense(p.x, p.theta)
        ip, ci, vals = kernel.sparse(p.x, p.theta)
        rows = np.repeat(np.arange(p.n), np.diff(ip))
        Ps = np.zeros_like(P)
        Ps[rows, ci] = True
        assert np.array_equal(P, Ps)
        assert np.array_equal(K[rows, ci], vals)   # same formula, same op order


def test_symmetry_bitwise_and_exact_zeros():
    p = config1()
    K, P = kernel.dense(p.x, p.theta)
    assert np.array_equal(K, K.T)
    assert np.array_equal(P, P.T)
    M, F = kernel.features(p.x, p.theta)
    u2 = kernel.local_sq(p.x[:, None, :], p.x[None, :, :], p.theta)
    share = (M[:, None, :] & M[None, :, :]).any(-1)
    outside = (u2 >= 1.0) & ~share
    np.fill_diagonal(outside, False)
    assert not P[outside].any() and np.all(K[outside] == 0.0)
    assert P[u2 < 1.0].all()


def test_positive_definite_prop1():
    # C_sparse is strictly PD, so K = C_sparse + sigma^2 I has lambda_min >= sigma^2.
    p = config1()
    K, _ = kernel.dense(p.x, p.theta)
    lam = np.linalg.eigvalsh(K)
    assert lam[0] >= p.theta.nugget * (1 - 1e-10)
    Kt = K - p.theta.nugget * np.eye(p.n)
    assert np.linalg.eigvalsh(Kt)[0] > 0


def test_textbook_variant_positive_definite():
    p = uniform_problem(400, 3, 5, r0=0.3, n1=1, n2=1, bump_radius=0.1, nugget=0.0, wendland_variant=1)
    p.theta.a[:] = 0.0
    K, _ = kernel.dense(p.x, p.theta)
    assert np.linalg.eigvalsh(K)[0] > 0


def test_permutation_invariance():
    p = uniform_problem(300, 2, 31, r0=0.1, n1=2, n2=3, bump_radius=0.2)
    K, P = kernel.dense(p.x, p.theta)
    perm = np.random.default_rng(0).permutation(p.n)
    K2, P2 = kernel.dense(p.x[perm], p.theta)
    assert np.array_equal(P2, P[np.ix_(perm, perm)])
    assert np.array_equal(K2, K[np.ix_(perm, perm)])


def test_row_equals_dense_row():
    p = uniform_problem(400, 3, 41, r0=0.15, n1=2, n2=2, bump_radius=0.3)
    K, P = kernel.dense(p.x, p.theta)
    for r in [0, 17, 399]:
        c, v = kernel.row(p.x, p.theta, r)
        assert np.array_equal(c, np.nonzero(P[r])[0])
        assert np.array_equal(v, K[r, c])


def test_infinite_bump_radius_drops_coordinate():
    # r = +inf on the time axis: membership decided by space only (Sec. 5.2 spatial bumps)
    h = np.array([[[0.5, 0.5, 100.0]]])
    r = np.array([[[0.1, 0.1, np.inf]]])
    th = Theta(1.0, np.array([0.01, 0.01, 0.5]), h, r, np.ones((1, 1)), np.ones((1, 1)), 0.0, 0)
    x = np.array([[0.5, 0.5, 0.0], [0.55, 0.5, 365.0], [0.7, 0.5, 100.0]])
    M, F = kernel.features(x, th)
    assert M[:, 0].tolist() == [True, True, False]
    assert F[0, 0] == 1.0
