"""Pins of the oracle's log-likelihood, SLQ log-det and kriging mean:
independent algorithms, closed forms on diagonal matrices, a library
density routine, the SplitMix64 published sequence, and the predictor's
identity at the training inputs (Sec. 3.1 Eq. Zmarg, Sec. 3.2, Sec. 3.3)."""
import math
import os

import numpy as np
import pytest
import scipy.stats

from oracle import kernel, likelihood, predict, slq
from workloads import Theta, uniform_problem, config1

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _y_from_z(K, z):
    return np.linalg.cholesky(K) @ z


def test_three_routes_agree_config1():
    p = config1()
    K, _ = kernel.dense(p.x, p.theta)
    y = _y_from_z(K, p.z_std)
    d = likelihood.dense_cholesky(K, y)
    ip, ci, vals, (M, F) = kernel.sparse(p.x, p.theta, return_features=True)
    A = kernel.to_scipy(ip, ci, vals, p.n)
    s = likelihood.sparse_lu(A, y)
    th0 = p.theta.copy()
    th0.a[:] = 0.0
    ipl, cil, vl = kernel.sparse(p.x, th0)
    Al = kernel.to_scipy(ipl, cil, vl, p.n)
    w = likelihood.split_woodbury(Al, F, y)
    for r in (s, w):
        assert abs(r["logdet"] - d["logdet"]) <= 1e-10 * abs(d["logdet"])
        assert abs(r["quad"] - d["quad"]) <= 1e-10 * abs(d["quad"])
        assert np.allclose(r["alpha"], d["alpha"], rtol=1e-8, atol=1e-10 * np.abs(d["alpha"]).max())
    # library density (scipy's multivariate normal, eigen-decomposition route)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(p.n), cov=K).logpdf(y)
    assert abs(d["loglik"] - ref) <= 1e-9 * abs(ref)


def test_diagonal_closed_form_no_bumps():
    # r0 below the minimum pair distance and all a = 0: K = (s0 + sigma^2) I.
    p = uniform_problem(500, 2, 3, r0=1e-6, n1=2, n2=2)
    p.theta.a[:] = 0.0
    p.theta.s0 = 1.7
    K, P = kernel.dense(p.x, p.theta)
    assert P.sum() == p.n
    y = p.z_std
    c = p.theta.s0 + p.theta.nugget
    expect = -0.5 * p.n * math.log(c) - 0.5 * float(y @ y) / c - 0.5 * p.n * math.log(2 * math.pi)
    assert abs(likelihood.dense_cholesky(K, y)["loglik"] - expect) <= 1e-12 * abs(expect)


def test_diagonal_closed_form_isolated_bumps():
    # n2 = 1 and each bump holds exactly one point: K diagonal with
    # k_p = s0 + sum_i f_i(p)^2 + sigma^2.
    x = np.array([[0.1, 0.1], [0.5, 0.5], [0.9, 0.2], [0.3, 0.8]])
    h = x[:3, None, :].copy()
    r = np.full((3, 1, 2), 0.05)
    a = np.array([[0.9], [0.6], [0.75]])
    th = Theta(1.0, np.array([1e-3, 1e-3]), h, r, a, np.ones((3, 1)), 0.01, 0)
    K, P = kernel.dense(x, th)
    assert np.count_nonzero(K - np.diag(np.diag(K))) == 0
    kp = np.array([1.0 + 0.81 + 0.01, 1.0 + 0.36 + 0.01, 1.0 + 0.5625 + 0.01, 1.01])
    assert np.allclose(np.diag(K), kp, rtol=1e-15)
    y = np.array([0.3, -1.2, 0.7, 2.0])
    expect = -0.5 * np.log(kp).sum() - 0.5 * (y * y / kp).sum() - 2 * math.log(2 * math.pi)
    assert abs(likelihood.dense_cholesky(K, y)["loglik"] - expect) < 1e-13


def test_splitmix64_published_sequence():
    with open(os.path.join(GOLD, "splitmix64_seed1234567.txt")) as f:
        ref = [int(l) for l in f if l.strip() and not l.startswith("#")]
    out = slq.splitmix64_sequence(1234567, 5)
    assert [int(v) for v in out] == ref


def test_rademacher_probe_is_counter_indexed_splitmix():
    # probe entry == sign of the SplitMix64 output at counter (l << 40 | i) + 1
    seq = slq.splitmix64_sequence(99, 64)
    z = slq.rademacher(99, 0, np.arange(64))
    assert np.array_equal(z, np.where((seq >> np.uint64(63)) != 0, -1.0, 1.0))
    big = slq.rademacher(7, 3, np.arange(200_000))
    assert abs(big.mean()) < 5 / math.sqrt(big.size)


def test_slq_exact_on_diagonal():
    # Hutchinson with Rademacher probes is exact on diagonal matrices and the
    # Jacobi-scaled matrix is I, so SLQ returns sum log d_p exactly.
    d = np.random.default_rng(1).uniform(0.5, 3.0, 400)
    r = slq.slq_logdet(np.diag(d), seed=5, n_probes=4, n_steps=10)
    assert abs(r["logdet"] - np.log(d).sum()) <= 1e-12 * abs(np.log(d).sum())
    assert np.all(r["steps"] == 1)


def test_slq_quadrature_exact_with_few_distinct_eigenvalues():
    # With at most k distinct eigenvalues, k-step Lanczos Gauss quadrature equals
    # z^T log(Ahat) z; compare per probe with a dense eigen-decomposition.
    rng = np.random.default_rng(2)
    n = 60
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([0.5, 1.0, 2.0, 4.0, 8.0], n // 5)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    r = slq.slq_logdet(A, seed=11, n_probes=6, n_steps=20)
    s = 1.0 / np.sqrt(np.diag(A))
    Ah = s[:, None] * A * s[None, :]
    w, V = np.linalg.eigh(Ah)
    logAh = (V * np.log(w)) @ V.T
    for l in range(6):
        z = slq.rademacher(11, l, np.arange(n))
        assert abs(r["gammas"][l] - z @ logAh @ z) <= 1e-8 * abs(z @ logAh @ z) + 1e-9


def test_slq_reorth_to_full_dimension_is_exact():
    # Lanczos with full re-orthogonalisation run to the full dimension n spans
    # the whole space, so its Gauss quadrature is z^T log(Ahat) z exactly; the
    # spectrum spreads over four decades with many distinct eigenvalues, where
    # the plain recurrence loses orthogonality long before n steps.
    rng = np.random.default_rng(12)
    n = 90
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.logspace(-2, 2, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    r = slq.slq_logdet(A, seed=3, n_probes=4, n_steps=n, reorth=True)
    s = 1.0 / np.sqrt(np.diag(A))
    Ah = s[:, None] * A * s[None, :]
    w, V = np.linalg.eigh(Ah)
    logAh = (V * np.log(w)) @ V.T
    for l in range(4):
        z = slq.rademacher(3, l, np.arange(n))
        ref = z @ logAh @ z
        assert abs(r["gammas"][l] - ref) <= 1e-9 * np.abs(z) @ np.abs(logAh) @ np.abs(z)


def test_slq_reorth_matches_plain_while_orthogonality_holds():
    # on a well-conditioned matrix and few steps the plain recurrence keeps its
    # vectors orthogonal to rounding, and both forms give the same quadrature
    p = config1()
    K, _ = kernel.dense(p.x, p.theta)
    a = slq.slq_logdet(K, seed=8, n_probes=3, n_steps=6)
    b = slq.slq_logdet(K, seed=8, n_probes=3, n_steps=6, reorth=True)
    assert np.allclose(a["gammas"], b["gammas"], rtol=1e-9, atol=0)


def test_slq_within_three_se_of_exact_config1():
    p = config1()
    K, _ = kernel.dense(p.x, p.theta)
    exact = likelihood.dense_cholesky(K, p.z_std)["logdet"]
    r = slq.slq_logdet(K, seed=2024, n_probes=30, n_steps=50)
    assert abs(r["logdet"] - exact) <= 3 * r["se"]
    assert abs(r["logdet"] - exact) <= 0.01 * abs(exact)


def test_predict_identity_at_training_inputs():
    p = uniform_problem(300, 2, 8, r0=0.12, n1=2, n2=2, bump_radius=0.25)
    K, _ = kernel.dense(p.x, p.theta)
    y = _y_from_z(K, p.z_std)
    alpha = likelihood.dense_cholesky(K, y)["alpha"]
    m = predict.mean(p.x, p.x, p.theta, alpha)
    assert np.allclose(m, y - p.theta.nugget * alpha, rtol=0, atol=1e-10 * np.abs(y).max())
    xs = np.random.default_rng(3).random((50, 2))
    assert np.allclose(predict.mean(xs, p.x, p.theta, alpha), predict.mean_rows(xs, p.x, p.theta, alpha),
                       rtol=1e-12, atol=1e-12)


def test_predict_closed_form_single_point():
    # one training point, no bumps, test point at u = 1/2: m = s0 f0(1/2) alpha
    th = Theta(1.5, np.array([1.0]), np.zeros((1, 1, 1)), np.ones((1, 1, 1)), np.zeros((1, 1)),
               np.ones((1, 1)), 0.2, 0)
    m = predict.mean(np.array([[0.5], [2.0]]), np.array([[0.0]]), th, np.array([3.0]))
    assert m[0] == 1.5 * 0.06103515625 * 3.0 and m[1] == 0.0


def test_variance_at_training_inputs_closed_form():
    # c = K e_p - sigma^2 e_p gives v_p = sigma^2 - sigma^4 (K^-1)_pp
    from workloads import uniform_problem
    p = uniform_problem(300, 2, 12, r0=0.1, n1=2, n2=2, bump_radius=0.3)
    K, _ = kernel.dense(p.x, p.theta)
    Kinv = np.linalg.inv(K)
    s2 = p.theta.nugget
    idx = np.arange(0, 300, 7)
    v = predict.variance(p.x[idx], p.x, p.theta)
    assert np.allclose(v, s2 - s2 * s2 * np.diag(Kinv)[idx], rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("with_core", [False, True])
def test_variance_is_the_joint_schur_complement(with_core):
    # v = 1 / (J^-1)_00 for the joint covariance J of (y(x*), z)
    from workloads import core_problem, uniform_problem
    p = core_problem(2, 2, n=250, seed=4) if with_core else uniform_problem(250, 2, 13, r0=0.1, n1=2, n2=2,
                                                                             bump_radius=0.3)
    K, _ = kernel.dense(p.x, p.theta)
    xs = np.random.default_rng(1).uniform(0, 1, (12, 2))
    v = predict.variance(xs, p.x, p.theta)
    prior = predict.prior_variance(xs, p.theta)
    rp, cols, vals = kernel.cross_entries(xs, p.x, p.theta)
    for s in range(xs.shape[0]):
        c = np.zeros(p.n)
        c[cols[rp[s]:rp[s + 1]]] = vals[rp[s]:rp[s + 1]]
        J = np.block([[np.array([[prior[s]]]), c[None, :]], [c[:, None], K]])
        assert math.isclose(v[s], 1.0 / np.linalg.inv(J)[0, 0], rel_tol=1e-8)
        assert 0.0 < v[s] <= prior[s]


def test_variance_far_from_data_is_the_prior():
    from workloads import uniform_problem
    p = uniform_problem(200, 2, 14, r0=0.1, n1=2, n2=2, bump_radius=0.2)
    xs = np.array([[5.0, 5.0], [-3.0, 0.5]])
    v = predict.variance(xs, p.x, p.theta)
    assert np.array_equal(v, predict.prior_variance(xs, p.theta))
    assert np.array_equal(v, np.full(2, p.theta.s0))


def test_variance_split_route_matches_dense():
    from workloads import uniform_problem
    p = uniform_problem(900, 2, 15, r0=0.07, n1=3, n2=2, bump_radius=0.25)
    xs = np.random.default_rng(2).uniform(-0.1, 1.1, (40, 2))
    assert np.allclose(predict.variance_split(xs, p.x, p.theta), predict.variance(xs, p.x, p.theta),
                       rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("with_tau2", [False, True])
def test_banded_split_equals_dense_cholesky(with_tau2):
    # the day-blocked route (block Cholesky of the local part, determinant
    # lemma, Woodbury) against LAPACK on the dense K of a small space-time set
    from workloads import config3, noise_variances
    p = config3(n_stations=50, n_days=40)
    th = p.theta.copy()
    if with_tau2:
        th.tau2 = noise_variances(p.n, 8, 0.0, 0.05)
    K, _ = kernel.dense(p.x, th)
    ref = likelihood.dense_cholesky(K, p.y)
    r = likelihood.banded_split(p.x, th, p.y)
    assert r["blocks"] == 40 and r["half_width"] == 2
    assert abs(r["logdet"] - ref["logdet"]) <= 1e-10 * abs(ref["logdet"])
    assert abs(r["quad"] - ref["quad"]) <= 1e-10 * abs(ref["quad"])
    # the input order does not matter (the points are grouped by day inside)
    perm = np.random.default_rng(1).permutation(p.n)
    th_p = th.copy()
    if with_tau2:
        th_p.tau2 = th.tau2[perm]
    r2 = likelihood.banded_split(p.x[perm], th_p, p.y[perm])
    assert abs(r2["logdet"] - r["logdet"]) <= 1e-11 * abs(r["logdet"])
    assert abs(r2["quad"] - r["quad"]) <= 1e-11 * abs(r["quad"])
