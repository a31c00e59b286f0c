"""Pins of the core-kernel oracle (``oracle.core``) against facts that do not
come from the oracle itself.

* Matern closed forms (nu = 1/2, 3/2, 5/2) against the general Bessel-function
  definition (scipy.special.kv), and the nu -> infinity limit against the
  Bessel form at a large nu.
* Eq. PScov (prefactor exponents d/4 and d/2, the average of Sigma in Q, and
  the reading Sigma(x) + Sigma(x') of the printed denominator) against a
  numerical convolution: with M = exp(-t^2/2), Paciorek's construction equals
  the normalised overlap integral of Gaussian kernels N(u; x, Sigma(x)/2 I)
  and N(u; x', Sigma(x')/2 I), here computed by trapezoidal quadrature.
* Special cases: constant fields reduce the nonstationary core to the
  stationary Matern; one basis function at its centre and far from it; the
  diagonal sigma(x)^2.
* Invariants: symmetry, positive definiteness (Schur product of two positive
  definite kernels), and the composition K = C_core o C_sparse + sigma^2 I
  with the nugget outside the product and the pattern unchanged.
"""
import math

import numpy as np
import pytest
from scipy import special

from oracle import core, kernel
from workloads import Core, core_problem, random_core, uniform_problem


def _matern_bessel(t, nu):
    t = np.asarray(t, np.float64)
    z = math.sqrt(2.0 * nu) * t
    out = np.ones_like(t)
    pos = z > 0
    out[pos] = 2.0 ** (1.0 - nu) / special.gamma(nu) * z[pos] ** nu * special.kv(nu, z[pos])
    return out


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_matern_closed_forms_vs_bessel(nu2):
    t = np.concatenate([[0.0, 1e-8], np.linspace(1e-3, 8.0, 400)])
    ref = _matern_bessel(t, nu2 / 2.0)
    got = core.matern(t, nu2)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-15)
    assert got[0] == 1.0


def test_matern_infinite_limit():
    # the Bessel form approaches exp(-t^2/2) with an error that halves when nu doubles
    t = np.linspace(0.05, 3.0, 60)
    errs = []
    for nu in (20.0, 40.0, 80.0):
        z = math.sqrt(2.0 * nu) * t
        # log form of the Bessel definition (kve keeps K_nu finite at these orders)
        logm = (1.0 - nu) * math.log(2.0) - special.gammaln(nu) + nu * np.log(z) + np.log(special.kve(nu, z)) - z
        errs.append(float(np.max(np.abs(core.matern(t, 0) - np.exp(logm)))))
    assert errs[2] < 3e-3
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2
    assert core.matern(0.0, 0) == 1.0


@pytest.mark.parametrize("nu2", [1, 3, 5])
def test_stationary_core_scales_each_coordinate(nu2):
    # one scale ell_k along coordinate k is distance 1: sigma0^2 M_nu(1) by the Bessel form
    c = Core(core.MATERN, nu2, 1.9, np.array([0.3, 2.0, 0.05]))
    x = np.array([0.1, 0.2, 0.3])
    ref = 1.9 ** 2 * _matern_bessel(np.array([1.0]), nu2 / 2.0)[0]
    for k in range(3):
        xq = x.copy()
        xq[k] += c.ell[k]
        assert math.isclose(float(core.value(x, xq, c)), ref, rel_tol=1e-12)
    # (ell_0, ell_1, 0) away: distance sqrt(2)
    xq = x + np.array([0.3, -2.0, 0.0])
    assert math.isclose(float(core.value(x, xq, c)), 1.9 ** 2 * _matern_bessel(np.array([math.sqrt(2.0)]), nu2 / 2.0)[0],
                        rel_tol=1e-12)


def _overlap_1d(mu1, v1, mu2, v2):
    """int N(u; mu1, v1) N(u; mu2, v2) du by the trapezoidal rule."""
    lo = min(mu1 - 12 * math.sqrt(v1), mu2 - 12 * math.sqrt(v2))
    hi = max(mu1 + 12 * math.sqrt(v1), mu2 + 12 * math.sqrt(v2))
    u = np.linspace(lo, hi, 20001)
    f = np.exp(-0.5 * (u - mu1) ** 2 / v1) / math.sqrt(2 * math.pi * v1) * \
        np.exp(-0.5 * (u - mu2) ** 2 / v2) / math.sqrt(2 * math.pi * v2)
    return float(np.trapezoid(f, u))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_paciorek_matches_gaussian_convolution(d):
    c = random_core(core.PACIOREK, d, seed=40 + d, nu2=0, ell=1.0, Sigma0=0.02, phi_sd=0.8)
    rng = np.random.default_rng(d)
    for _ in range(6):
        x = rng.uniform(0, 1, d)
        xq = x + rng.normal(0, 0.12, d)
        sp, Sp = core.fields(x, c)
        sq, Sq = core.fields(xq, c)

        def overlap(a, va, b, vb):
            return np.prod([_overlap_1d(a[k], va, b[k], vb) for k in range(d)])

        I = overlap(x, Sp / 2, xq, Sq / 2)
        norm = math.sqrt(overlap(x, Sp / 2, x, Sp / 2) * overlap(xq, Sq / 2, xq, Sq / 2))
        ref = float(sp) * float(sq) * I / norm
        got = float(core.value(x, xq, c))
        assert ref > 1e-6
        assert abs(got - ref) <= 1e-9 * ref, (got, ref)


@pytest.mark.parametrize("nu2", [0, 1, 3, 5])
def test_constant_fields_reduce_to_stationary(nu2):
    d = 2
    ns = random_core(core.PACIOREK, d, seed=3, nu2=nu2, Sigma0=2.5, ell=0.1)
    ns.phi_sigma = np.zeros_like(ns.phi_sigma)
    ns.phi_Sigma = np.zeros_like(ns.phi_Sigma)
    st = Core(core.MATERN, nu2, ns.sigma0, np.array(ns.ell) * math.sqrt(2.5))
    rng = np.random.default_rng(0)
    xp, xq = rng.uniform(0, 1, (500, d)), rng.uniform(0, 1, (500, d))
    assert np.allclose(core.value(xp, xq, ns), core.value(xp, xq, st), rtol=1e-13, atol=0)


def test_fields_at_and_away_from_a_basis_centre():
    c = Core(core.PACIOREK, 5, 1.7, np.ones(3), 0.3, centers=np.array([[0.25, 0.75]]),
             width=np.array([0.1, 0.2, 1.0]), phi_sigma=np.array([0.4]), phi_Sigma=np.array([-1.1]))
    s, S = core.fields(np.array([[0.25, 0.75], [50.0, -50.0], [0.35, 0.75]]), c)
    assert math.isclose(s[0], 1.7 * math.exp(0.4), rel_tol=1e-15)
    assert math.isclose(S[0], 0.3 * math.exp(-1.1), rel_tol=1e-15)
    assert s[1] == 1.7 and math.isclose(S[1], 0.3, rel_tol=1e-15)
    # one width away along the first coordinate: s_1 = exp(-1/2)
    assert math.isclose(s[2], 1.7 * math.exp(0.4 * math.exp(-0.5)), rel_tol=1e-14)


@pytest.mark.parametrize("kind", [core.MATERN, core.PACIOREK])
def test_core_diagonal_and_symmetry(kind):
    c = random_core(kind, 3, seed=9)
    rng = np.random.default_rng(1)
    xp, xq = rng.uniform(0, 1, (300, 3)), rng.uniform(0, 1, (300, 3))
    assert np.array_equal(core.value(xp, xq, c), core.value(xq, xp, c))
    s, _ = core.fields(xp, c)
    assert np.allclose(core.value(xp, xp, c), s * s, rtol=1e-15, atol=0)


@pytest.mark.parametrize("nu2", [0, 1, 3, 5])
def test_paciorek_positive_definite(nu2):
    c = random_core(core.PACIOREK, 2, seed=21, nu2=nu2, ell=0.15, phi_sd=1.0)
    x = np.random.default_rng(5).uniform(0, 1, (250, 2))
    C = core.value(x[:, None, :], x[None, :, :], c)
    w = np.linalg.eigvalsh(C)
    assert w.min() > -1e-10 * w.max()


@pytest.mark.parametrize("kind", [core.MATERN, core.PACIOREK])
def test_entries_are_core_times_sparse_plus_nugget(kind):
    p = core_problem(kind, 2, n=400, seed=2)
    th0 = p.theta.copy()
    th0.core = None
    K, P = kernel.dense(p.x, p.theta)
    K0, P0 = kernel.dense(p.x, th0, nugget=False)
    C = core.value(p.x[:, None, :], p.x[None, :, :], p.theta.core)
    assert np.array_equal(P, P0)
    ref = C * K0 + p.theta.nugget * np.eye(p.n)
    assert np.allclose(K, ref, rtol=1e-14, atol=1e-300)
    # diagonal: sigma(x)^2 (s0 + sum_i f_i^2) + nugget
    M, F = kernel.features(p.x, p.theta)
    s, _ = core.fields(p.x, p.theta.core)
    assert np.allclose(np.diag(K), s * s * (p.theta.s0 + (F * F).sum(1)) + p.theta.nugget, rtol=1e-14)
    np.linalg.cholesky(K)
    # the sparse builder agrees with the dense one
    ip, ci, vv = kernel.sparse(p.x, p.theta)
    Ks = kernel.to_scipy(ip, ci, vv, p.n).toarray()
    assert np.array_equal(Ks != 0, P & (K != 0)) and np.allclose(Ks, K, rtol=1e-15, atol=0)


def test_no_core_is_unchanged():
    p = uniform_problem(300, 2, 4)
    K_a, _ = kernel.dense(p.x, p.theta)
    p.theta.core = Core(core.NONE)
    K_b, _ = kernel.dense(p.x, p.theta)
    assert np.array_equal(K_a, K_b)
