"""Seeded synthetic inputs for the sparse-covariance GP hot path.

This module only draws random numbers and lays them out: points, kernel
hyper-parameters, observations, request streams.  It holds none of the
method's arithmetic (no kernel, predicate, solve or log-det), so both the
HIP path and the CPU oracle may take their inputs from it.

Every generator uses ``numpy.random.default_rng(seed)`` with a fixed draw
order, so a (config, seed) pair always yields bitwise-identical arrays.

Where a workload needs a quantity that only the method can produce (the
Wendland radius of the 100k-point mixture, chosen so that rows hold about
50 nonzeros), the value is read from ``calibration.json``, which the
committed script ``workloads/calibrate.py`` writes by calling the oracle.

The workloads stand in for the paper's data sets (Sec. 3.3 runtime study:
N = 50k-200k scattered 2-D points; Sec. 5.2: about 1.04M daily space-time
observations on a station grid, d = 3, with bump functions); the real
station records are not used.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


@dataclasses.dataclass
class Core:
    """Core kernel C_core of C_y = C_core x C_sparse (Eq. sparseCov).

    kind: 0 none (C_core = 1), 1 stationary Matern sigma0^2 M_nu(|(x-x')/ell|),
    2 parametric nonstationary (Eq. PScov) with log sigma(x) = log sigma0 +
    sum_m s_m(x) phi_sigma[m], log Sigma(x) = log Sigma0 + sum_m s_m(x)
    phi_Sigma[m] and Gaussian radial basis functions s_m with centres
    ``centers`` (M, d) and per-coordinate widths ``width`` (d,).
    nu2 = 2 nu in {1, 3, 5}, or 0 for nu = infinity.
    """

    kind: int
    nu2: int = 5
    sigma0: float = 1.0
    ell: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(3))
    Sigma0: float = 1.0
    centers: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 1)))
    width: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(3))
    phi_sigma: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    phi_Sigma: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))

    @property
    def n_basis(self) -> int:
        return int(np.asarray(self.phi_sigma).shape[0])

    def copy(self) -> "Core":
        return Core(int(self.kind), int(self.nu2), float(self.sigma0), np.array(self.ell, np.float64),
                    float(self.Sigma0), np.array(self.centers, np.float64), np.array(self.width, np.float64),
                    np.array(self.phi_sigma, np.float64), np.array(self.phi_Sigma, np.float64))


@dataclasses.dataclass
class Theta:
    """Hyper-parameters of C_sparse plus the nugget (Sec. 2.1, Eq. C_sparse).

    Shapes: r0 (d,), h (n1, n2, d), r (n1, n2, d), a (n1, n2), b (n1, n2).
    ``r`` may hold +inf to make a bump ignore a coordinate.
    ``wendland_variant`` 0 is the polynomial as printed (35 u^3), 1 is the
    textbook Wendland phi_{3,3} (32 u^3).
    """

    s0: float
    r0: np.ndarray
    h: np.ndarray
    r: np.ndarray
    a: np.ndarray
    b: np.ndarray
    nugget: float
    wendland_variant: int = 0
    core: "Core | None" = None
    # per-point error variances tau^2(x_p) of Eq. Zcov added to the nugget on
    # the diagonal: None, a float64 array (n,) in original point order, or a
    # CUDA float64 tensor of that shape (used in place by the library binding)
    tau2: object = None

    @property
    def d(self) -> int:
        return int(self.r0.shape[0])

    @property
    def n1(self) -> int:
        return int(self.a.shape[0])

    @property
    def n2(self) -> int:
        return int(self.a.shape[1])

    def copy(self) -> "Theta":
        return Theta(float(self.s0), self.r0.copy(), self.h.copy(), self.r.copy(),
                     self.a.copy(), self.b.copy(), float(self.nugget),
                     int(self.wendland_variant), None if self.core is None else self.core.copy(),
                     self.tau2)


@dataclasses.dataclass
class Problem:
    """One data set with its hyper-parameters and observations."""

    name: str
    x: np.ndarray                    # (n, d) float64, original order
    theta: Theta
    y: Optional[np.ndarray] = None   # (n,) residual z - W beta, or None
    z_std: Optional[np.ndarray] = None  # (n,) N(0,1) draws to be coloured by a caller
    cell: Optional[np.ndarray] = None   # suggested binning cell size per coordinate

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])


def _calibration() -> dict:
    path = os.path.join(_HERE, "calibration.json")
    with open(path) as f:
        return json.load(f)


def _bumps(rng, n1, n2, lo, hi, radius, amp_lo=0.5, amp_hi=1.0):
    """Centres uniform on the box [lo, hi), radii fixed, amplitudes U[amp_lo, amp_hi], b = 1."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d = lo.shape[0]
    h = lo + (hi - lo) * rng.random((n1, n2, d))
    r = np.broadcast_to(np.asarray(radius, np.float64), (n1, n2, d)).copy()
    a = rng.uniform(amp_lo, amp_hi, (n1, n2))
    b = np.ones((n1, n2))
    return h, r, a, b


def noise_variances(n: int, seed: int, lo: float = 0.0, hi: float = 0.05) -> np.ndarray:
    """Per-point error variances tau^2(x_p) ~ U(lo, hi) (Eq. Zcov's Delta),
    float64 (n,) in original point order."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def uniform_problem(n: int, d: int, seed: int, *, r0=0.05, n1=2, n2=2, bump_radius=0.2,
                    s0=1.0, nugget=1e-2, amp=(0.5, 1.0), wendland_variant=0,
                    name: str = "uniform") -> Problem:
    """n points uniform on [0,1]^d with n1 x n2 bumps; y is left to the caller.

    Draw order: points, bump centres, amplitudes, then n standard normals.
    """
    rng = np.random.default_rng(seed)
    x = rng.random((n, d))
    h, r, a, b = _bumps(rng, n1, n2, np.zeros(d), np.ones(d), bump_radius, *amp)
    z = rng.standard_normal(n)
    r0v = np.broadcast_to(np.asarray(r0, np.float64), (d,)).copy()
    th = Theta(s0, r0v, h, r, a, b, nugget, wendland_variant)
    return Problem(name, x, th, y=None, z_std=z, cell=r0v * 1.15)


def config1() -> Problem:
    """Plain method at n = 2000: uniform points on [0,1]^2, Wendland radius 0.05,
    2 x 2 bumps (radius 0.2), nugget 1e-2.  y ~ N(0, K) is formed by the caller
    from ``z_std`` (a Cholesky colouring needs the covariance itself)."""
    p = uniform_problem(2000, 2, 1, r0=0.05, n1=2, n2=2, bump_radius=0.2, name="cfg1-n2000-2d")
    return p


def gmm_points(rng, n: int, n_comp: int = 20):
    means = rng.random((n_comp, 2))
    sds = rng.uniform(0.02, 0.1, n_comp)
    comp = rng.integers(0, n_comp, n)
    x = means[comp] + sds[comp, None] * rng.standard_normal((n, 2))
    return x


def smooth_field_2d(x):
    return np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])


def gmm_problem(n: int, seed: int, r0: float, bump_radius: float, *, n1=4, n2=4,
                nugget=1e-2, name="gmm") -> Problem:
    """n points from a 20-component isotropic Gaussian mixture (means U[0,1]^2,
    sd U[0.02, 0.1], equal weights, no clipping); 4 x 4 bumps with centres on
    the unit square; y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.1^2).

    Draw order: mixture, bumps, noise."""
    rng = np.random.default_rng(seed)
    x = gmm_points(rng, n)
    h, r, a, b = _bumps(rng, n1, n2, np.zeros(2), np.ones(2), bump_radius)
    y = smooth_field_2d(x) + 0.1 * rng.standard_normal(n)
    r0v = np.array([r0, r0])
    th = Theta(1.0, r0v, h, r, a, b, nugget, 0)
    return Problem(name, x, th, y=y, cell=r0v * 1.15)


def random_core(kind: int, d: int, seed: int, *, nu2: int = 5, n_basis: int = 4, ell: float = 0.08,
                sigma0: float = 1.3, Sigma0: float = 1.0, width: float = 0.35, phi_sd: float = 0.6) -> Core:
    """A core kernel with seeded parameters: basis centres U[0,1]^d, coefficients
    N(0, phi_sd^2) (so sigma(x) and Sigma(x) vary by a factor of a few over the unit
    cube), per-coordinate scales ell and widths ``width``."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, 1.0, size=(n_basis, d))
    phi_s = rng.normal(0.0, phi_sd, size=n_basis)
    phi_S = rng.normal(0.0, phi_sd, size=n_basis)
    ellv = np.ones(3)
    ellv[:d] = ell
    wv = np.ones(3)
    wv[:d] = width
    return Core(int(kind), int(nu2), float(sigma0), ellv, float(Sigma0), centers, wv, phi_s, phi_S)


def core_problem(kind: int, d: int, n: int = 1500, seed: int = 11, nu2: int = 5, **kw) -> Problem:
    """A uniform problem (2 x 2 bumps) whose kernel carries a core kernel."""
    p = uniform_problem(n, d, seed, r0=0.09 if d == 1 else (0.07 if d == 2 else 0.15), n1=2, n2=2,
                        bump_radius=0.25, name=f"core{kind}-d{d}-n{n}")
    p.theta.core = random_core(kind, d, seed + 1000, nu2=nu2, **kw)
    return p


def config2() -> Problem:
    """n = 100,000 points from the mixture, 16 bumps (4 x 4, radius 0.02); the
    Wendland radius comes from the calibration file (mean row length ~50)."""
    cal = _calibration()
    return gmm_problem(100_000, 2, cal["cfg2_r0"], 0.02, name="cfg2-n100k-gmm")


def spacetime_points(rng, n_stations: int, n_days: int):
    st = rng.random((n_stations, 2))
    days = np.arange(n_days, dtype=np.float64)
    x = np.empty((n_stations * n_days, 3))
    x[:, 0] = np.repeat(st[:, 0], n_days)   # station-major order
    x[:, 1] = np.repeat(st[:, 1], n_days)
    x[:, 2] = np.tile(days, n_stations)
    return x


def config3(n_stations: int = 3000, n_days: int = 365, seed: int = 3) -> Problem:
    """Space-time: stations uniform on [0,1]^2 times integer days 0..364 in
    station-major order (n = 1,095,000, d = 3).  Anisotropic Wendland radii
    (0.03, 0.03, 3 days); 16 x 4 space-time bumps with radii (0.05, 0.05, 14
    days); y = sin(2 pi s1) cos(2 pi s2) + 0.5 sin(2 pi t / 365) + N(0, 0.1^2).

    Draw order: stations, bumps, noise."""
    rng = np.random.default_rng(seed)
    x = spacetime_points(rng, n_stations, n_days)
    h, r, a, b = _bumps(rng, 16, 4, np.zeros(3), np.array([1.0, 1.0, 365.0]),
                        np.array([0.05, 0.05, 14.0]))
    y = (np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
         + 0.5 * np.sin(2 * np.pi * x[:, 2] / 365.0)
         + 0.1 * rng.standard_normal(x.shape[0]))
    r0v = np.array([0.03, 0.03, 3.0])
    th = Theta(1.0, r0v, h, r, a, b, 1e-2, 0)
    # cell: radius in space; one day in time (integer days, three rings reach |dt| <= 2)
    cell = np.array([0.03 * 1.0001, 0.03 * 1.0001, 1.0001])
    return Problem(f"cfg3-spacetime-{n_stations}x{n_days}", x, th, y=y, cell=cell)


def spacetime_core(kind: int, seed: int = 33, nu2: int = 5, n_basis: int = 8) -> Core:
    """A core kernel for the space-time workload: scales ell = (0.05, 0.05, 10
    days); for the nonstationary core, basis centres uniform over the domain
    [0,1]^2 x [0,365] days with widths (0.25, 0.25, 60 days) and coefficients
    N(0, 0.5^2)."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.0, 1.0, size=(n_basis, 3)) * np.array([1.0, 1.0, 365.0])
    phi_s = rng.normal(0.0, 0.5, size=n_basis)
    phi_S = rng.normal(0.0, 0.5, size=n_basis)
    return Core(int(kind), int(nu2), 1.0, np.array([0.05, 0.05, 10.0]), 1.0, centers,
                np.array([0.25, 0.25, 60.0]), phi_s, phi_S)


# ------------------------------------------------------------------ MCMC ---

@dataclasses.dataclass
class McmcPriors:
    """Prior bounds and initial proposal scales for the chain of Appendix C.

    beta ~ N(0, beta_var I); s0 ~ U(0, s0_max); r0_k ~ U(0, r0_max_k);
    nugget ~ U(0, nugget_max); h_ijk ~ U(lo_k, hi_k); r_ijk ~ U(0, r_max_k);
    a_ij ~ Bernoulli(pi_ij), pi_ij ~ U(0, 1); with a Matern core also
    sigma0 ~ U(0, sigma0_max) and ell_k ~ U(0, ell_max_k).  sd_* are the
    initial random-walk standard deviations of each coordinate.
    """

    lo: np.ndarray
    hi: np.ndarray
    r0_max: np.ndarray
    r_max: np.ndarray
    ell_max: np.ndarray = dataclasses.field(default_factory=lambda: np.full(3, 1e5))
    beta_var: float = 100.0 ** 2
    s0_max: float = 1e5
    nugget_max: float = 1e5
    sigma0_max: float = 1e5
    sd_beta: float = 0.05
    sd_s0: float = 0.05
    sd_r0: float = 0.002
    sd_nugget: float = 0.001
    sd_core: float = 0.02
    sd_h: float = 0.01
    sd_r: float = 0.005


def mcmc_draws(seed: int, n_iter: int, p: int, d2: int, d3: int, nb: int) -> list:
    """Random numbers of n_iter chain iterations, drawn in a fixed order per
    iteration: z1 (p normals, block 1), u1; z2 (d2 normals, block 2), u2;
    z3 (d3 normals, block 3), u3; ua (nb uniforms, amplitude proposals), u4;
    ub (nb uniforms, Gibbs draws of pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_iter):
        out.append(dict(z1=rng.standard_normal(p), u1=rng.random(), z2=rng.standard_normal(d2), u2=rng.random(),
                        z3=rng.standard_normal(d3), u3=rng.random(), ua=rng.random(nb), u4=rng.random(),
                        ub=rng.random(nb)))
    return out


def mean_covariates(x: np.ndarray) -> np.ndarray:
    """Covariates of a linear prior mean: an intercept and the coordinates,
    as a (1 + d, n) array (row k = covariate k)."""
    return np.ascontiguousarray(np.vstack([np.ones(x.shape[0]), np.asarray(x, np.float64).T]))


# ---------------------------------------------------------------- serving ---

def config4_pool(n_datasets: int = 16, base_seed: int = 4000):
    """Pool of mixture data sets with n log-uniform in [5k, 300k]; every radius
    is scaled by sqrt(1e5 / n) so rows keep about 50 nonzeros."""
    cal = _calibration()
    pool = []
    for k in range(n_datasets):
        rng = np.random.default_rng(base_seed + k)
        n = int(round(math.exp(rng.uniform(math.log(5e3), math.log(3e5)))))
        scale = math.sqrt(1e5 / n)
        p = gmm_problem(n, base_seed + k, cal["cfg2_r0"] * scale, 0.02 * scale,
                        name=f"cfg4-pool{k}-n{n}")
        pool.append(p)
    return pool


def perturb_theta(rng, th: Theta, sd: float = 0.05) -> Theta:
    """MCMC-style proposal: independent log-normal multipliers exp(N(0, sd^2))
    on r0 (one per coordinate), every bump radius, every amplitude and the
    nugget."""
    t = th.copy()
    t.r0 = t.r0 * np.exp(sd * rng.standard_normal(t.r0.shape))
    t.r = t.r * np.exp(sd * rng.standard_normal(t.r.shape))
    t.a = t.a * np.exp(sd * rng.standard_normal(t.a.shape))
    t.nugget = float(t.nugget * math.exp(sd * rng.standard_normal()))
    return t


def config4_requests(n_requests: int = 512, rate: float = 50.0, seed: int = 4,
                     n_datasets: int = 16):
    """Poisson stream of log-likelihood requests: (arrival_s, dataset_index, theta)."""
    rng = np.random.default_rng(seed)
    pool_meta = config4_pool(n_datasets)
    t = 0.0
    reqs = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(0, n_datasets))
        reqs.append((t, k, perturb_theta(rng, pool_meta[k].theta)))
    return pool_meta, reqs


def config5_requests(n_requests: int = 1000, seed: int = 5, m_lo: int = 1000,
                     m_hi: int = 50000, n_days: int = 365):
    """Prediction requests on the space-time training set: m ~ U{m_lo..m_hi}
    test points, uniform on the unit square times a uniform integer day."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_requests):
        m = int(rng.integers(m_lo, m_hi + 1))
        xs = np.empty((m, 3))
        xs[:, :2] = rng.random((m, 2))
        xs[:, 2] = rng.integers(0, n_days, m).astype(np.float64)
        out.append(xs)
    return out


def rademacher_counter_doc() -> str:
    """The probe generator shared in definition (not in code) by both sides.

    Probe l, original point index i, seed s: the counter k = (l << 40 | i) + 1
    indexes the SplitMix64 sequence started at state s, i.e. the value is the
    SplitMix64 output function applied to s + k * 0x9E3779B97F4A7C15 (mod 2^64);
    the entry is -1 if bit 63 of that output is set, else +1.
    """
    return rademacher_counter_doc.__doc__
