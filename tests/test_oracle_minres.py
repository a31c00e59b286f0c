"""Pins of the MINRES oracle (Paige and Saunders' method; the paper's solver,
Sec. 3.3): it must reproduce a direct solve, agree with SciPy's MINRES, keep its
residual estimate non-increasing, and solve a symmetric indefinite system on
which conjugate gradients break down."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import kernel, likelihood
from oracle.minres import minres
from workloads import uniform_problem


def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (q * ev) @ q.T


def test_matches_direct_solve_spd_jacobi():
    A = _spd(200, 1e4, 1)
    b = np.random.default_rng(2).standard_normal(200)
    d = np.diag(A).copy()
    r = minres(A, b, lambda v: v / d, rtol=1e-10)
    ref = np.linalg.solve(A, b)
    assert r["converged"] and r["relres"] <= 1e-10
    assert np.abs(r["x"] - ref).max() <= 1e-8 * np.abs(ref).max()


def test_agrees_with_scipy_minres():
    A = _spd(150, 1e3, 3)
    b = np.random.default_rng(4).standard_normal(150)
    mine = minres(A, b, lambda v: v, rtol=1e-13)
    ref, info = spla.minres(A, b, rtol=1e-14, maxiter=2000)
    assert info == 0
    assert np.abs(mine["x"] - ref).max() <= 1e-8 * np.abs(ref).max()


def test_residual_estimate_non_increasing():
    A = _spd(120, 1e5, 5)
    b = np.random.default_rng(6).standard_normal(120)
    d = np.diag(A).copy()
    ph = np.array(minres(A, b, lambda v: v / d, rtol=1e-12)["phibar"])
    assert np.all(np.diff(ph) <= 1e-12 * ph[0])


def test_indefinite_system():
    rng = np.random.default_rng(7)
    n = 100
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.concatenate([-np.geomspace(0.5, 50, n // 2), np.geomspace(0.5, 50, n - n // 2)])
    A = (q * ev) @ q.T
    b = rng.standard_normal(n)
    r = minres(A, b, lambda v: v, rtol=1e-12)
    ref = np.linalg.solve(A, b)
    assert r["converged"]
    assert np.abs(r["x"] - ref).max() <= 1e-8 * np.abs(ref).max()
    # conjugate gradients meet non-positive curvature on this matrix
    x = np.zeros(n); rr = b.copy(); p = rr.copy(); curv = []
    for _ in range(n):
        Ap = A @ p
        curv.append(p @ Ap)
        a = (rr @ rr) / curv[-1]
        x += a * p
        rn = rr - a * Ap
        p = rn + (rn @ rn) / (rr @ rr) * p
        rr = rn
    assert min(curv) <= 0.0


def test_kernel_matrix_matches_cholesky():
    p = uniform_problem(400, 2, 11, r0=0.12, n1=2, n2=2, bump_radius=0.25)
    K, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(K) @ p.z_std
    ref = likelihood.dense_cholesky(K, y)
    d = np.diag(K).copy()
    r = minres(K, y, lambda v: v / d, rtol=1e-12)
    assert r["converged"]
    assert np.abs(r["x"] - ref["alpha"]).max() <= 1e-9 * np.abs(ref["alpha"]).max()
    assert abs(float(y @ r["x"]) - ref["quad"]) <= 1e-10 * abs(ref["quad"])


def test_warm_start_from_the_solution():
    A = _spd(80, 1e3, 9)
    b = np.random.default_rng(10).standard_normal(80)
    ref = np.linalg.solve(A, b)
    r = minres(A, b, lambda v: v, x0=ref, rtol=1e-10)
    assert r["iters"] == 0 and r["converged"]
    # from a perturbed start it still converges to the same solution
    r = minres(A, b, lambda v: v, x0=ref + 1e-3, rtol=1e-10)
    assert r["converged"] and np.abs(r["x"] - ref).max() <= 1e-8 * np.abs(ref).max()
