"""GPU parity of binning and assembly against the FP64 oracle.

Pattern and CSR indices must be bit-exact (the support predicate is the same
float64 expression on both sides).  FP64 entries: relative error <= 1e-12
(floor 1e-14 max|K|); float32 entries (mixed form): <= 1.2e-7 (one float32
rounding of a float64 value).  Bitwise symmetry K_pq == K_qp."""
import numpy as np
import pytest

from oracle import kernel
from workloads import Theta, config1, config2, uniform_problem
from gpu_util import PLAIN_BOUND, assert_pattern_equal, dev, export, host, rel, to_scipy, value_errors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
F32_TOL = 1.2e-7


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


def run_case(ctx, p, prec=0, cell="default", what=""):
    from paper_2411_05869_amd import FP64
    print(f"[case] {what} n={p.n} d={p.d} prec={prec} cell={cell}", flush=True)
    ds = ctx.dataset(dev(p.x), cell=p.cell if cell == "default" else cell)
    K = ctx.assemble(ds, p.theta, prec)
    rp, col, val = export(ctx, K)
    ip, ci, vo = kernel.sparse(p.x, p.theta)
    assert_pattern_equal(rp, col, ip, ci, what)
    err = value_errors(val, vo)
    assert err <= (FP64_TOL if prec == FP64 else F32_TOL), f"{what}: value error {err}"
    A = to_scipy(rp, col, val, p.n)
    assert (A != A.T).nnz == 0, f"{what}: not bitwise symmetric"
    assert K.nnz == ip[-1]
    return K, rp, col, val


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_small_uniform(ctx, d, prec):
    p = uniform_problem(400, d, 100 + d, r0=0.08 if d > 1 else 0.01, n1=3, n2=3, bump_radius=0.2)
    run_case(ctx, p, prec, what=f"uniform d={d}")


@pytest.mark.parametrize("cell", [None, [0.5, 0.5], [0.013, 0.02], [0.2, 0.007]])
def test_cell_size_does_not_change_pattern(ctx, cell):
    p = uniform_problem(500, 2, 7, r0=0.06, n1=2, n2=3, bump_radius=0.15)
    run_case(ctx, p, 0, cell=cell, what=f"cell={cell}")


def test_anisotropic_radii_3d(ctx):
    rng = np.random.default_rng(3)
    x = np.column_stack([rng.random(600), rng.random(600), rng.integers(0, 30, 600).astype(float)])
    th = Theta(1.3, np.array([0.2, 0.1, 3.0]), np.column_stack([rng.random(8), rng.random(8), rng.uniform(0, 30, 8)]).reshape(4, 2, 3),
               np.tile(np.array([0.2, 0.3, 5.0]), (4, 2, 1)), rng.uniform(0.5, 1, (4, 2)), np.ones((4, 2)), 0.02)
    from workloads import Problem
    p = Problem("aniso", x, th, cell=np.array([0.2, 0.1, 1.0]))
    run_case(ctx, p, 0, what="anisotropic")


def test_infinite_bump_radius(ctx):
    rng = np.random.default_rng(4)
    x = np.column_stack([rng.random(300), rng.random(300), rng.integers(0, 20, 300).astype(float)])
    r = np.tile(np.array([0.25, 0.25, np.inf]), (2, 2, 1))
    th = Theta(1.0, np.array([0.1, 0.1, 2.0]), rng.random((2, 2, 3)), r, np.ones((2, 2)), np.ones((2, 2)), 0.01)
    from workloads import Problem
    run_case(ctx, Problem("spatial-bumps", x, th, cell=np.array([0.1, 0.1, 2.0])), 0, what="inf radius")


def test_edge_cases(ctx):
    from workloads import Problem
    # a single point
    p = uniform_problem(1, 2, 1, r0=0.1, n1=1, n2=1)
    run_case(ctx, p, 0, what="n=1")
    # duplicated points: u0^2 = 0 -> local pair; nugget only on the index diagonal
    x = np.array([[0.3, 0.3], [0.3, 0.3], [0.9, 0.1]])
    th = Theta(1.0, np.array([0.1, 0.1]), np.array([[[0.3, 0.31]]]), np.full((1, 1, 2), 0.05), np.ones((1, 1)),
               np.ones((1, 1)), 0.5)
    run_case(ctx, Problem("dups", x, th, cell=None), 0, what="duplicates")
    # no bumps at all (n1 = 0): special case (1) of Sec. 2.3
    th0 = Theta(2.0, np.array([0.1, 0.1]), np.zeros((0, 0, 2)), np.zeros((0, 0, 2)), np.zeros((0, 0)),
                np.zeros((0, 0)), 0.1)
    run_case(ctx, Problem("nobumps", np.random.default_rng(5).random((300, 2)), th0), 0, what="n1=0")
    # amplitudes all zero: bumps structurally absent
    p2 = uniform_problem(300, 2, 6, r0=0.1, n1=2, n2=2)
    p2.theta.a[:] = 0.0
    run_case(ctx, p2, 0, what="a=0")
    # one bump covering everything: every row is dense (long rows everywhere)
    th1 = Theta(1.0, np.array([0.05, 0.05]), np.array([[[0.5, 0.5]]]), np.full((1, 1, 2), 5.0), np.ones((1, 1)),
                np.ones((1, 1)), 0.1)
    run_case(ctx, Problem("dense", np.random.default_rng(6).random((700, 2)), th1), 1, what="dense group")
    # points far outside the bumps and each other (diagonal matrix)
    p3 = uniform_problem(200, 3, 8, r0=1e-6, n1=1, n2=1, bump_radius=1e-3)
    run_case(ctx, p3, 0, what="diagonal")


def test_config1(ctx):
    run_case(ctx, config1(), 0, what="cfg1 fp64")
    run_case(ctx, config1(), 1, what="cfg1 mixed")


@pytest.mark.parametrize("prec", [0, 1])
def test_config2(ctx, prec):
    run_case(ctx, config2(), prec, what=f"cfg2 {'fp64' if prec == 0 else 'mixed'}")


def test_binning_is_permutation_and_deterministic(ctx):
    p = config1()
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    perm = host(ds.permutation())
    assert np.array_equal(np.sort(perm), np.arange(p.n))
    ds2 = ctx.dataset(dev(p.x), cell=p.cell)
    assert np.array_equal(host(ds2.permutation()), perm)
    K1 = ctx.assemble(ds, p.theta, 0)
    K2 = ctx.assemble(ds2, p.theta, 0)
    a, b = export(ctx, K1), export(ctx, K2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("prec", [0, 1])
def test_permutation_invariance(ctx, prec):
    # shuffled input points: the exported matrix (in the caller's order) is the
    # original one under the permutation, pattern and values bitwise; the
    # quadratic form agrees to rounding (the binned order inside a cell follows
    # the input order, so sums run in another order)
    from paper_2411_05869_amd import LOGDET_NONE
    p = uniform_problem(800, 3, 17, r0=0.15, n1=3, n2=2, bump_radius=0.3)
    perm = np.random.default_rng(4).permutation(p.n)
    y = np.random.default_rng(5).standard_normal(p.n)
    out = []
    for xx, yy in ((p.x, y), (p.x[perm], y[perm])):
        ds = ctx.dataset(dev(xx), cell=p.cell)
        K = ctx.assemble(ds, p.theta, prec)
        out.append((to_scipy(*export(ctx, K), p.n), ctx.loglik(K, dev(yy), logdet_mode=LOGDET_NONE)))
    (A, r1), (A2, r2) = out
    Ap = A[perm][:, perm].tocsr()
    Ap.sort_indices()
    A2.sort_indices()
    assert np.array_equal(A2.indptr, Ap.indptr) and np.array_equal(A2.indices, Ap.indices)
    assert np.array_equal(A2.data, Ap.data)
    print(f"[permutation prec={prec}] nnz {A.nnz} quad rel {rel(r1['quad'], r2['quad']):.2e}")
    assert rel(r1["quad"], r2["quad"]) <= (1e-12 if prec == 0 else 1e-9)


def test_invalid_theta_is_einval(ctx):
    from paper_2411_05869_amd import GPError
    p = uniform_problem(50, 2, 1)
    ds = ctx.dataset(dev(p.x))
    bad = p.theta.copy()
    bad.r0 = np.array([-1.0, 0.1])
    with pytest.raises(GPError) as e:
        ctx.assemble(ds, bad)
    assert e.value.name == "GP_EINVAL"
    bad = p.theta.copy()
    bad.a = bad.a.copy()
    bad.a[0, 0] = np.nan
    with pytest.raises(GPError) as e:
        ctx.assemble(ds, bad)
    assert e.value.name == "GP_EINVAL"
    x = p.x.copy()
    x[3, 1] = np.inf
    with pytest.raises(GPError) as e:
        ctx.dataset(dev(x))
    assert e.value.name == "GP_EINVAL"


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-5)])
def test_sixty_four_groups(ctx, prec, tol):
    """n1 = 64 groups, as many as a point's mask holds: masks use bit 63 and most
    masked points lie in several groups (2.6 on average), so the shared lists
    U_M are long and overlap.  Pattern and values, then the log-likelihood
    against the oracle: exact log det; SLQ with the oracle's probes, plain
    (whose three-term recurrence amplifies the two sides' different summation
    orders: held to PLAIN_BOUND) and with full re-orthogonalisation on both sides
    (within the bar)."""
    from oracle import likelihood, slq
    from paper_2411_05869_amd import LOGDET_EXACT, LOGDET_SLQ_REORTH
    p = uniform_problem(1200, 2, 64, r0=0.03, n1=64, n2=1, bump_radius=0.12)
    K, rp, col, val = run_case(ctx, p, prec, what="64 groups")
    Kd, _ = kernel.dense(p.x, p.theta)
    y = np.linalg.cholesky(Kd) @ p.z_std
    ref = likelihood.dense_cholesky(Kd, y)
    r = ctx.loglik(K, dev(y), logdet_mode=LOGDET_EXACT)
    seed = 64
    opts = dict(seed=seed, n_probes=30, n_lanczos=50)
    rs = ctx.loglik(K, dev(y), **opts)
    ro = ctx.loglik(K, dev(y), logdet_mode=LOGDET_SLQ_REORTH, **opts)
    o = slq.slq_logdet(Kd, seed=seed, n_probes=30, n_steps=50)
    oo = slq.slq_logdet(Kd, seed=seed, n_probes=30, n_steps=50, reorth=True)
    e_ll = rel(r["loglik"], ref["loglik"])
    e_slq, e_ro = rel(rs["logdet"], o["logdet"]), rel(ro["logdet"], oo["logdet"])
    print(f"[64 groups prec={prec}] nnz {K.nnz} ({K.nnz / p.n:.0f} per row); exact-mode loglik rel {e_ll:.2e}; "
          f"SLQ against the oracle's SLQ: plain rel {e_slq:.2e}, re-orthogonalised rel {e_ro:.2e}")
    assert r["status"] == 0 and rs["status"] == 0 and ro["status"] == 0
    assert e_ll <= tol and e_ro <= tol
    assert e_slq <= max(tol, PLAIN_BOUND)


def _group_layout(x, theta):
    """The grouping of the masked rows recomputed from the oracle's group
    membership: distinct masks, list sizes |U_M| = sum of the rows of every
    distinct mask sharing a group, entries in group blocks, and the list
    entries the one- and multi-column products stage (per tile of 16 and per
    super-tile of 64 rows of a mask)."""
    M, _ = kernel.features(x, theta)
    bits = (M.astype(np.uint64) << np.arange(M.shape[1], dtype=np.uint64)).sum(axis=1) if M.shape[1] else \
        np.zeros(len(x), np.uint64)
    masked = bits[bits != 0]
    dm, mult = np.unique(masked, return_counts=True)
    share = (dm[:, None] & dm[None, :]) != 0
    nu = share.astype(np.int64) @ mult.astype(np.int64)
    tiles = (mult + 15) // 16
    stiles = (mult + 63) // 64
    return dict(group_rows=int(len(masked)), group_masks=int(len(dm)), group_list_entries=int(nu.sum()),
                nnz_group=int((mult * nu).sum()), gemv_stage_entries=int((tiles * nu).sum()),
                gemm_stage_entries=int((stiles * nu).sum()))


@pytest.mark.parametrize("case", ["64 groups", "config 1", "config 2", "one dense group", "no bumps"])
def test_group_layout_against_oracle_membership(ctx, case):
    """The grouping of the masked rows (distinct masks, their lists, the
    tiles of the group-block products) against the same counts recomputed from
    the oracle's group membership."""
    from workloads import Problem
    if case == "64 groups":
        p = uniform_problem(1200, 2, 64, r0=0.03, n1=64, n2=1, bump_radius=0.12)
    elif case == "config 1":
        p = config1()
    elif case == "config 2":
        p = config2()
    elif case == "one dense group":
        th1 = Theta(1.0, np.array([0.05, 0.05]), np.array([[[0.5, 0.5]]]), np.full((1, 1, 2), 5.0), np.ones((1, 1)),
                    np.ones((1, 1)), 0.1)
        p = Problem("dense", np.random.default_rng(6).random((700, 2)), th1)
    else:
        th0 = Theta(2.0, np.array([0.1, 0.1]), np.zeros((0, 0, 2)), np.zeros((0, 0, 2)), np.zeros((0, 0)),
                    np.zeros((0, 0)), 0.1)
        p = Problem("nobumps", np.random.default_rng(5).random((300, 2)), th0)
    want = _group_layout(p.x, p.theta)
    K = ctx.assemble(ctx.dataset(dev(p.x), cell=p.cell), p.theta, 1)
    lo = K.layout()
    K.close()
    got = {k: lo[k] for k in want}
    print(f"[group layout {case}] {got}")
    assert got == want
