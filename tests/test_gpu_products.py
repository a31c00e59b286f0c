"""GPU parity of the matrix products y = K x and Y = K X (gp_matvec: the
group-block GEMV and the CSR SpMV for one right-hand side, the MFMA group
blocks and the CSR SpMM for 2..32) against the oracle's matrix.

The GPU adds the same products in another order, so every row of the FP64
form is held to |y_p - y_ref,p| <= 1e-13 (|K| |x|)_p, y_ref the product with
the oracle's float64 values.  The mixed form stores each value rounded to
float32 (relative error <= 2^-24) and multiplies in float64, so its bound is
(2^-24 + 1e-13) (|K| |x|)_p; float32 accumulation would break it (about
sqrt(row length) 2^-24).  Sizes: config 1 (n = 2000; several tiles, a ragged tail, dense
group rows) with 1, 2, 7 and 32 right-hand sides, and the n = 1,095,000
space-time workload on sampled rows (oracle rows one at a time, the launch
configuration of the benchmark), and n = 1003 (an incomplete last group of four
rows for the 32-column path) with a dense cluster of rows longer than 128
entries beside short ones.  The one-column product's int16 column offsets are
checked where they fit (config 1) and where they do not (cells wider than 32767
binned positions: the product reads the int32 columns).  Shape errors in the
binding are refused before any device work."""
import numpy as np
import pytest

from oracle import kernel
from workloads import config1, config3
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05869_amd import Context
    return Context()


def _check_rows(y, ref, bound, prec, what):
    tol = 1e-13 if prec == 0 else 2.0 ** -24 + 1e-13
    err = np.abs(y - ref)
    worst = float(np.max(err / (bound + 1e-300)))
    print(f"[{what}] worst |dy| / (|K||x|) {worst:.2e} (bound {tol:.2e})")
    assert np.all(err <= tol * bound + 1e-300), what


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 7, 32])
def test_products_config1(ctx, prec, k):
    p = config1()
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    rng = np.random.default_rng(10 + k)
    X = rng.standard_normal((p.n, k)) if k > 1 else rng.standard_normal(p.n)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, prec)
    Y = host(ctx.matvec(K, dev(X)))
    absA = abs(A)
    _check_rows(Y, A @ X, absA @ np.abs(X), prec, f"cfg1 prec={prec} k={k}")


@pytest.fixture(scope="module")
def cfg3_rows():
    p = config3()
    M, F = kernel.features(p.x, p.theta)
    rng = np.random.default_rng(31)
    masked = np.nonzero(M.any(axis=1))[0]
    rows = np.unique(np.concatenate([rng.choice(p.n, 40, replace=False), rng.choice(masked, 20, replace=False)]))
    return p, {int(r): kernel.row(p.x, p.theta, int(r), M, F) for r in rows}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 32])
def test_products_config3_sampled_rows(ctx, cfg3_rows, prec, k):
    import torch
    p, orows = cfg3_rows
    rng = np.random.default_rng(40 + k)
    X = rng.standard_normal((p.n, k)) if k > 1 else rng.standard_normal(p.n)
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, prec)
    Y = host(ctx.matvec(K, dev(X)))
    K.close()
    torch.cuda.empty_cache()
    rows = sorted(orows)
    ref, bound = [], []
    for r in rows:
        c, v = orows[r]
        ref.append(v @ X[c])
        bound.append(np.abs(v) @ np.abs(X[c]))
    _check_rows(Y[rows], np.array(ref), np.array(bound), prec, f"cfg3 prec={prec} k={k} ({len(rows)} rows)")


def test_binding_refuses_bad_shapes(ctx):
    import torch
    p = config1()
    ds = ctx.dataset(dev(p.x), cell=p.cell)
    K = ctx.assemble(ds, p.theta, 0)
    with pytest.raises(ValueError):
        ctx.matvec(K, dev(np.zeros(p.n - 1)))
    with pytest.raises(ValueError):
        ctx.matvec(K, dev(np.zeros((p.n, 2, 2))))
    alpha = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    pred = ctx.predictor(ds, p.theta, alpha)
    with pytest.raises(ValueError):
        ctx.predict(pred, dev(np.zeros((5, 3))))
    with pytest.raises(ValueError):
        ctx.predict(pred, dev(np.zeros((5, 2))), out=torch.zeros(4, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        ctx.predict_var(K, p.theta, dev(np.zeros(10)))
    with pytest.raises(ValueError):
        ctx.mean_residual(None, [], dev(np.zeros(p.n)), out=torch.zeros(3, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("k", [1, 7, 32])
def test_products_ragged_and_long_rows(ctx, prec, k):
    # n = 1003 (the last group of four rows is incomplete) and a dense cluster
    # whose rows hold more than 128 local entries (the long-row path), next to
    # scattered short rows
    from workloads import Problem, Theta
    rng = np.random.default_rng(77)
    x = np.concatenate([0.5 + 0.03 * rng.standard_normal((500, 2)), rng.random((503, 2))])
    th = Theta(1.0, np.array([0.04, 0.04]), np.array([[[0.2, 0.8]], [[0.8, 0.2]]]), np.full((2, 1, 2), 0.15),
               np.ones((2, 1)), np.ones((2, 1)), 0.05)
    p = Problem("ragged-long", x, th, cell=None)
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    lens = np.diff(A.indptr)
    assert p.n % 4 != 0 and lens.max() > 128 and lens.min() < 128
    X = rng.standard_normal((p.n, k)) if k > 1 else rng.standard_normal(p.n)
    ds = ctx.dataset(dev(p.x))
    K = ctx.assemble(ds, p.theta, prec)
    Y = host(ctx.matvec(K, dev(X)))
    _check_rows(Y, A @ X, abs(A) @ np.abs(X), prec, f"ragged/long prec={prec} k={k} (rows > 128: {(lens > 128).sum()})")


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_tiny_sizes(ctx, n):
    # fewer points than one group of four rows, and one or two groups: the
    # products (1 and 32 columns) and a whole log-likelihood (CG, SLQ and
    # the exact mode) against the oracle's dense matrix
    from oracle import likelihood
    from paper_2411_05869_amd import LOGDET_EXACT
    from workloads import uniform_problem
    p = uniform_problem(n, 2, 90 + n, r0=0.6, n1=1, n2=1, bump_radius=0.5)
    A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
    Kd = A.toarray()
    rng = np.random.default_rng(n)
    ds = ctx.dataset(dev(p.x))
    K = ctx.assemble(ds, p.theta, 0)
    for k in (1, 32):
        X = rng.standard_normal((p.n, k)) if k > 1 else rng.standard_normal(p.n)
        Y = host(ctx.matvec(K, dev(X)))
        _check_rows(Y, A @ X, abs(A) @ np.abs(X), 0, f"n={n} k={k}")
    y = rng.standard_normal(p.n)
    ref = likelihood.dense_cholesky(Kd, y)
    for mode in (0, LOGDET_EXACT):
        r = ctx.loglik(K, dev(y), logdet_mode=mode)
        print(f"[tiny n={n} mode={mode}] loglik {r['loglik']:.12g} ref {ref['loglik']:.12g} steps {r['lanczos_steps']}")
        assert r["status"] == 0
        assert abs(r["quad"] - ref["quad"]) <= 1e-10 * abs(ref["quad"])
        if mode == LOGDET_EXACT or n == 1:  # one point: the probe estimate is exact
            assert abs(r["logdet"] - ref["logdet"]) <= 1e-10 * max(1.0, abs(ref["logdet"]))


@pytest.mark.parametrize("prec", [0, 1])
def test_column_offsets_and_their_fallback(ctx, prec):
    # the one-column product stores local columns as int16 offsets from the row
    # when they fit: here (cells 0.4 high, about 20,000 points per row of
    # cells) they do not, so the product reads the int32 columns; on config 1
    # they fit.  Both against the oracle.
    from workloads import Problem, Theta
    rng = np.random.default_rng(5)
    x = rng.random((80000, 2))
    th = Theta(1.0, np.array([0.0005, 0.4]), np.zeros((0, 0, 2)), np.zeros((0, 0, 2)), np.zeros((0, 0)),
               np.zeros((0, 0)), 0.1)
    for p, fits in ((Problem("wide offsets", x, th, cell=np.array([0.0005, 0.6])), False), (config1(), True)):
        A = kernel.to_scipy(*kernel.sparse(p.x, p.theta), p.n)
        xv = rng.standard_normal(p.n)
        ds = ctx.dataset(dev(p.x), cell=p.cell)
        K = ctx.assemble(ds, p.theta, prec)
        before = K.held_bytes()
        y = host(ctx.matvec(K, dev(xv)))
        grown = K.held_bytes() - before
        print(f"[offsets {p.name} prec={prec}] cache bytes {grown} (2 (nnz + 64) = {2 * (K.nnz + 64)})")
        assert grown == (2 * (K.nnz + 64) if fits else 0)
        _check_rows(y, A @ xv, abs(A) @ np.abs(xv), prec, f"offsets {p.name} prec={prec}")
