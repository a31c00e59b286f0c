"""Helpers shared by the GPU parity tests (no test functions here)."""
import numpy as np
import scipy.sparse as sp

# SLQ with plain three-term Lanczos on both sides, identical probes: the
# recurrence amplifies the two sides' rounding (other summation orders, and
# alpha formed as v.Av minus the previous step's w.v instead of v.(Av - beta
# v_prev), equal in exact arithmetic), so the plain estimates are held to this
# relative bound; with full re-orthogonalisation on both sides the estimates
# are held to the parity bar (1e-8 float64, 1e-5 mixed).
PLAIN_BOUND = 2e-6


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def export(ctx, K):
    rp, col, val = ctx.export_csr(K)
    return host(rp).astype(np.int64), host(col).astype(np.int64), host(val)


def to_scipy(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def assert_pattern_equal(rp, col, ip, ci, what=""):
    assert rp.shape == ip.shape, f"{what}: row pointer length"
    if not np.array_equal(rp, ip):
        bad = np.nonzero(np.diff(rp) != np.diff(ip))[0]
        raise AssertionError(f"{what}: row lengths differ in {bad.size} rows, first {bad[:5]} "
                             f"gpu {np.diff(rp)[bad[:5]]} oracle {np.diff(ip)[bad[:5]]}")
    assert np.array_equal(col, ci), f"{what}: column indices differ"


def value_errors(val, ref):
    """max relative error with an absolute floor of 1e-14 * max|ref|."""
    scale = np.abs(ref).max() if ref.size else 1.0
    err = np.abs(val - ref)
    return float((err / (np.abs(ref) + 1e-14 * scale)).max()) if ref.size else 0.0


def rel(a, b):
    return abs(a - b) / abs(b)
