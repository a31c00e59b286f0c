"""Scheduling logic of the serving loop, driven by a CPU fake backend:
completion of every request, FIFO admission, the HBM budget never exceeded,
rejection of requests that can never fit, overlap across slots, batching of
prediction requests and of small likelihoods, the exact footprint replacing
the estimate, and per-request error reporting."""
import threading
import time

import numpy as np
import pytest

from paper_2411_05869_amd.serve import LoglikRequest, PredictRequest, Server, latency_stats


class FakeBackend:
    def __init__(self, n_slots, work_s=0.02, fail_on=None):
        self.n_slots = n_slots
        self.work_s = work_s
        self.lock = threading.Lock()
        self.running = 0
        self.max_running_bytes = 0
        self.running_bytes = 0
        self.starts = []
        self.fail_on = fail_on or set()
        self.batches = []

    def footprint(self, req):
        if isinstance(req, LoglikRequest):
            return int(req.theta["bytes"])
        return 1000 * req.xs.shape[0]

    def _enter(self, fp, tag):
        with self.lock:
            self.running_bytes += fp
            self.max_running_bytes = max(self.max_running_bytes, self.running_bytes)
            self.starts.append(tag)

    def _leave(self, fp):
        with self.lock:
            self.running_bytes -= fp

    def run_loglik(self, slot, req):
        fp = self.footprint(req)
        self._enter(fp, req.rid)
        try:
            time.sleep(self.work_s)
            if req.rid in self.fail_on:
                raise RuntimeError("injected failure")
            return {"loglik": -float(req.rid), "slot": slot}
        finally:
            self._leave(fp)

    def run_predict(self, slot, reqs):
        fp = sum(self.footprint(r) for r in reqs)
        self._enter(fp, tuple(r.rid for r in reqs))
        self.batches.append(len(reqs))
        try:
            time.sleep(self.work_s)
            return [r.xs.sum(axis=1) for r in reqs]
        finally:
            self._leave(fp)


def ll(rid_bytes, arrival=0.0):
    return LoglikRequest("d", {"bytes": rid_bytes}, 1, arrival)


def test_all_complete_with_correct_results():
    be = FakeBackend(3)
    reqs = [ll(100, 0.001 * i) for i in range(20)]
    comps = Server(be, 10_000).run(reqs)
    assert [c.result["loglik"] for c in comps] == [-float(i) for i in range(20)]
    st = latency_stats(comps)
    assert st["completed"] == 20 and st["failed"] == 0 and st["p99_ms"] >= st["p50_ms"] > 0


def test_fifo_with_one_slot():
    be = FakeBackend(1, work_s=0.005)
    reqs = [ll(100, 0.0) for _ in range(10)]
    Server(be, 10_000).run(reqs)
    assert be.starts == list(range(10))


def test_budget_is_never_exceeded():
    be = FakeBackend(4, work_s=0.01)
    rng = np.random.default_rng(0)
    reqs = [ll(int(rng.integers(100, 600)), 0.0) for _ in range(40)]
    srv = Server(be, 1000)
    comps = srv.run(reqs)
    assert all(c.error is None for c in comps)
    assert be.max_running_bytes <= 1000
    assert srv.peak_reserved <= 1000


def test_request_that_never_fits_is_rejected():
    be = FakeBackend(2)
    reqs = [ll(100), ll(5000), ll(100)]
    comps = Server(be, 1000).run(reqs)
    assert comps[1].error.startswith("GP_ENOMEM")
    assert comps[0].error is None and comps[2].error is None


def test_slots_overlap():
    be = FakeBackend(4, work_s=0.05)
    reqs = [ll(10, 0.0) for _ in range(8)]
    t = time.perf_counter()
    comps = Server(be, 10_000).run(reqs)
    elapsed = time.perf_counter() - t
    assert elapsed < 0.05 * 8 * 0.6      # 8 x 50 ms of work on 4 slots
    # the time-average number of busy slots: about 4 here, 1 on one slot
    assert latency_stats(comps)["mean_slots_busy"] > 2.5
    one = latency_stats(Server(FakeBackend(1, work_s=0.02), 10_000).run([ll(10, 0.0) for _ in range(4)]))
    assert 0.9 <= one["mean_slots_busy"] <= 1.0 + 1e-9


def test_prediction_requests_are_batched_and_split():
    be = FakeBackend(1, work_s=0.03)
    rng = np.random.default_rng(1)
    xs = [rng.random((int(rng.integers(2, 9)), 2)) for _ in range(6)]
    reqs = [ll(10, 0.0)] + [PredictRequest("p", x, 0, 0.0) for x in xs]
    comps = Server(be, 1 << 30).run(reqs)
    assert max(be.batches) > 1
    for c, x in zip(comps[1:], xs):
        assert np.array_equal(c.result, x.sum(axis=1))


def test_backend_failure_is_reported_per_request():
    be = FakeBackend(2, fail_on={3})
    comps = Server(be, 10_000).run([ll(10, 0.0) for _ in range(6)])
    assert "injected failure" in comps[3].error
    assert all(c.error is None for i, c in enumerate(comps) if i != 3)


class BatchingBackend(FakeBackend):
    """Fake backend that batches likelihoods marked small and reports an exact
    footprint (factor x the estimate) once a request has started."""

    def __init__(self, n_slots, work_s=0.02, exact_factor=1.0):
        super().__init__(n_slots, work_s)
        self.exact_factor = exact_factor
        self.loglik_batches = []

    def can_batch_loglik(self, a, b):
        return a.theta.get("small", False) and b.theta.get("small", False)

    def _report(self, slot, reqs):
        if self.on_exact_footprint is not None:
            self.on_exact_footprint(slot, int(sum(self.footprint(r) for r in reqs) * self.exact_factor))

    def run_loglik(self, slot, req):
        self._report(slot, [req])
        return super().run_loglik(slot, req)

    def run_loglik_batch(self, slot, reqs):
        self._report(slot, reqs)
        fp = sum(self.footprint(r) for r in reqs)
        self._enter(fp, tuple(r.rid for r in reqs))
        self.loglik_batches.append([r.rid for r in reqs])
        try:
            time.sleep(self.work_s)
            return [{"loglik": -float(r.rid), "slot": slot} for r in reqs]
        finally:
            self._leave(fp)


def test_small_likelihoods_are_batched_and_split():
    be = BatchingBackend(1, work_s=0.03)
    big = LoglikRequest("d", {"bytes": 100}, 1, 0.0)
    small = [LoglikRequest("d", {"bytes": 10, "small": True}, 1, 0.0) for _ in range(6)]
    srv = Server(be, 1 << 20, max_loglik_batch=4)
    comps = srv.run([big] + small)
    assert all(c.error is None for c in comps)
    assert [c.result["loglik"] for c in comps] == [-float(i) for i in range(7)]
    assert be.loglik_batches[0] == [1, 2, 3, 4] and be.loglik_batches[1] == [5, 6]
    assert [c.batch for c in comps] == [1, 4, 4, 4, 4, 2, 2]


def _concurrency(comps):
    ev = sorted([(c.start, 1) for c in comps] + [(c.done, -1) for c in comps], key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_exact_footprint_replaces_the_estimate():
    # estimates of 300 bytes against a budget of 1000 admit three requests at
    # once; the exact footprint reported after assembly replaces each estimate
    big = BatchingBackend(4, work_s=0.03, exact_factor=2.0)
    srv = Server(big, 1000)
    comps = srv.run([ll(300, 0.0) for _ in range(8)])
    assert all(c.error is None for c in comps)
    assert len(srv.corrections) == 8 and all(exact == 2 * est for est, exact in srv.corrections)
    assert srv.peak_reserved >= 1200 and _concurrency(comps) <= 3
    # smaller than estimated: the freed reservation admits a fourth request
    small = BatchingBackend(4, work_s=0.05, exact_factor=0.5)
    srv = Server(small, 1000)
    comps = srv.run([ll(300, 0.0) for _ in range(8)])
    assert all(c.error is None for c in comps)
    assert all(exact * 2 == est for est, exact in srv.corrections)
    assert _concurrency(comps) == 4
