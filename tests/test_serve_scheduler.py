"""Scheduling logic of the serving loop, driven by a CPU fake backend:
completion of every request, FIFO admission, the HBM budget never exceeded,
rejection of requests that can never fit, overlap across slots, batching of
prediction requests, and per-request error reporting."""
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
    Server(be, 10_000).run(reqs)
    elapsed = time.perf_counter() - t
    assert elapsed < 0.05 * 8 * 0.6      # 8 x 50 ms of work on 4 slots


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
