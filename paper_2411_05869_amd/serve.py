"""Continuous-batching request loop for log-likelihood and prediction requests.

Requests arrive over time (e.g. the hyper-parameter proposals of many MCMC
chains, Sec. 3.1 and Appendix C of the paper, and kriging-mean queries,
Sec. 3.2).  The server keeps the binned data sets and the prediction caches
resident on the device and runs requests on ``n_slots`` slots.  Each slot owns
a HIP stream, a library context bound to it and a host worker thread; the
library calls release the GIL, so the slots' work overlaps on the GPU.

Admission is first-in first-out under an HBM budget: the request at the head
of the queue starts as soon as a slot is free and its footprint estimate fits
in the budget not reserved by running requests.  A request whose footprint
exceeds the whole budget is rejected with GP_ENOMEM.  The estimate is made
before the matrix exists (n times a per-data-set row-length estimate); once
the slot has assembled the matrix the backend reports the footprint computed
from the exact entry count and the reservation is corrected to it (the slot
then also runs under a hard per-context budget of that size).

Requests that are waiting together are batched when the backend can run them
in shared launches: log-likelihoods of small problems (gp_loglik_batch: the
matrices stacked block-diagonally, each problem with its own scalars and
stopping test) and predictions (gp_predict_batch: the rows of all requests
back to back with a row-offset table, each request with its own predictor);
the results are split afterwards.

The scheduling logic is independent of the device: a ``Backend`` runs one
request (or batch) and estimates footprints.  ``GpuBackend`` uses the HIP
library; tests drive the scheduler with a CPU fake backend.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Any, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class LoglikRequest:
    dataset: str
    theta: Any
    precision: int = 1
    arrival: float = 0.0
    rid: int = -1


@dataclasses.dataclass
class PredictRequest:
    predictor: str
    xs: Any                    # (m, d) float64 numpy array or device tensor
    precision: int = 0
    arrival: float = 0.0
    rid: int = -1


@dataclasses.dataclass
class Completion:
    rid: int
    kind: str
    arrival: float
    start: float
    done: float
    slot: int
    result: Any = None
    error: Optional[str] = None
    batch: int = 1

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Backend:
    """Runs requests; must be safe to call from one thread per slot."""

    n_slots: int = 1
    # set by the Server while it runs: on_exact_footprint(slot, nbytes) corrects
    # the reservation of the slot's running request to nbytes
    on_exact_footprint = None

    def footprint(self, req) -> int:
        raise NotImplementedError

    def run_loglik(self, slot: int, req: LoglikRequest):
        raise NotImplementedError

    def run_predict(self, slot: int, reqs: List[PredictRequest]):
        raise NotImplementedError

    def can_batch(self, a: PredictRequest, b: PredictRequest) -> bool:
        """Whether b may join a's prediction launch (default: same predictor)."""
        return a.predictor == b.predictor and a.precision == b.precision

    def can_batch_loglik(self, a: LoglikRequest, b: LoglikRequest) -> bool:
        """Whether b may join a's likelihood launches (default: never)."""
        return False

    def run_loglik_batch(self, slot: int, reqs: List[LoglikRequest]):
        raise NotImplementedError


class Server:
    """FIFO admission by footprint over ``backend.n_slots`` slots."""

    def __init__(self, backend: Backend, hbm_budget: int, max_predict_batch_points: int = 1 << 20,
                 max_loglik_batch: int = 16):
        self.backend = backend
        self.n_slots = backend.n_slots
        self.budget = int(hbm_budget)
        self.max_batch_points = max_predict_batch_points
        self.max_loglik_batch = max_loglik_batch
        self.peak_reserved = 0
        self.corrections = []      # (estimate, exact) per reported footprint

    def run(self, requests: List[Any], timeout: float = 3600.0) -> List[Completion]:
        """Serves ``requests`` (each with an ``arrival`` offset in seconds from
        the call) and returns one Completion per request, in request order."""
        for i, r in enumerate(requests):
            if r.rid < 0:
                r.rid = i
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: collections.deque = collections.deque()
        done: Dict[int, Completion] = {}
        cv = threading.Condition()
        finished: collections.deque = collections.deque()
        work = [queue.Queue() for _ in range(self.n_slots)]
        free = list(range(self.n_slots))
        reserved = 0
        slot_fp = [0] * self.n_slots     # reservation of each slot's running request
        t0 = time.perf_counter()

        def on_exact(slot, nbytes):
            nonlocal reserved
            with cv:
                self.corrections.append((slot_fp[slot], int(nbytes)))
                reserved += int(nbytes) - slot_fp[slot]
                slot_fp[slot] = int(nbytes)
                self.peak_reserved = max(self.peak_reserved, reserved)
                cv.notify_all()   # a smaller reservation may admit the next request now

        self.backend.on_exact_footprint = on_exact

        def now():
            return time.perf_counter() - t0

        def worker(slot):
            while True:
                item = work[slot].get()
                if item is None:
                    return
                batch, fp = item
                start = now()
                err = None
                try:
                    if isinstance(batch[0], LoglikRequest):
                        if len(batch) == 1:
                            res = [self.backend.run_loglik(slot, batch[0])]
                        else:
                            res = self.backend.run_loglik_batch(slot, batch)
                    else:
                        res = self.backend.run_predict(slot, batch)
                except Exception as e:  # reported per request, the slot stays usable
                    err = f"{type(e).__name__}: {e}"
                    res = [None] * len(batch)
                t = now()
                with cv:
                    for r, out in zip(batch, res):
                        kind = "loglik" if isinstance(r, LoglikRequest) else "predict"
                        finished.append(Completion(r.rid, kind, r.arrival, start, t, slot, out, err, len(batch)))
                    finished.append(("slot", slot, fp))
                    cv.notify_all()

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.n_slots)]
        for th in threads:
            th.start()
        total = len(requests)
        try:
            with cv:
                while len(done) < total:
                    if now() > timeout:
                        raise TimeoutError("serving did not finish in time")
                    t = now()
                    while pending and pending[0].arrival <= t:
                        waiting.append(pending.popleft())
                    # collect completions: free slots and budget
                    while finished:
                        item = finished.popleft()
                        if isinstance(item, tuple):
                            _, slot, _fp = item
                            free.append(slot)
                            free.sort()
                            reserved -= slot_fp[slot]
                            slot_fp[slot] = 0
                        else:
                            done[item.rid] = item
                    # admit from the head while a slot is free and the footprint fits
                    while waiting and free:
                        head = waiting[0]
                        fp = self.backend.footprint(head)
                        if fp > self.budget:
                            waiting.popleft()
                            done[head.rid] = Completion(head.rid, type(head).__name__, head.arrival, t, t, -1, None,
                                                        f"GP_ENOMEM: footprint {fp} exceeds the budget {self.budget}")
                            continue
                        if reserved + fp > self.budget:
                            break
                        batch = [waiting.popleft()]
                        if isinstance(head, PredictRequest):
                            # merge waiting requests the backend can run in the same launch
                            pts = _npts(head.xs)
                            keep = collections.deque()
                            while waiting:
                                r = waiting.popleft()
                                fr = self.backend.footprint(r)
                                if (isinstance(r, PredictRequest) and _can_batch(self.backend, head, r)
                                        and pts + _npts(r.xs) <= self.max_batch_points
                                        and reserved + fp + fr <= self.budget):
                                    batch.append(r)
                                    pts += _npts(r.xs)
                                    fp += fr
                                else:
                                    keep.append(r)
                            waiting.extend(keep)
                        elif self.max_loglik_batch > 1 and _can_batch_loglik(self.backend, head, head):
                            # merge waiting likelihoods of small problems
                            keep = collections.deque()
                            while waiting:
                                r = waiting.popleft()
                                fr = self.backend.footprint(r)
                                if (len(batch) < self.max_loglik_batch and isinstance(r, LoglikRequest)
                                        and _can_batch_loglik(self.backend, head, r)
                                        and reserved + fp + fr <= self.budget):
                                    batch.append(r)
                                    fp += fr
                                else:
                                    keep.append(r)
                            waiting.extend(keep)
                        reserved += fp
                        self.peak_reserved = max(self.peak_reserved, reserved)
                        slot = free.pop(0)
                        slot_fp[slot] = fp
                        work[slot].put((batch, fp))
                    if len(done) >= total:
                        break
                    wait = 0.05
                    if pending:
                        wait = max(0.0, min(wait, pending[0].arrival - now()))
                    if not finished:
                        cv.wait(timeout=wait)
        finally:
            for q in work:
                q.put(None)
            for th in threads:
                th.join(timeout=60)
            self.backend.on_exact_footprint = None
        return [done[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def _npts(xs) -> int:
    return int(xs.shape[0])


def _can_batch(backend, a: PredictRequest, b: PredictRequest) -> bool:
    f = getattr(backend, "can_batch", None)
    return f(a, b) if f is not None else Backend.can_batch(backend, a, b)


def _can_batch_loglik(backend, a: LoglikRequest, b: LoglikRequest) -> bool:
    f = getattr(backend, "can_batch_loglik", None)
    return bool(f(a, b)) if f is not None else False


def latency_stats(comps: List[Completion]) -> dict:
    """p50/p99/mean latency and throughput; ``mean_slots_busy`` is the time-average
    number of slots running a request (or batch) between the first start and the
    last completion."""
    ok = [c for c in comps if c.error is None]
    lat = np.array([c.latency for c in ok]) if ok else np.zeros(0)
    span = (max(c.done for c in ok) - min(c.arrival for c in ok)) if ok else float("nan")
    # one interval per slot run (a batch's requests share it)
    runs = {(c.slot, c.start, c.done) for c in ok}
    busy_span = (max(c.done for c in ok) - min(c.start for c in ok)) if ok else float("nan")
    busy = sum(e - s for _, s, e in runs) / busy_span if ok and busy_span > 0 else float("nan")
    return dict(completed=len(ok), failed=len(comps) - len(ok),
                p50_ms=float(np.percentile(lat, 50) * 1e3) if lat.size else float("nan"),
                p99_ms=float(np.percentile(lat, 99) * 1e3) if lat.size else float("nan"),
                mean_ms=float(lat.mean() * 1e3) if lat.size else float("nan"),
                throughput_per_s=len(ok) / span if ok and span > 0 else float("nan"),
                mean_slots_busy=round(float(busy), 3))


# ------------------------------------------------------------------ GPU backend

class GpuBackend(Backend):
    """Runs requests through the HIP library, one context and stream per slot.

    Likelihoods of problems with at most ``batch_max_n`` points are batched
    (gp_loglik_batch); larger ones run alone."""

    def __init__(self, n_slots: int = 4, device: int = 0, solve_opts: Optional[dict] = None,
                 batch_max_n: int = 50_000, hard_budget: bool = True):
        import torch

        from . import Context
        self.torch = torch
        self.n_slots = n_slots
        self.device = device
        self.dev = torch.device("cuda", device)
        self.setup = Context(device)
        self.streams = [torch.cuda.Stream(device) for _ in range(n_slots)]
        self.ctxs = [Context(device, stream=s) for s in self.streams]
        self.datasets: Dict[str, Any] = {}
        self.predictors: Dict[str, Any] = {}
        self.opts = dict(seed=2411, n_probes=30, n_lanczos=50)
        self.opts.update(solve_opts or {})
        self.row_estimate: Dict[str, float] = {}
        self.batch_max_n = batch_max_n
        self.hard_budget = hard_budget

    def add_dataset(self, name: str, x, y, cell=None, row_estimate: float = 100.0):
        torch = self.torch
        xd = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=self.dev)
        yd = torch.as_tensor(np.ascontiguousarray(y), dtype=torch.float64, device=self.dev)
        ds = self.setup.dataset(xd, cell=cell)
        torch.cuda.synchronize(self.device)
        self.datasets[name] = (ds, yd)
        self.row_estimate[name] = row_estimate

    def add_predictor(self, name: str, dataset: str, theta, alpha=None, precision: int = 0):
        """Caches alpha = K^-1 y for theta (solved here if not given)."""
        torch = self.torch
        ds, yd = self.datasets[dataset]
        if alpha is None:
            K = self.setup.assemble(ds, theta, precision)
            alpha = torch.empty(ds.n, dtype=torch.float64, device=self.dev)
            self.setup.solve(K, yd, alpha)
            K.close()
        core = getattr(theta, "core", None)
        kind = int(core.kind) if core is not None else 0
        self.predictors[name] = (self.setup.predictor(ds, theta, alpha), ds.d, kind)
        torch.cuda.synchronize(self.device)

    def can_batch(self, a: PredictRequest, b: PredictRequest) -> bool:
        # one gp_predict_batch launch takes predictors of one dimension and core kind
        pa, pb = self.predictors[a.predictor], self.predictors[b.predictor]
        return a.precision == b.precision and pa[1:] == pb[1:]

    def can_batch_loglik(self, a: LoglikRequest, b: LoglikRequest) -> bool:
        na, nb = self.datasets[a.dataset][0].n, self.datasets[b.dataset][0].n
        return a.precision == b.precision and max(na, nb) <= self.batch_max_n

    def _loglik_bytes(self, n: int, nnz: float, precision: int, batched: bool) -> int:
        """Device bytes of one likelihood: the matrix (CSR, int16 column
        offsets, row quads of the 32-column products at one union entry of a
        column id and four values per 1.5 nonzeros or fewer, block-Jacobi
        blocks), the solver's vectors and Lanczos blocks with the work space's
        growth margin, and for a batch the stacked copy of the matrix."""
        vb = 4 if precision == 1 else 8
        csr = nnz * (4 + vb) + 24 * n
        col16 = 2 * (nnz + 64)
        quads = nnz / 1.5 * (4 + 4 * vb) + 6 * n
        bjac = 48 * n
        mat = csr + col16 + quads + bjac
        work = 1.25 * n * (3 * 32 * 8 + 10 * 8) + 16 * n + (1 << 20)
        return int(mat * (2 if batched else 1) + work)

    def footprint(self, req) -> int:
        if isinstance(req, LoglikRequest):
            n = self.datasets[req.dataset][0].n
            return self._loglik_bytes(n, n * self.row_estimate[req.dataset], req.precision,
                                      n <= self.batch_max_n)
        return int(_npts(req.xs) * (8 * 3 + 8) + (1 << 16))

    def _assembled(self, slot: int, reqs: List[LoglikRequest], Ks) -> None:
        """Reports (and returns) the footprint computed from the exact entry
        counts of the assembled matrices; also raises the data sets' row-length
        estimates to what the matrices hold."""
        exact = 0
        for r, K in zip(reqs, Ks):
            self.row_estimate[r.dataset] = max(self.row_estimate[r.dataset], K.nnz / K.n * 1.1)
            exact += self._loglik_bytes(K.n, K.nnz, r.precision, len(reqs) > 1)
        if self.on_exact_footprint is not None:
            self.on_exact_footprint(slot, exact)
        return exact

    def _run(self, slot: int, reqs: List[LoglikRequest]):
        ctx = self.ctxs[slot]
        with self.torch.cuda.stream(self.streams[slot]):
            base = ctx.memory()[0]
            Ks = []
            try:
                for r in reqs:
                    ds, _ = self.datasets[r.dataset]
                    Ks.append(ctx.assemble(ds, r.theta, r.precision))
                exact = self._assembled(slot, reqs, Ks)
                if self.hard_budget:
                    ctx.set_hbm_budget(base + exact)
                ys = [self.datasets[r.dataset][1] for r in reqs]
                if len(reqs) == 1:
                    res = [ctx.loglik(Ks[0], ys[0], raise_on_error=False, **self.opts)]
                else:
                    res = ctx.loglik_batch(Ks, ys, raise_on_error=False, **self.opts)
                for r, K in zip(res, Ks):
                    r["nnz"] = K.nnz
                    r["batch"] = len(reqs)
            finally:
                for K in Ks:
                    K.close()
                if self.hard_budget:
                    ctx.set_hbm_budget(0)
        return res

    def run_loglik(self, slot: int, req: LoglikRequest):
        return self._run(slot, [req])[0]

    def run_loglik_batch(self, slot: int, reqs: List[LoglikRequest]):
        return self._run(slot, reqs)

    def run_predict(self, slot: int, reqs: List[PredictRequest]):
        torch = self.torch
        ctx = self.ctxs[slot]
        preds = [self.predictors[r.predictor][0] for r in reqs]
        with torch.cuda.stream(self.streams[slot]):
            parts = [torch.as_tensor(np.ascontiguousarray(r.xs), dtype=torch.float64, device=self.dev)
                     if not isinstance(r.xs, torch.Tensor) else r.xs for r in reqs]
            xs = parts[0] if len(parts) == 1 else torch.cat(parts, 0)
            off = np.concatenate([[0], np.cumsum([q.shape[0] for q in parts])])
            m = ctx.predict_batch(preds, xs, off, precision=reqs[0].precision)
            host = m.cpu().numpy()
        out, o = [], 0
        for p in parts:
            out.append(host[o:o + p.shape[0]])
            o += p.shape[0]
        return out


# ------------------------------------------------------------------ CLI

def serve_loglik_stream(n_requests: int = 512, rate: float = 50.0, n_slots: int = 4, budget_gb: float = 64.0,
                        precision: int = 1, verbose: bool = True):
    """The MCMC-proposal workload: Poisson arrivals of log-likelihood requests
    on a pool of 16 mixture data sets (n log-uniform in [5k, 300k])."""
    from workloads import config4_requests
    from . import PRECOND_JACOBI
    pool, reqs = config4_requests(n_requests=n_requests, rate=rate)
    be = GpuBackend(n_slots=n_slots, solve_opts=dict(precond=PRECOND_JACOBI))
    for k, p in enumerate(pool):
        be.add_dataset(f"d{k}", p.x, p.y, cell=p.cell, row_estimate=60.0)
    requests = [LoglikRequest(f"d{k}", th, precision, arrival=t) for (t, k, th) in reqs]
    srv = Server(be, hbm_budget=int(budget_gb * 2 ** 30))
    comps = srv.run(requests)
    st = latency_stats(comps)
    st["peak_reserved_gb"] = srv.peak_reserved / 2 ** 30
    if verbose:
        print(st, flush=True)
    return st, comps


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--slots", type=int, default=4)
    args = ap.parse_args()
    st, _ = serve_loglik_stream(args.requests, args.rate, args.slots)
    print(json.dumps(st))
