"""Benchmark of the sparse-covariance exact-GP hot path on one MI355X.

Workload: the space-time data set (3,000 stations x 365 days, n = 1,095,000,
d = 3; anisotropic Wendland radii (0.03, 0.03, 3 days); 16 x 4 space-time
bumps; nugget 1e-2), resident on the device.  One step is one pass of the
hot path for one hyper-parameter vector:
    assemble K(theta) + sigma^2 I  ->  log-likelihood (block-Jacobi PCG for
    y^T K^-1 y to rtol 1e-10, SLQ log det with 30 probes x 80 Lanczos steps,
    a depth at which the estimate of this workload has converged to within
    0.2 standard errors of its 128-step value for six probe seeds: with 50
    steps its quadrature bias is 0.1-0.3%, several standard errors)
    ->  posterior mean at 10,000 test points with the solved alpha.
The mixed form (float32 values and PCG products, float64 residuals,
Lanczos vectors and reductions) is the headline; the float64 form is
timed on the same GPU.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K nnz/s + loglik evals/s at n=1M (mixed vs FP64); p50/p99 request latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n, nnz, vbytes, xbytes):
    # values + column ids + row pointers + one read of x + one write of y
    return nnz * (vbytes + 4) + (n + 1) * 8 + n * xbytes + n * xbytes


def spmm_bytes(n, nnz, vbytes, k, xbytes):
    # values + column ids + row pointers + X read once + Y written + scale vector
    return nnz * (vbytes + 4) + (n + 1) * 8 + 2 * n * k * xbytes + n * xbytes


def spmv_format_bytes(n, lo, vbytes, xbytes=8):
    """Bytes one one-column product must move in the format the library stores
    (gp_matrix_layout): the group blocks' values (no column ids), the other
    entries' values and column ids (int16 offsets when built), the row
    pointer and group-skip count of every row, x once and y once, the group
    rows' partial y read back, and per group tile of 16 rows its U_M list
    (column id and x value per entry)."""
    cb = 2 if lo["col16"] else 4
    return (lo["nnz_group"] * vbytes + lo["nnz_csr"] * (vbytes + cb) + n * (8 + 4 + 2 * xbytes)
            + lo["group_rows"] * xbytes + lo["gemv_stage_entries"] * (4 + xbytes))


def spmm_format_bytes(n, lo, vbytes, k=32, xbytes=8):
    """Bytes one 32-column product must move in the stored format: the group
    blocks' values, the four-row union entries (column id, four values), the
    listed rows' codes, X read once, Y written once, the group rows' partial
    Y read back, the row scale, and per group super-tile of 64 rows its U_M
    list (column id and X row)."""
    row = k * xbytes
    return (lo["nnz_group"] * vbytes + lo["quad_entries"] * (4 + 4 * vbytes) + lo["listed_rows"] * 4
            + n * (2 * row + xbytes) + lo["group_rows"] * row + lo["gemm_stage_entries"] * (4 + row))


def copy_peak_gbs(torch, dev, nbytes=1 << 30, reps=5):
    """Measured device-to-device copy rate (read + write bytes per second) of a
    1 GiB buffer, best of reps, timed with events on the current stream."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * nbytes / best / 1e9


EXACT_LOGLIK = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                            "spacetime_n1095000_exact.json")
TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "traffic_spacetime_n1095000.md")
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2411_05869_amd", "csrc")
# kernel groups whose HBM traffic the counter summary records: (source file, the
# kernels of one launch of the group, mixed form on the space-time workload)
TRAFFIC_GROUPS = {
    # the conjugate-gradient product: float32 values, float64 vectors
    "spmv_f32val_f64": ("spmv.hip", ("k_group_spmv<float, double, double, double>(",
                                     "k_spmv<float, double, double, double>(")),
    # the 32-column SLQ product: MFMA group blocks, their piece sums, the row quads
    "spmm": ("spmv.hip", ("k_group_spmm_mfma<float, double, true>(", "k_group_reduce<double>(",
                          "k_spmm_quad<float, true>(")),
    # the assembly's main kernels (float32 values)
    "assembly": ("assemble.hip", ("k_mask<3>(", "k_fvals<3>(", "k_local_rows<3, false, double, 0>(",
                                  "k_ulists(", "k_ugather<3>(", "k_local_rows<3, true, float, 0>(",
                                  "k_group_tile_fill<3, float, 0>(")),
}
CALIB_BYTES = 1 << 30


def vs_exact(r, workload):
    """Errors of a GPU log-likelihood against the exact one of the same workload
    (the oracle's day-blocked split, stored by tests/golden/make_spacetime_exact.py):
    the quadratic form and log-likelihood relative, the SLQ log det in its
    standard errors; None when the stored value is missing or for another workload."""
    try:
        with open(EXACT_LOGLIK) as f:
            g = json.load(f)
    except (OSError, ValueError):
        return None
    if g.get("workload") != workload:
        return None
    return dict(quad_rel=abs(r["quad"] - g["quad"]) / abs(g["quad"]),
                logdet_gap_se=abs(r["logdet"] - g["logdet"]) / r["logdet_se"],
                logdet_rel=abs(r["logdet"] - g["logdet"]) / abs(g["logdet"]),
                loglik_rel=abs(r["loglik"] - g["loglik"]) / abs(g["loglik"]), exact_loglik=g["loglik"])


ORACLE_SLQ = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                          "spacetime_n1095000_slq.json")


def vs_oracle_slq(r, workload, seed, probes, steps):
    """The GPU's SLQ log det against the oracle's with the same probes and step
    count (plain Lanczos on both sides; tests/golden/make_spacetime_slq.py);
    None when no stored estimate matches."""
    try:
        with open(ORACLE_SLQ) as f:
            g = json.load(f)
    except (OSError, ValueError):
        return None
    if (g.get("workload"), g.get("seed"), g.get("probes"), g.get("steps")) != (workload, seed, probes, steps):
        return None
    return dict(logdet_rel=abs(r["logdet"] - g["logdet"]) / abs(g["logdet"]), oracle_logdet=g["logdet"],
                seed=seed, probes=probes, steps=steps)


def source_sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic(group):
    """HBM bytes per launch of a kernel group from the committed counter summary,
    or None when it is missing or the group's source changed since it was taken."""
    try:
        fields = {}
        for line in open(TRAFFIC_PROFILE):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
        src = os.path.join(CSRC, TRAFFIC_GROUPS[group][0])
        if fields.get(f"{group}.source_sha256") != source_sha256(src):
            return None
        return int(fields[f"{group}.traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def summarize_pmc(fetch_dir, write_dir, command):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the kernel groups, scaled by
    what the same counters read for a copy of CALIB_BYTES bytes in the same run."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        rows = [r for r in csv.DictReader(open(f[0])) if r["Counter_Name"] == counter]
        copy = max(float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower())
        per = {}
        for g, (_, kernels) in TRAFFIC_GROUPS.items():
            for k in kernels:
                v = [float(r["Counter_Value"]) for r in rows if k in r["Kernel_Name"]]
                per[(g, k)] = (sum(v) / len(v), len(v)) if v else (0.0, 0)
        return copy, per

    cf, pf = load(fetch_dir, "FETCH_SIZE")
    cw, pw = load(write_dir, "WRITE_SIZE")
    sf, sw = CALIB_BYTES / (cf * 1024.0), CALIB_BYTES / (cw * 1024.0)
    lines = ["# HBM traffic of the main kernels on the space-time workload (n = 1,095,000), mixed form",
             "", "Two counter runs of the same command on one MI355X (run from /tmp with TMPDIR=/tmp), "
             "one with `--pmc FETCH_SIZE`, one with `--pmc WRITE_SIZE`:", "", "```", command, "```", "",
             f"Calibration: a device-to-device copy of {CALIB_BYTES} bytes (bench.py --copy-calibration) read "
             f"FETCH_SIZE {cf:.0f} KiB and WRITE_SIZE {cw:.0f} KiB; scale factors {sf:.4f} (fetch), {sw:.4f} (write).",
             "", "| group | kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | scaled MB/dispatch |",
             "|---|---|---:|---:|---:|---:|"]
    tail = ["", "Figures read by bench.py (one launch of a group = one dispatch of each of its kernels, scaled):", ""]
    for g, (src, kernels) in TRAFFIC_GROUPS.items():
        fetch = write = 0.0
        for k in kernels:
            (fv, fn), (wv, _) = pf[(g, k)], pw[(g, k)]
            fetch += fv * 1024.0 * sf
            write += wv * 1024.0 * sw
            lines.append(f"| {g} | `{k[:-1]}` | {fn} | {fv:.0f} | {wv:.0f} | {(fv * sf + wv * sw) * 1024 / 1e6:.1f} |")
        tail += [f"- {g}.fetch_bytes_per_launch: {int(fetch)}", f"- {g}.write_bytes_per_launch: {int(write)}",
                 f"- {g}.traffic_bytes_per_launch: {int(fetch + write)}",
                 f"- {g}.source_sha256: `{source_sha256(os.path.join(CSRC, src))}`"]
    lines += tail + [""]
    with open(TRAFFIC_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


STATS_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                             "loglik_step_spacetime_n1095000_kernel_stats.md")


def summarize_stats(stats_csv, bench_json, command, top=40):
    """Writes the kernel-statistics summary of a `rocprofv3 --kernel-trace --stats`
    run of bench.py (its kernel_stats.csv and the JSON line the same run printed)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    b = json.load(open(bench_json))
    lines = ["# Kernel statistics of bench.py on the space-time workload (n = 1,095,000, 87.35M nonzeros)", "",
             "`rocprofv3 --kernel-trace --stats` of the command below on one MI355X (run from /tmp with TMPDIR=/tmp); "
             "the bench line it printed is summarised after the table.", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("gps::(anonymous namespace)::", "")
        name = name.split("(")[0] if "(" in name else name
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / tot:.2f} |")
    ro = b["roofline"]
    lines += ["", "Bench line of the same run (library event timing on the library's streams):", "",
              f"- value {b['value']} loglik evals/s ({b['ms_per_step']} ms per step), fp64 {b['fp64']['value']}",
              f"- roofline: kernel {ro['kernel']}, {ro['avg_us']} us per launch, {ro['achieved']} GB/s, frac {ro['frac']}",
              f"- isolated steps (log det after the solve, one stream): "
              + ", ".join(f"{k} {v['avg_us']} us" for k, v in (b.get("roofline_isolated") or {}).items()
                          if isinstance(v, dict)),
              f"- assembly kernels {b['assemble_kernels_ms']} ms, wall {b['assemble_ms']} ms", ""]
    with open(STATS_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


OVERLAP_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "serving_overlap_mixture_4slots.md")


def serve_overlap(n_requests):
    """The first n_requests of the config-4 likelihood stream queued at once on 4
    slots without batching (the run a kernel trace of the slots' overlap is
    taken from); prints the host-side statistics as one JSON line."""
    from paper_2411_05869_amd import PRECOND_JACOBI
    from paper_2411_05869_amd.serve import GpuBackend, LoglikRequest, Server, latency_stats
    from workloads import config4_requests
    pool, reqs = config4_requests(n_requests=n_requests, rate=50.0)
    be = GpuBackend(n_slots=4, solve_opts=dict(precond=PRECOND_JACOBI), batch_max_n=0)
    for k, q in enumerate(pool):
        be.add_dataset(f"d{k}", q.x, q.y, cell=q.cell, row_estimate=60.0)
    requests = [LoglikRequest(f"d{k}", th, 1, arrival=0.0) for (_, k, th) in reqs]
    comps = Server(be, hbm_budget=64 << 30).run(requests)
    st = latency_stats(comps)
    st.update(requests=len(requests), slots=4, saturation_evals_per_s=round(len(requests) / max(c.done for c in comps), 2))
    print(json.dumps(st), flush=True)


def summarize_overlap(trace_csv, bench_json, command):
    """Writes the summary of a `rocprofv3 --kernel-trace` run of
    `bench.py --serve-overlap`: from the first assembly kernel to the last
    kernel, how long kernels of one, two, three or more HIP streams ran at
    the same time (each slot has a main stream and a side stream for the log
    det), and each stream's busy time."""
    import csv
    rows = list(csv.DictReader(open(trace_csv)))
    t0 = min(int(r["Start_Timestamp"]) for r in rows if "k_mask" in r["Kernel_Name"])
    ks = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Stream_Id"]) for r in rows
          if int(r["Start_Timestamp"]) >= t0]
    t1 = max(e for _, e, _ in ks)
    ev = sorted([(s_, 1, st) for s_, _, st in ks] + [(e, -1, st) for _, e, st in ks], key=lambda v: (v[0], v[1]))
    active = {}
    at_least = {1: 0, 2: 0, 3: 0, 4: 0}
    weighted = 0
    last = t0
    for t, d, st in ev:
        nbusy = sum(1 for v in active.values() if v > 0)
        for k in at_least:
            if nbusy >= k:
                at_least[k] += t - last
        weighted += nbusy * (t - last)
        last = t
        active[st] = active.get(st, 0) + d
    busy = {}
    for s_, e, st in ks:
        b = busy.setdefault(st, [0, 0])
        b[0] += 1
        b[1] += e - s_
    span = t1 - t0
    host = json.load(open(bench_json))
    lines = ["# Overlap of the serving slots' kernels (config-4 mixture likelihoods, 4 slots)", "",
             "`rocprofv3 --kernel-trace` of the command below on one MI355X (run from /tmp with TMPDIR=/tmp): "
             f"the first {host['requests']} likelihood requests of the config-4 stream queued at once on 4 slots, "
             "no batching. Each slot has its own HIP stream and context, and each context a second stream for the "
             "log det. Times from the first assembly kernel to the end of the last kernel.", "", "```", command,
             "```", "",
             f"- span {span / 1e6:.1f} ms; kernels of at least 1 / 2 / 3 / 4 streams running: "
             + " / ".join(f"{at_least[k] / 1e6:.1f} ms ({100 * at_least[k] / span:.0f}%)" for k in (1, 2, 3, 4)),
             f"- streams with a kernel running, averaged over the time any runs: {weighted / max(at_least[1], 1):.2f}",
             f"- host side (the same run): {host['saturation_evals_per_s']} evals/s, mean slots busy "
             f"{host['mean_slots_busy']}, p50 {host['p50_ms']:.0f} ms, p99 {host['p99_ms']:.0f} ms", "",
             "| stream | kernels | busy ms | busy % of span |", "|---|---:|---:|---:|"]
    for st, (cnt, b) in sorted(busy.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {st} | {cnt} | {b / 1e6:.1f} | {100 * b / span:.0f} |")
    lines.append("")
    with open(OVERLAP_PROFILE, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def cpu_serving(n_sample):
    """The oracle on sampled serving requests, on this host (single-threaded
    KD-tree, SuperLU and NumPy elementwise work): config 4, n_sample requests
    of the 512-request stream (a seeded choice), each the exact log-likelihood
    of its proposal on its data set (KD-tree pattern, float64 entries, SuperLU);
    config 5, the posterior mean at 64 test points of the first request by the
    oracle's cross-covariance rows over the 1,095,000 training points (any
    fixed weight vector: the time does not depend on it).  Prints one JSON line."""
    import numpy as np

    from oracle import kernel, likelihood
    from workloads import config3, config4_requests, config5_requests
    pool, reqs = config4_requests(n_requests=512, rate=50.0)
    pick = np.random.default_rng(44).choice(len(reqs), size=n_sample, replace=False)
    lat, ns = [], []
    for i in sorted(pick):
        _, k, th = reqs[i]
        q = pool[k]
        t0 = time.perf_counter()
        likelihood.sparse_lu(kernel.to_scipy(*kernel.sparse(q.x, th), q.n), q.y)
        lat.append(time.perf_counter() - t0)
        ns.append(q.n)
        log(f"cpu serving: request {i} n={q.n} {lat[-1]:.2f} s")
    p = config3()
    xs = config5_requests(1)[0][:64]
    w = np.random.default_rng(55).standard_normal(p.n)
    t0 = time.perf_counter()
    rp, cols, vals = kernel.cross_entries(xs, p.x, p.theta)
    _ = np.array([vals[rp[s]:rp[s + 1]] @ w[cols[rp[s]:rp[s + 1]]] for s in range(xs.shape[0])])
    tp = time.perf_counter() - t0
    lat_s = sorted(lat)
    out = dict(kind="oracle", host_cpus=os.cpu_count(),
               loglik=dict(requests=n_sample, n=[int(v) for v in ns], mean_s=round(float(np.mean(lat)), 3),
                           p50_s=round(lat_s[len(lat_s) // 2], 3), max_s=round(lat_s[-1], 3),
                           evals_per_s=round(n_sample / float(np.sum(lat)), 3)),
               predict=dict(points=int(xs.shape[0]), seconds=round(tp, 2), points_per_s=round(xs.shape[0] / tp, 2),
                            training_points=int(p.n)))
    print(json.dumps(out), flush=True)


def cpu_baseline(p):
    """The oracle on a bounded sample of the same workload (same point density):
    stations in [0, 0.5]^2, days 0..72 -> about 55k points, 2.3M nonzeros."""
    from oracle import kernel, likelihood
    sel = (p.x[:, 0] < 0.5) & (p.x[:, 1] < 0.5) & (p.x[:, 2] < 73)
    x, y = p.x[sel], p.y[sel]
    t0 = time.perf_counter()
    ip, ci, vo = kernel.sparse(x, p.theta)
    t1 = time.perf_counter()
    r = likelihood.sparse_lu(kernel.to_scipy(ip, ci, vo, x.shape[0]), y)
    t2 = time.perf_counter()
    try:
        from threadpoolctl import threadpool_info
        blas = [dict(api=i.get("internal_api"), threads=i.get("num_threads")) for i in threadpool_info()]
    except Exception:  # reported as unknown
        blas = None
    try:
        with open(EXACT_LOGLIK) as f:
            ex = json.load(f)
        exact = dict(seconds=ex["seconds"], n=ex["n"], method=ex["method"],
                     note="the oracle's exact log-likelihood of the whole workload (day-blocked split), "
                          "timed once when tests/golden/make_spacetime_exact.py wrote it, on an 8-core host")
    except (OSError, KeyError, ValueError):
        exact = None
    return dict(value=1.0 / (t2 - t0), unit="loglik evals/s", cores=1, kind="oracle",
                sample=f"same generator and theta restricted to stations in [0,0.5]^2 x days 0-72: n={x.shape[0]}, "
                       f"nnz={int(ip[-1])}; KD-tree pattern + float64 entries ({t1 - t0:.2f} s, "
                       f"{ip[-1] / (t1 - t0):.3g} nnz/s) then SuperLU exact log-likelihood ({t2 - t1:.2f} s); "
                       f"single-threaded (cKDTree, NumPy elementwise, SuperLU)",
                host_cpus=os.cpu_count(), blas_threads=blas, full_workload_exact=exact,
                nnz_per_s=float(ip[-1] / (t1 - t0)), n=int(x.shape[0]), loglik=r["loglik"]), (sel, ip[-1])


def serving_legs(args, ctx, ds, p, alpha):
    """Continuous batching: (1) the MCMC-proposal stream (Poisson, 50 req/s,
    mixture data sets with n log-uniform in [5k, 300k], mixed precision,
    SLQ 30 x 50, PCG rtol 1e-10; problems of at most 50k points batched by
    gp_loglik_batch) -> p50/p99 latency and evals/s, then the first
    --serve-saturation requests all queued at once on 1 slot, on 4 slots and
    on 4 slots with batching (evals/s: the slots' overlap and the batching's
    gain); (2) posterior means on the resident space-time training set,
    requests of 1k-50k test points: all queued at once (points/s), then
    Poisson at half that rate (p50/p99)."""
    import numpy as np

    from paper_2411_05869_amd.serve import GpuBackend, LoglikRequest, PredictRequest, Server, latency_stats
    from workloads import config4_requests, config5_requests
    res = {}
    from paper_2411_05869_amd import PRECOND_JACOBI
    pool, reqs = config4_requests(n_requests=args.serve_requests, rate=50.0)
    # point Jacobi: on the 2-D mixture sets, whose dense clusters fill cells with
    # many points, the cell-block preconditioner takes more CG iterations
    backends = {}

    def backend(slots, batch_max_n):
        key = (slots, batch_max_n)
        if key not in backends:
            be = GpuBackend(n_slots=slots, solve_opts=dict(precond=PRECOND_JACOBI), batch_max_n=batch_max_n)
            for k, q in enumerate(pool):
                be.add_dataset(f"d{k}", q.x, q.y, cell=q.cell, row_estimate=60.0)
            backends[key] = be
        return backends[key]

    def stream(be, rs, zero_arrival=False):
        requests = [LoglikRequest(f"d{k}", th, 1, arrival=0.0 if zero_arrival else t) for (t, k, th) in rs]
        srv = Server(be, hbm_budget=64 << 30)
        comps = srv.run(requests)
        st = latency_stats(comps)
        bad = [c.result["status"] for c in comps if c.error is None and c.result["status"] != 0]
        over = [ex / est for est, ex in srv.corrections if est > 0]
        st.update(requests=len(requests), nonzero_status=len(bad),
                  batches=int(sum(1 for c in comps if c.batch > 1)),
                  mean_batch=round(float(np.mean([c.batch for c in comps])), 2),
                  peak_reserved_gb=round(srv.peak_reserved / 2 ** 30, 3),
                  exact_over_estimate=[round(min(over), 3), round(max(over), 3)] if over else None)
        if zero_arrival:
            span = max(c.done for c in comps)
            st["saturation_evals_per_s"] = round(len(requests) / span, 2)
        return st

    log(f"serving: {len(reqs)} log-likelihood requests at 50 req/s on 4 slots")
    st = stream(backend(4, 50_000), reqs)
    st.update(rate_per_s=50.0, slots=4, precond="jacobi", batch_max_n=50_000,
              workload="mixture data sets n in [5k, 300k] (16 in the pool), log-normal proposals, mixed precision")
    res["loglik_stream"] = st
    sat = reqs[:args.serve_saturation]
    res["loglik_saturation"] = {}
    for label, slots, bmax in (("1slot", 1, 0), ("4slot", 4, 0), ("4slot_batched", 4, 50_000)):
        log(f"serving saturation: {len(sat)} requests at once, {label}")
        res["loglik_saturation"][label] = stream(backend(slots, bmax), sat, zero_arrival=True)
    # predictions on the resident training set (alpha from the last mixed step)
    be = backend(4, 50_000)
    be.datasets["train"] = (ds, None)
    be.predictors["train"] = (ctx.predictor(ds, p.theta, alpha), p.d, 0)
    xs = config5_requests(n_requests=args.predict_requests, seed=5)
    log(f"serving: {len(xs)} prediction requests")
    sat = [PredictRequest("train", x, 1, 0.0) for x in xs]
    comps = Server(be, hbm_budget=64 << 30).run(sat)
    span = max(c.done for c in comps)
    pts = sum(x.shape[0] for x in xs)
    rate = len(xs) / span
    rng = np.random.default_rng(55)
    arr = np.cumsum(rng.exponential(1.0 / (0.5 * rate), len(xs)))
    comps2 = Server(be, hbm_budget=64 << 30).run([PredictRequest("train", x, 1, float(t)) for x, t in zip(xs, arr)])
    st2 = latency_stats(comps2)
    st2.update(requests=len(xs), saturation_points_per_s=round(pts / span, 1),
               saturation_requests_per_s=round(rate, 2), poisson_rate_per_s=round(0.5 * rate, 2),
               max_batch=max(c.batch for c in comps))
    res["predict_stream"] = st2
    log(f"serving done: {json.dumps(res)}")
    return res


def variance_leg(ctx, ds, p, xs, npts=64):
    """Posterior variance at npts of the prediction points (batches of 32):
    wall time per point, iterations and the sparse product's share."""
    import torch

    from paper_2411_05869_amd import FP64, MIXED
    res = {}
    for name, prec in (("mixed", MIXED), ("fp64", FP64)):
        K = ctx.assemble(ds, p.theta, prec)
        pts = xs[:npts].contiguous()
        ctx.predict_var(K, p.theta, pts[:32].contiguous())  # warm the work space
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        v, r = ctx.predict_var(K, p.theta, pts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        K.close()
        sp = prof.get("spmm", (0, 0.0))
        res[name] = dict(points=npts, seconds=round(dt, 4), points_per_s=round(npts / dt, 2),
                         iters=r["iters"], max_batch_iters=r["max_batch_iters"], relres=r["relres"],
                         spmm_ms=round(sp[1], 2), spmm_avg_us=round(1e3 * sp[1] / max(sp[0], 1), 1),
                         vector_ms=round(prof.get("var_vector_ops", (0, 0.0))[1], 2),
                         mean_var=float(v.mean()))
        log(f"variance {name}: {res[name]}")
    return res


def mcmc_leg(ctx, n_iter=8):
    """MCMC training (four Metropolis-Hastings blocks and the Gibbs step per
    iteration) on the 100k-point mixture workload, mixed form with SLQ."""
    import numpy as np
    import torch

    from paper_2411_05869_amd.mcmc import Chain
    from workloads import McmcPriors, config2, mcmc_draws, mean_covariates
    p = config2()
    th = p.theta.copy()
    th.a = np.ones_like(th.a)
    W = mean_covariates(p.x)
    z = np.array([0.2, 0.5, -0.4]) @ W + p.y
    dev = torch.device("cuda", 0)
    ds = ctx.dataset(torch.tensor(p.x, device=dev), cell=p.cell)
    pri = McmcPriors(lo=np.zeros(3), hi=np.ones(3), r0_max=np.full(3, 0.5), r_max=np.full(3, 0.2))
    nb = th.a.size
    draws = mcmc_draws(19, n_iter + 1, W.shape[0], 4, 2 * nb * 2, nb)
    ch = Chain(ctx, ds, torch.tensor(z, device=dev), torch.tensor(W, device=dev), th, np.zeros(W.shape[0]),
               np.full(th.a.shape, 0.5), pri)
    ch.step(draws[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [ch.step(dr) for dr in draws[1:]]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ch.close()
    acc = np.sum([r["acc"] for r in recs], axis=0).tolist()
    res = dict(workload=f"{p.name}: n={p.n}, 3 mean coefficients, 16 bumps (64 centre/radius coordinates)",
               iterations=n_iter, seconds=round(dt, 3), iters_per_s=round(n_iter / dt, 3), accepted_per_block=acc,
               loglik_first=recs[0]["loglik"], loglik_last=recs[-1]["loglik"])
    log(f"mcmc: {res}")
    return res


def core_legs(ctx, ds, p, y, xs, opts, reps=2):
    """Same space-time workload with a core kernel (stationary Matern nu = 5/2,
    then the nonstationary core): assemble wall time, one mixed-form step
    (assemble + likelihood + 10k-point prediction) and the prediction alone."""
    import copy

    import torch

    from paper_2411_05869_amd import MIXED
    from workloads import spacetime_core
    res = {}
    alpha = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for name, kind in (("matern52", 1), ("paciorek_nu52", 2)):
        th = copy.copy(p.theta)
        th.core = spacetime_core(kind)
        asm, steps, preds = [], [], []
        r = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            K = ctx.assemble(ds, th, MIXED)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = ctx.loglik(K, y, alpha_out=alpha, **opts)
            pred = ctx.predictor(ds, th, alpha)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ctx.predict(pred, xs, precision=MIXED)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            asm.append(t1 - t0)
            steps.append(t3 - t0)
            preds.append(t3 - t2)
            nnz = K.nnz
            K.close()
            pred.close()
        res[name] = dict(assemble_ms=round(1e3 * min(asm), 3), nnz_per_s=round(nnz / min(asm), 1),
                         step_ms=round(1e3 * min(steps), 2), evals_per_s=round(1 / min(steps), 3),
                         predict_10k_ms=round(1e3 * min(preds), 3), cg_iters=r["cg_iters"],
                         minres_iters=r["minres_iters"], loglik=r["loglik"])
        log(f"core {name}: {res[name]}")
    return res


def assembly_only(p, x, reps):
    """Assembles the workload reps times in each precision (after one warm-up
    call) with the library's per-kernel event timing; prints one JSON line."""
    import torch

    from paper_2411_05869_amd import FP64, MIXED, Context
    ctx = Context()
    ds = ctx.dataset(x, cell=p.cell)
    out = dict(workload=p.name, n=p.n, reps=reps)
    for name, prec in (("mixed", MIXED), ("fp64", FP64)):
        ctx.assemble(ds, p.theta, prec).close()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for i in range(reps):
            K = ctx.assemble(ds, p.theta, prec)
            nnz = K.nnz
            K.close()
            log(f"assembly {i + 1}/{reps} {name} done")
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        prof = ctx.profile_read()
        ctx.profile(False)
        kern = {k: round(v[1] / reps, 4) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
        kms = sum(kern.values())
        vb = 4 if prec == MIXED else 8
        b = nnz * (4 + vb) + (p.n + 1) * 8
        out[name] = dict(nnz=nnz, wall_ms=round(1e3 * wall, 3), kernels_ms=round(kms, 3), kernels=kern,
                         output_bytes=b, frac_of_8tbs=round(b / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lanczos", type=int, default=80, help="Lanczos steps of the timed log det (30 probes)")
    ap.add_argument("--stations", type=int, default=3000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-saturation", type=int, default=128)
    ap.add_argument("--predict-requests", type=int, default=1000)
    ap.add_argument("--no-core", action="store_true")
    ap.add_argument("--no-var", action="store_true")
    ap.add_argument("--no-mcmc", action="store_true")
    ap.add_argument("--var-points", type=int, default=64)
    ap.add_argument("--isolated-steps", type=int, default=2,
                    help="mixed steps with the log det after the solve (per-kernel rooflines without overlap)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device-to-device first (reference dispatch for HBM counters)")
    ap.add_argument("--assembly-only", type=int, default=0, metavar="REPS",
                    help="only assemble the workload REPS times per precision (profiling runs) and print the times")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("STATS_CSV", "BENCH_JSON", "COMMAND"),
                    help="write the kernel-statistics summary from a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="write the SpMV traffic summary from two rocprofv3 --pmc output folders and exit")
    ap.add_argument("--serve-overlap", type=int, default=0, metavar="REQUESTS",
                    help="only queue the first REQUESTS config-4 likelihoods at once on 4 slots (trace runs)")
    ap.add_argument("--summarize-overlap", nargs=3, metavar=("TRACE_CSV", "BENCH_JSON", "COMMAND"),
                    help="write the slots' overlap summary from a rocprofv3 --kernel-trace run and exit")
    ap.add_argument("--cpu-serving", type=int, default=0, metavar="REQUESTS",
                    help="only time the oracle on REQUESTS sampled config-4 requests and 64 config-5 test points")
    args = ap.parse_args()
    if args.cpu_serving:
        cpu_serving(args.cpu_serving)
        return
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_overlap:
        summarize_overlap(*args.summarize_overlap)
        return
    if args.serve_overlap:
        serve_overlap(args.serve_overlap)
        return
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on one GPU; "
              "sharding the rows across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_05869_amd import FP64, MIXED, Context
    from workloads import config3, config5_requests

    p = config3(n_stations=args.stations)
    log(f"workload {p.name}: n={p.n} d={p.d}")
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.empty(CALIB_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = copy_peak_gbs(torch, dev)
    log(f"measured 1 GiB device copy: {copy_gbs:.0f} GB/s (read + write)")
    x = torch.tensor(p.x, device=dev)
    y = torch.tensor(p.y, device=dev)
    if args.assembly_only:
        assembly_only(p, x, args.assembly_only)
        return
    xs_np = config5_requests(1, seed=5, m_lo=10000, m_hi=10000)[0]
    xs = torch.tensor(xs_np, device=dev)
    ctx = Context()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds = ctx.dataset(x, cell=p.cell)
    torch.cuda.synchronize()
    t_bin = time.perf_counter() - t0
    alpha = torch.empty(p.n, dtype=torch.float64, device=dev)
    opts = dict(seed=2411, n_probes=30, n_lanczos=args.lanczos)

    def step(prec, o=None):
        K = ctx.assemble(ds, p.theta, prec)
        r = ctx.loglik(K, y, alpha_out=alpha, **(o or opts))
        pred = ctx.predictor(ds, p.theta, alpha)
        ctx.predict(pred, xs, precision=prec)
        info = dict(nnz=K.nnz, max_row=K.max_row, bytes=K.bytes, layout=K.layout())
        K.close()
        pred.close()
        return r, info

    # Inside the timed steps only the two products are timed with events (each
    # timed launch group adds two events to its stream); the per-kernel
    # breakdown comes from extra steps after them with every group timed.
    timed_names = {MIXED: ["spmv_f32val_f64", "spmm"], FP64: ["spmv_f64", "spmm"]}

    def timed(prec, steps, warmup, o=None, profiled=0):
        for i in range(warmup):
            step(prec, o)
            log(f"warmup {i + 1}/{warmup} prec={prec} done")
        torch.cuda.synchronize()
        ctx.profile(True, only=timed_names[prec])
        t0 = time.perf_counter()
        res = []
        for i in range(steps):
            res.append(step(prec, o))
            log(f"step {i + 1}/{steps} prec={prec}: loglik={res[-1][0]['loglik']:.10g} "
                f"cg_iters={res[-1][0]['cg_iters']}")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        full = None
        if profiled > 0:
            ctx.profile(True)
            for _ in range(profiled):
                step(prec, o)
            full = ctx.profile_read()
        ctx.profile(False)
        return dt, res, prof, full

    def assemble_wall(prec, reps=5):
        # wall time of the whole assemble call (host work and synchronisations
        # included), device idle at the start; median of reps
        ws = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            K = ctx.assemble(ds, p.theta, prec)
            torch.cuda.synchronize()
            ws.append(time.perf_counter() - t0)
            K.close()
        return sorted(ws)[reps // 2]

    n_prof = 2
    dt_m, res_m, prof_m, full_m = timed(MIXED, args.steps, args.warmup, profiled=n_prof)
    dt_d, res_d, prof_d, full_d = timed(FP64, args.fp64_steps, min(args.warmup, 1), profiled=1)
    # the same mixed step with 50 Lanczos steps, for comparison with the converged depth
    o50 = dict(opts, n_lanczos=50)
    dt_50, res_50, _, _ = timed(MIXED, 2, 0, o50)
    # the same mixed step with the log det after the solve on one stream: each
    # kernel then runs alone, and its launch times give its own roofline
    prof_ser, dt_ser = None, None
    if args.isolated_steps > 0:
        ctx.set_concurrency(False)
        dt_ser, _, prof_ser, _ = timed(MIXED, args.isolated_steps, 0)
        ctx.set_concurrency(True)
    asm_wall_m = assemble_wall(MIXED)
    asm_wall_d = assemble_wall(FP64)
    r_m, info_m = res_m[-1]
    r_d, info_d = res_d[-1]
    ms_step = 1e3 * dt_m / args.steps
    evals_m = args.steps / dt_m
    evals_d = args.fp64_steps / dt_d
    asm_ms_m = sum(v[1] for k, v in full_m.items() if k.startswith("asm_") or k == "scan") / n_prof
    asm_ms_d = sum(v[1] for k, v in full_d.items() if k.startswith("asm_") or k == "scan")
    n, nnz = p.n, info_m["nnz"]

    # the main kernels of the timed region: bytes per launch in the stored
    # format (gp_matrix_layout), the plain-CSR figure of the same matrix
    # beside it, and the mean launch time from the library's events
    lo = info_m["layout"]
    models = {"spmv_f32val_f64": (spmv_format_bytes(n, lo, 4), spmv_bytes(n, nnz, 4, 8)),
              "spmm": (spmm_format_bytes(n, lo, 4), spmm_bytes(n, nnz, 4, 32, 8))}

    def roofline(name, prof=None):
        cnt, tot = (prof or prof_m)[name]
        avg_s = tot / cnt / 1e3
        b, bcsr = models[name]
        achieved = b / avg_s / 1e9
        return dict(bound="hbm", kernel=name, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=stored_traffic(name), avg_us=round(avg_s * 1e6, 2),
                    launches=cnt, bytes_per_launch=int(b), bytes_model="stored format (gp_matrix_layout)",
                    effective_plain_csr=dict(bytes_per_launch=int(bcsr), achieved=round(bcsr / avg_s / 1e9, 1),
                                             frac=round(bcsr / avg_s / 1e9 / HBM_PEAK_GBS, 4)))

    present = [k for k in models if k in prof_m]
    dom = max(present, key=lambda k: prof_m[k][1])
    roof = roofline(dom)
    others = {k: roofline(k) for k in present if k != dom}
    isolated = None
    if prof_ser is not None:
        isolated = dict(ms_per_step=round(1e3 * dt_ser / args.isolated_steps, 2),
                        note="log det after the solve on one stream, kernels alone",
                        **{k: roofline(k, prof_ser) for k in models if k in prof_ser})
        # in the timed steps the log det's stream shares the GPU with the solve, so
        # the launch times above include the other stream's work; the same kernel
        # alone, from the steps with the log det after the solve:
        if dom in isolated:
            a = isolated[dom]
            roof["note"] = "timed steps: launch times include the concurrent log-det stream's kernels"
            roof["alone"] = dict(avg_us=a["avg_us"], achieved=a["achieved"], frac=a["frac"],
                                 effective_plain_csr_frac=a["effective_plain_csr"]["frac"],
                                 region="steps with the log det after the solve (roofline_isolated)")
    asm_b = nnz * 8.1
    others["assembly"] = dict(bound="hbm", achieved=round(asm_b / (asm_ms_m / 1e3) / 1e9, 1), peak=HBM_PEAK_GBS,
                              unit="GB/s", frac=round(asm_b / (asm_ms_m / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                              bytes_per_launch=int(asm_b), bytes_model="8.1 B per stored entry (int32 column id, "
                              "float32 value, row pointer and point data)", kernels_ms=round(asm_ms_m, 3),
                              traffic=stored_traffic("assembly"))
    r50 = res_50[-1][0]

    out = dict(metric=METRIC, value=round(evals_m, 4), unit="loglik evals/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 2), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32/f64", data="synthetic",
               config=dict(workload=f"space-time {p.name}: n={n}, d=3, r0=(0.03,0.03,3d), 16x4 bumps, nugget 1e-2; "
                                    f"step = assemble + PCG(rtol 1e-10) + SLQ(30x{args.lanczos}) + predict(10k points)",
                           n=n, nnz=nnz, max_row=info_m["max_row"]),
               nnz_per_s=round(nnz / asm_wall_m, 1), assemble_ms=round(1e3 * asm_wall_m, 3),
               assemble_kernels_ms=round(asm_ms_m, 3),
               fp64=dict(value=round(evals_d, 4), unit="loglik evals/s", ms_per_step=round(1e3 * dt_d / args.fp64_steps, 2),
                         nnz_per_s=round(nnz / asm_wall_d, 1), assemble_ms=round(1e3 * asm_wall_d, 3),
                         assemble_kernels_ms=round(asm_ms_d, 3),
                         loglik=r_d["loglik"], cg_iters=r_d["cg_iters"], vs_exact=vs_exact(r_d, p.name),
                         vs_oracle_slq=vs_oracle_slq(r_d, p.name, opts["seed"], opts["n_probes"],
                                                     opts["n_lanczos"])),
               mixed=dict(loglik=r_m["loglik"], logdet=r_m["logdet"], quad=r_m["quad"], logdet_se=r_m["logdet_se"],
                          cg_iters=r_m["cg_iters"], refreshes=r_m["refreshes"], relres=r_m["relres"],
                          rel_vs_fp64=abs(r_m["loglik"] - r_d["loglik"]) / abs(r_d["loglik"]),
                          vs_exact=vs_exact(r_m, p.name),
                          vs_oracle_slq=vs_oracle_slq(r_m, p.name, opts["seed"], opts["n_probes"], opts["n_lanczos"])),
               mixed_30x50=dict(value=round(2 / dt_50, 4), unit="loglik evals/s", ms_per_step=round(1e3 * dt_50 / 2, 2),
                                logdet=r50["logdet"], logdet_se=r50["logdet_se"], vs_exact=vs_exact(r50, p.name)),
               binning_ms=round(1e3 * t_bin, 2),
               roofline=roof,
               roofline_other=others,
               roofline_isolated=isolated,
               hbm_copy_gbs=round(copy_gbs, 1),
               matrix_layout=lo,
               kernels_ms_per_step={k: round(v[1] / n_prof, 3) for k, v in sorted(full_m.items(),
                                                                                   key=lambda kv: -kv[1][1])},
               kernels_note=f"per-kernel times from {n_prof} mixed steps after the timed ones, every launch group "
                            "timed; inside the timed steps only the two products are",
               paper_context="paper: ~66 s per likelihood (37 s covariance) at N=1,038,723 on 256 A100 (Sec. 5.2)")
    if not args.no_serve:
        out["serving"] = serving_legs(args, ctx, ds, p, alpha)
    if not args.no_core:
        out["core"] = core_legs(ctx, ds, p, y, xs, opts)
    if not args.no_var:
        out["variance"] = variance_leg(ctx, ds, p, xs, args.var_points)
    if not args.no_mcmc:
        out["mcmc"] = mcmc_leg(ctx)
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample) ...")
        cb, (sel, snnz) = cpu_baseline(p)
        out["cpu_baseline"] = cb
        # same sample on the GPU for a like-for-like ratio
        xs_s = torch.tensor(p.x[sel], device=dev)
        ys_s = torch.tensor(p.y[sel], device=dev)
        ds_s = ctx.dataset(xs_s, cell=p.cell)
        a_s = torch.empty(xs_s.shape[0], dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            K = ctx.assemble(ds_s, p.theta, FP64)
            rs = ctx.loglik(K, ys_s, alpha_out=a_s, **opts)
            K.close()
        torch.cuda.synchronize()
        out["cpu_baseline"]["gpu_fp64_same_sample_evals_per_s"] = round(3 / (time.perf_counter() - t0), 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
