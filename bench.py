"""Benchmark of the downsampling hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on): M4
with x -- 100,000,000 float64 points y (three sinusoids + N(0, 0.1) noise +
1% +-50 spikes) on int64 timestamps with gaps uniform in 1..1000, n_out =
4,000 (1,000 bins equidistant in x located by search-sorted).  One step is
one full ts_m4 call: bin edges, the argmin/argmax scan over y, the per-bin
merge/selection and the compaction.  Inputs are resident in HBM before the
timed region.

Printed: one JSON line with the input throughput (GB/s of y, the bytes the
algorithm must read), the roofline of the dominant kernel (the scan; its
duration measured live with HIP events that the library's launch stamps with
the dispatch's own start and end times), and the CPU oracle timed on the host as a baseline.  Unless
--no-extra: the other configurations (MinMax 1e6, MinMaxLTTB 5e8, plain
LTTB 1e8), batched vs plain (512 series) and served vs plain (zoom requests
over 64 resident series).  The oracle runs only in the CPU-baseline leg
(the baseline timing and the parity samples); --no-cpu-baseline skips it.

    python bench.py [--steps K] [--warmup W] [--workload m4x|minmax|minmaxlttb]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "m4x": dict(algo="m4", n=100_000_000, n_out=4000, desc="M4 with int64 x, float64 y (3 sinusoids + "
                "noise + 1% spikes), N=1e8, n_out=4000, bins equidistant in x via search-sorted"),
    "minmax": dict(algo="minmax", n=1_000_000, n_out=1000, desc="MinMax no x, float32 random walk, "
                   "N=1e6, n_out=1000"),
    "minmaxlttb": dict(algo="minmaxlttb", n=500_000_000, n_out=2000, desc="MinMaxLTTB no x, float32 "
                       "random walk with 5% constant runs, N=5e8, n_out=2000, minmax_ratio=4"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(name):
    import synthetic as S
    w = WORKLOADS[name]
    if name == "m4x":
        x, y = S.m4_with_x(w["n"], seed=1)
        return x, y
    if name == "minmax":
        return None, S.walk(w["n"], np.float32, seed=0)
    y = S.walk(w["n"], np.float32, seed=2)
    S.tie_runs(y, 0.05, seed=2)
    return None, y


def scan_source_hash():
    h = hashlib.sha256()
    for f in ("scan.hip", "scan_core.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2307_05389_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current scan source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    e = d.get(workload, {})
    if e.get("kernel") != kernel or e.get("source_hash") != scan_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_share():
    """Host cores this process may use, capped at 16 (the host CPU share of
    one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _median_runs(fn, budget_s, max_runs=50):
    times, res = [], None
    t_start = time.perf_counter()
    while (len(times) < 3 or time.perf_counter() - t_start < budget_s) and len(times) < max_runs:
        t0 = time.perf_counter()
        res = fn()
        times.append(time.perf_counter() - t0)
    return float(np.median(times)), len(times), res


def cpu_baseline(name, x, y, w, budget_s=8.0):
    """The oracle on the host: single-threaded, and (MinMax / M4) with its bins
    split over every core of the host share (the paper's parallel=True mode;
    the same per-bin loop, identical output)."""
    import oracle
    if w["algo"] == "minmaxlttb":
        serial = lambda: oracle.minmaxlttb(y, w["n_out"], 4, x=x)
    else:
        serial = lambda: getattr(oracle, w["algo"])(y, w["n_out"], x=x)
    med1, runs1, res = _median_runs(serial, budget_s)
    single = {"value": round(y.nbytes / med1 / 1e9, 3), "unit": "GB/s", "cores": 1,
              "median_ms": round(med1 * 1e3, 2), "runs": runs1}
    out = {"value": single["value"], "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"the full workload ({len(y):,} points), {runs1} single-thread runs, median "
                     f"{med1 * 1e3:.1f} ms", "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
           "single_core": single}
    if w["algo"] in ("minmax", "m4"):
        T = cpu_share()
        medT, runsT, resT = _median_runs(
            lambda: oracle.binned_parallel(w["algo"], y, w["n_out"], x=x, threads=T), budget_s / 2)
        if not np.array_equal(resT, res):
            raise RuntimeError("bin-parallel oracle differs from the serial oracle")
        out.update({"value": round(y.nbytes / medT / 1e9, 3), "cores": T,
                    "sample": f"the full workload ({len(y):,} points), bins split over {T} threads, {runsT} runs, "
                              f"median {medT * 1e3:.1f} ms; single thread: {runs1} runs, median "
                              f"{med1 * 1e3:.1f} ms"})
    return out, res


def time_calls(fn, st, reps, sync_reps=None):
    """Mean ms per call over `reps` calls enqueued back to back between two
    HIP events (the throughput a stream of calls sees, as in the headline
    steps), and the median ms of calls timed one at a time with a host sync
    in between (launch latency included)."""
    import torch
    # the GPU idles while the host prepares each case (inputs, oracle
    # checks): calls for ~100 ms first bring it back to its steady clock
    t0 = time.perf_counter()
    k = 0
    while k < 3 or (time.perf_counter() - t0 < 0.1 and k < 2000):
        fn()
        k += 1
        if k % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        fn()
    b.record(st)
    b.synchronize()
    mean_ms = a.elapsed_time(b) / reps
    ts = []
    for _ in range(sync_reps or max(3, reps // 4)):
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return mean_ms, float(np.median(ts))


def bench_batched(seed=3, n_series=512, reps=10, check_oracle=True, tuning=None, plain=True):
    """Batched vs plain on the mixed batch: 512 series, lengths log-uniform in
    1e4..2e7, dtypes f32/f16/i16/u8, MinMax / M4, n_out 500..4000.  With
    check_oracle (part of the CPU-baseline leg), a sample of tasks is also
    recomputed by the oracle on the host."""
    import torch
    import paper_2307_05389_amd as tsds
    import synthetic as S
    specs = S.batch_specs(n_series, seed=seed)
    log(f"[bench] batched: generating {n_series} series on the GPU")
    ys = [S.device_walk_cast(s["n"], s["dtype"], s["seed"]) for s in specs]
    total_bytes = sum(y.numel() * y.element_size() for y in ys)
    tasks = [dict(algo=s["algo"], y=y, n_out=s["n_out"]) for s, y in zip(specs, ys)]
    b = tsds.Batch(tasks)
    if tuning is None:
        tune = b.autotune()
    else:   # a fixed tuning (profiling runs: no autotune candidates in the trace)
        b.set_tuning(*tuning)
        tune = b.tuning()
    group_bytes = {}
    for sp, y in zip(specs, ys):
        k = str(sp["dtype"])
        group_bytes[k] = group_bytes.get(k, 0) + y.numel() * y.element_size()
    st = torch.cuda.current_stream()
    b.run(graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        b.run(graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / reps
    batched = [r.clone() for r in b.results()]
    if not plain:
        b.close()
        return {"batched_ms": round(t_batch, 4), "batched_GBps": round(total_bytes / t_batch / 1e6, 1),
                "group_bytes": group_bytes, "replays": reps + 1,
                "tuning": {"chunk_bytes": tune[0], "small_bin": tune[1], "grid_blocks": tune[2]}}
    # plain: one single-series call per task on one stream (own outputs, one
    # shared workspace), eager and replayed from a torch-captured graph
    outs = [torch.empty(s["n_out"], dtype=torch.int64, device=y.device) for s, y in zip(specs, ys)]
    cnts = torch.zeros(len(specs), dtype=torch.int64, device=ys[0].device)
    need = max(tsds.workspace_bytes(s["algo"], y, s["n_out"]) for s, y in zip(specs, ys))
    ws = torch.empty(need, dtype=torch.uint8, device=ys[0].device)

    def plain(stream):
        for i, (s, y) in enumerate(zip(specs, ys)):
            tsds.downsample_into(s["algo"], y, s["n_out"], outs[i], cnts[i:i + 1], workspace=ws, stream=stream)

    plain(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(reps):
        plain(st)
    e1.record(st)
    torch.cuda.synchronize()
    t_plain_eager = e0.elapsed_time(e1) / reps
    wall_plain = (time.perf_counter() - t0) * 1e3 / reps
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        plain(torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        g.replay()
    e1.record(st)
    torch.cuda.synchronize()
    t_plain_graph = e0.elapsed_time(e1) / reps
    cnt_h = cnts.cpu().tolist()
    identical = all(torch.equal(batched[i], outs[i][: cnt_h[i]]) for i in range(len(specs)))
    # oracle on a sample of tasks
    ok = None
    if check_oracle:
        import oracle
        rng = np.random.default_rng(0)
        sample = sorted(rng.choice(len(specs), 6, replace=False).tolist())
        ok = True
        for i in sample:
            s = specs[i]
            yh = ys[i].cpu().numpy()
            exp = getattr(oracle, s["algo"])(yh, s["n_out"])
            ok &= bool(np.array_equal(batched[i].cpu().numpy(), exp))
    b.close()
    return {
        "workload": "512 series, lengths log-uniform 1e4..2e7 (sum %d points, %.2f GB), dtypes f32/f16/i16/u8, "
                    "MinMax / M4 alternating, n_out 500..4000" % (sum(s["n"] for s in specs), total_bytes / 1e9),
        "batched_ms": round(t_batch, 4), "batched_GBps": round(total_bytes / t_batch / 1e6, 1),
        "plain_eager_ms": round(t_plain_eager, 4), "plain_eager_wall_ms": round(wall_plain, 4),
        "plain_graph_ms": round(t_plain_graph, 4),
        "speedup_vs_plain_eager": round(t_plain_eager / t_batch, 2),
        "speedup_vs_plain_graph": round(t_plain_graph / t_batch, 2),
        "identical_to_plain": identical, "oracle_sample_bit_exact": ok, "group_bytes": group_bytes,
        "tuning": {"chunk_bytes": tune[0], "small_bin": tune[1], "grid_blocks": tune[2]},
    }


def bench_served(full=False, n_series=64, n_points=200_000_000, check_oracle=True):
    """Serving: 64 resident series of 2e8 float32 points with int64 timestamps
    (gaps 1..100); Poisson arrivals of zoom/pan requests (window width
    log-uniform 0.1%..100% of the range, n_out 800..4000, MinMaxLTTB ratio 4);
    latency from the scheduled arrival to the indices in host memory."""
    import torch
    import paper_2307_05389_amd as tsds
    import synthetic as S
    log(f"[bench] served: generating {n_series} x {n_points:,} points on the GPU")
    series = []
    for s in range(n_series):
        x = S.device_timestamps(n_points, 10_000 + s, gap_max=100)
        y = S.device_walk(n_points, 20_000 + s)
        series.append((x, y))
    torch.cuda.synchronize()
    x_first = [int(x[0].item()) for x, _ in series]
    x_last = [int(x[-1].item()) for x, _ in series]
    resident_gb = sum(x.numel() * 8 + y.numel() * 4 for x, y in series) / 1e9
    qps_list = [100.0, 1000.0, 5000.0, 10000.0, 20000.0] if full else [1000.0, 5000.0, 10000.0, 20000.0]
    n_req, n_warm = 10000, 500

    def run(srv, qps, seed):
        reqs = S.zoom_requests(n_req + n_warm, n_series, x_first, x_last, seed=seed, qps=qps)
        t0 = srv.now() + 0.05
        sched = {}
        done = {}
        k = 0
        while len(done) < len(reqs):
            now = srv.now()
            while k < len(reqs) and now >= t0 + reqs[k]["t"]:
                q = reqs[k]
                rid = srv.submit(q["series"], q["xa"], q["xb"], q["n_out"])
                sched[rid] = (t0 + q["t"], k)
                k += 1
                now = srv.now()
            for r in srv.poll():
                done[r["id"]] = r
            if k < len(reqs):
                wait = t0 + reqs[k]["t"] - srv.now()
                if wait > 2e-4:
                    time.sleep(min(wait - 1e-4, 1e-3))
            elif len(done) < len(reqs):
                time.sleep(2e-4)
        lat, slat, pts, bs = [], [], 0, []
        first, last = None, 0.0
        by_k = {}
        for rid, r in done.items():
            ta, kk = sched[rid]
            by_k[kk] = r
            if kk < n_warm:
                continue
            lat.append(r["t_done"] - ta)
            slat.append(r["t_done"] - r["t_submit"])
            pts += r["i1"] - r["i0"]
            bs.append(r["batch_size"])
            first = ta if first is None else min(first, ta)
            last = max(last, r["t_done"])
        lat = np.array(lat) * 1e3
        slat = np.array(slat) * 1e3
        return {"qps": qps, "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "server_p50_ms": round(float(np.percentile(slat, 50)), 3),
                "server_p99_ms": round(float(np.percentile(slat, 99)), 3),
                "points_per_s": round(pts / (last - first), 1),
                "mean_batch": round(float(np.mean(bs)), 2)}, by_k, reqs

    p99_bound_ms = 1.0
    out = {"workload": f"{n_series} resident series x {n_points:,} float32 points + int64 timestamps "
                       f"({resident_gb:.1f} GB), MinMaxLTTB ratio 4, n_out 800..4000, {n_req} requests "
                       f"(+{n_warm} warm-up) per rate, the same request trace for both modes",
           "served": [], "plain": []}
    # both modes on the same trace per rate; served and plain alternate so
    # that neither sees a systematically warmer GPU
    srv = tsds.Server(series, n_streams=4, max_batch=32, max_nout=4000, minmax_ratio=4)
    plain = tsds.Server(series, plain=True, max_nout=4000, minmax_ratio=4)
    served_first = None
    identical = True
    for i, qps in enumerate(qps_list):
        log(f"[bench] served at {qps} QPS")
        stats, by_k, reqs = run(srv, qps, seed=4 + i)
        out["served"].append(stats)
        log(f"[bench] plain FIFO at {qps} QPS")
        pstats, pk, _ = run(plain, qps, seed=4 + i)
        out["plain"].append(pstats)
        identical &= all(np.array_equal(by_k[k]["indices"], pk[k]["indices"]) for k in by_k)
        if i == 0:
            served_first = (by_k, reqs)
    srv.close()
    plain.close()
    by_k, reqs = served_first
    out["identical_served_vs_plain"] = bool(identical)
    out["p99_bound_ms"] = p99_bound_ms
    for mode in ("served", "plain"):
        ok = [r["qps"] for r in out[mode] if r["p99_ms"] <= p99_bound_ms]
        out[f"{mode}_max_qps_p99_within_bound"] = max(ok) if ok else None
    # oracle on a few requests (window copied to the host; CPU-baseline leg)
    ok = None
    if check_oracle:
        import oracle
        ok = True
        for k in (n_warm, n_warm + 1, n_warm + 2):
            r, q = by_k[k], reqs[k]
            x, y = series[q["series"]]
            xh = x[r["i0"]: r["i1"]].cpu().numpy()
            yh = y[r["i0"]: r["i1"]].cpu().numpy()
            exp = r["i0"] + oracle.minmaxlttb(yh, q["n_out"], 4, x=xh)
            ok &= bool(np.array_equal(exp, r["indices"]))
    out["oracle_sample_bit_exact"] = ok
    del series
    torch.cuda.empty_cache()
    return out


def _exact_bucket_sums(v, starts):
    """Exact sums and exact sums of |v| of float32 values v over the buckets
    [starts[k], starts[k+1]), as Python integers times 2^-149: every float32 is
    an integer multiple of 2^-149, so the sums are grouped by exponent (the
    per-exponent integer sums stay below 2^53 and are exact in float64) and
    combined in Python integers."""
    bits = np.ascontiguousarray(v, np.float32).view(np.uint32)
    e = ((bits >> 23) & 0xFF).astype(np.int64)
    mant = (bits & 0x7FFFFF).astype(np.int64) + np.where(e > 0, 1 << 23, 0)
    shift = np.maximum(e - 1, 0)                    # value = mant * 2^(shift - 149)
    sgn = np.where(bits >> 31, -1, 1)
    bucket = np.repeat(np.arange(len(starts) - 1), np.diff(starts))
    key = bucket * 256 + shift
    sums = np.bincount(key, weights=(sgn * mant).astype(np.float64), minlength=256 * (len(starts) - 1))
    abss = np.bincount(key, weights=mant.astype(np.float64), minlength=256 * (len(starts) - 1))
    out, out_abs = [], []
    for k in range(len(starts) - 1):
        row, arow = sums[256 * k: 256 * k + 256], abss[256 * k: 256 * k + 256]
        nz = np.nonzero(arow)[0]
        out.append(sum(int(row[j]) << int(j) for j in nz))
        out_abs.append(sum(int(arow[j]) << int(j) for j in nz))
    return out, out_abs


def lttb_mean_error(tsds, yd, y, n_out, sel=None):
    """Largest error of the GPU's LTTB bucket centres (the FP64 means of the
    next bucket) against the exact rational means, relative to the bucket's
    mean |value| (= |mean| when the values share a sign).  float32 y, no x:
    X is the index, whose means are exact (reported too)."""
    from fractions import Fraction
    import torch
    seld = None if sel is None else torch.from_numpy(sel).to(yd.device)
    cx, cy = tsds.lttb_centres(yd, n_out, sel=seld)
    cx, cy = cx.cpu().numpy(), cy.cpu().numpy()
    idx = np.arange(len(y), dtype=np.int64) if sel is None else sel
    m, nb = len(idx), n_out - 2
    b = np.array([1 + (k * (m - 2)) // nb for k in range(nb + 1)], np.int64)
    vals = y if sel is None else y[sel]
    sums, abss = _exact_bucket_sums(vals[b[1]: b[nb]], b[1: nb + 1] - b[1])
    isum = np.add.reduceat(idx[b[1]: b[nb]], (b[1: nb] - b[1]))
    worst_y = worst_x = 0.0
    for k in range(nb - 1):
        cnt = int(b[k + 2] - b[k + 1])
        if abss[k]:
            err = abs(Fraction(float(cy[k])) - Fraction(sums[k], cnt << 149)) / Fraction(abss[k], cnt << 149)
            worst_y = max(worst_y, float(err))
        worst_x = max(worst_x, float(abs(Fraction(float(cx[k])) - Fraction(int(isum[k]), cnt)) / Fraction(int(isum[k]), cnt)))
    return max(worst_x, worst_y), worst_y


def bench_configs(reps_small=200, reps_big=20, check_oracle=True, only=None):
    """The other configurations: MinMax at 1e6 (latency-bound), MinMaxLTTB at
    5e8 (preselection scan + candidate LTTB) and plain LTTB at 1e8 (the
    paper's Table 1 LTTB row, one workgroup walking the buckets), each timed
    with HIP events around the whole call and, with check_oracle (part of
    the CPU-baseline leg), checked against the oracle on the host."""
    import torch
    import paper_2307_05389_amd as tsds
    from paper_2307_05389_amd import _lib as L
    import synthetic as S
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    out = []

    sync_ms = {}

    def timed(fn, reps):
        ms, ms_sync = time_calls(fn, st, reps)
        sync_ms["last"] = ms_sync
        return ms

    cases = [
        ("minmax", "MinMax no x, float32 random walk, N=1e6, n_out=1000", lambda: S.walk(1_000_000, np.float32, seed=0),
         1000, reps_small, "tsdownsample MinMax float32 N=1e6 parallel: 0.23 ms (17.4 GB/s)"),
        ("minmaxlttb", "MinMaxLTTB no x, float32 random walk with 5% constant runs, N=5e8, n_out=2000, ratio 4",
         lambda: S.tie_runs(S.walk(500_000_000, np.float32, seed=2), 0.05, seed=2), 2000, reps_big,
         "tsdownsample MinMaxLTTB float32 N=1e9 parallel: 89.17 ms (44.9 GB/s); N=1e8: 9.56 ms"),
        ("lttb", "plain LTTB no x, float32 random walk, N=1e8, n_out=2000", lambda: S.walk(100_000_000, np.float32, seed=5),
         2000, reps_big, "tsdownsample LTTB float32 N=1e8 (sequential only): 173.72 ms (2.3 GB/s)"),
    ]
    want = lambda name: only is None or name in only
    for algo, desc, gen, n_out, reps, paper in cases:
        if not want(algo):
            continue
        log(f"[bench] config {algo}: generating")
        y = gen()
        yd = torch.from_numpy(y).to(dev)
        o = torch.empty(n_out, dtype=torch.int64, device=dev)
        c = torch.zeros(1, dtype=torch.int64, device=dev)
        need = tsds.workspace_bytes(algo, yd, n_out, minmax_ratio=4)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        fn = lambda: tsds.downsample_into(algo, yd, n_out, o, c, minmax_ratio=4, workspace=ws, stream=st)
        ms = timed(fn, reps)
        got = o[: int(c.item())].cpu().numpy()
        parity = None
        if check_oracle:
            import oracle
            ref = oracle.minmaxlttb(y, n_out, 4) if algo == "minmaxlttb" else getattr(oracle, algo)(y, n_out)
            parity = "bit-exact" if np.array_equal(got, ref) else "MISMATCH"
        line = {"algo": algo, "workload": desc, "n": int(y.size), "n_out": n_out, "ms": round(ms, 4),
                "ms_single_call": round(sync_ms["last"], 4),
                "GBps": round(y.nbytes / ms / 1e6, 1), "points_per_s": round(y.size / ms * 1e3, 1),
                "frac_of_hbm_peak": round(y.nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                "parity_vs_oracle": parity,
                "paper_context": paper + "; 32-thread Xeon E5-2650 v2, other hardware"}
        if algo in ("lttb", "minmaxlttb"):
            sel = None
            if algo == "minmaxlttb":   # the candidates: first point, interior MinMax, last point
                pre = tsds.minmax(yd[1:-1], n_out * 4).cpu().numpy() + 1
                sel = np.concatenate([[0], pre, [y.size - 1]]).astype(np.int64)
            err, err_y = lttb_mean_error(tsds, yd, y, n_out, sel)
            line["max_mean_rel_err"] = err
            line["mean_err_reference"] = "exact rational bucket means; error relative to the bucket's mean |value|"
            # a walk identical to the oracle's uses no near-tie acceptance
            line["near_ties"] = 0 if parity == "bit-exact" else None
        out.append(line)
        if algo == "minmaxlttb":
            # the MinMax variant of the same 5e8-point series (n_out 2000: 1000 bins)
            fn = lambda: tsds.downsample_into("minmax", yd, 2000, o, c, workspace=ws2, stream=st)
            ws2 = torch.empty(max(tsds.workspace_bytes("minmax", yd, 2000), 256), dtype=torch.uint8, device=dev)
            ms = timed(fn, reps * 2)
            got = o[: int(c.item())].cpu().numpy()
            parity = None
            if check_oracle:
                import oracle
                ref = oracle.binned_parallel("minmax", y, 2000, threads=cpu_share())
                parity = "bit-exact" if np.array_equal(got, ref) else "MISMATCH"
            out.append({"algo": "minmax", "workload": "MinMax no x, float32 random walk with 5% constant runs, "
                        "N=5e8, n_out=2000", "n": int(y.size), "n_out": 2000, "ms": round(ms, 4),
                        "ms_single_call": round(sync_ms["last"], 4),
                        "GBps": round(y.nbytes / ms / 1e6, 1), "points_per_s": round(y.size / ms * 1e3, 1),
                        "frac_of_hbm_peak": round(y.nbytes / ms / 1e6 / HBM_PEAK_GBS, 4),
                        "kernel": L.scan_config(yd.dtype, y.size, 1000)[2], "parity_vs_oracle": parity,
                        "paper_context": "tsdownsample MinMax float32 N=1e9 parallel: 88.75 ms (45.1 GB/s); "
                                         "32-thread Xeon E5-2650 v2, other hardware"})
            log(f"[bench] config minmax 5e8: {ms:.3f} ms")
            del ws2
        log(f"[bench] config {algo}: {ms:.3f} ms")
        del yd, ws, y
        torch.cuda.empty_cache()

    # EveryNth over 1e8 points (reads no data: a launch plus n_out index writes)
    # and the fused gather of an M4 selection's (x, y) for drawing.
    if not (want("everynth") or want("m4+gather") or want("nan_m4")):
        return out
    import ctypes
    sp = ctypes.c_void_p(st.cuda_stream)
    if want("everynth"):
        out.append(_config_everynth(tsds, L, st, timed, reps_small, check_oracle))
    if not (want("m4+gather") or want("nan_m4")):
        return out
    out += _config_m4_gather_nan(tsds, L, S, dev, st, sp, timed, reps_big, check_oracle)
    return out


def _config_everynth(tsds, L, st, timed, reps_small, check_oracle):
    import ctypes
    import torch
    dev = torch.device("cuda:0")
    log("[bench] config everynth")
    n = 100_000_000
    yd = torch.zeros(n, dtype=torch.float32, device=dev)
    o = torch.empty(2000, dtype=torch.int64, device=dev)
    c = torch.zeros(1, dtype=torch.int64, device=dev)
    s = L.series(yd)
    sp = ctypes.c_void_p(st.cuda_stream)
    ms = timed(lambda: L.check(L.lib().ts_everynth(ctypes.byref(s), 2000, L._ptr(o), L._ptr(c), sp)), reps_small)
    parity = None
    if check_oracle:
        import oracle
        parity = "bit-exact" if np.array_equal(o[: int(c.item())].cpu().numpy(), oracle.everynth(n, 2000)) \
            else "MISMATCH"
    log(f"[bench] config everynth: {ms:.4f} ms")
    del yd
    return {"algo": "everynth", "workload": "EveryNth, N=1e8, n_out=2000", "n": n, "n_out": 2000,
            "ms": round(ms, 4), "parity_vs_oracle": parity,
            "paper_context": "tsdownsample EveryNth: about 0.02 ms at every size; 32-thread Xeon E5-2650 v2, "
                             "other hardware"}


def _config_m4_gather_nan(tsds, L, S, dev, st, sp, timed, reps_big, check_oracle):
    import ctypes
    import torch
    out = []
    log("[bench] config m4+gather")
    n = 100_000_000
    yd = S.device_walk(n, seed=1, device=dev, dtype=torch.float64)
    xd = S.device_timestamps(n, seed=1, device=dev)
    o = torch.empty(4000, dtype=torch.int64, device=dev)
    c = torch.zeros(1, dtype=torch.int64, device=dev)
    xs = torch.empty(4000, dtype=torch.int64, device=dev)
    ys = torch.empty(4000, dtype=torch.float64, device=dev)
    need = tsds.workspace_bytes("m4", yd, 4000, x=xd)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    s = L.series(yd, xd)

    def m4_gather():
        tsds.downsample_into("m4", yd, 4000, o, c, x=xd, workspace=ws, stream=st)
        L.check(L.lib().ts_gather(ctypes.byref(s), L._ptr(o), L._ptr(c), 4000, L._ptr(xs), L._ptr(ys), sp))
    ms = timed(m4_gather, reps_big * 5)
    ms_m4 = timed(lambda: tsds.downsample_into("m4", yd, 4000, o, c, x=xd, workspace=ws, stream=st), reps_big * 5)
    m4_gather()
    m = int(c.item())
    ok = bool(torch.equal(xs[:m], xd[o[:m]]) and torch.equal(ys[:m], yd[o[:m]]))
    out.append({"algo": "m4+gather", "workload": "M4 with int64 x, float64 random walk, N=1e8, n_out=4000, "
                "then the gather of the selected (x, y)", "n": n, "n_out": 4000, "ms": round(ms, 4),
                "ms_m4_alone": round(ms_m4, 4), "gather_values_match_indexing": ok})
    log(f"[bench] config m4+gather: {ms:.4f} ms (m4 alone {ms_m4:.4f} ms)")

    # NaN-aware M4 on the same series with 1% of y set to NaN.
    log("[bench] config nan_m4")
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    yd[torch.rand(n, device=dev, generator=g) < 0.01] = float("nan")
    need = tsds.workspace_bytes("nan_m4", yd, 4000, x=xd)
    wsn = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    fn = lambda: tsds.downsample_into("nan_m4", yd, 4000, o, c, x=xd, workspace=wsn, stream=st)
    ms = timed(fn, reps_big * 5)
    parity = None
    if check_oracle:
        import oracle
        got = o[: int(c.item())].cpu().numpy()
        parity = "bit-exact" if np.array_equal(got, oracle.nan_m4(yd.cpu().numpy(), 4000, x=xd.cpu().numpy())) \
            else "MISMATCH"
    out.append({"algo": "nan_m4", "workload": "NaN-aware M4 with int64 x, float64 random walk with 1% NaN, N=1e8, "
                "n_out=4000", "n": n, "n_out": 4000, "ms": round(ms, 4), "GBps": round(n * 8 / ms / 1e6, 1),
                "frac_of_hbm_peak": round(n * 8 / ms / 1e6 / HBM_PEAK_GBS, 4), "parity_vs_oracle": parity})
    log(f"[bench] config nan_m4: {ms:.4f} ms")
    del yd, xd, ws, wsn
    torch.cuda.empty_cache()
    return out


def bench_dtypes(reps=40, check_oracle=True):
    """MinMax and M4 over 1 GB of uniform random values in the narrow dtypes
    of the paper's Table 1 (u8: 1e9 points; i16 and f16: 5e8 points), no x,
    with 1,000 and 100,000 bins; timed with HIP events around the whole call
    and (CPU-baseline leg) checked against the oracle."""
    import torch
    import paper_2307_05389_amd as tsds
    from paper_2307_05389_amd import _lib as L
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(12)
    lines = []
    for name, n in (("uint8", 1_000_000_000), ("int16", 500_000_000), ("float16", 500_000_000)):
        log(f"[bench] dtypes: {name} x {n:,}")
        if name == "float16":
            yd = torch.randn(n, generator=g, device=dev, dtype=torch.float32).to(torch.float16)
        else:
            tdt = getattr(torch, name)
            info = torch.iinfo(tdt)
            yd = torch.randint(info.min, info.max + 1, (n,), generator=g, device=dev, dtype=torch.int64).to(tdt)
        yh = yd.cpu().numpy() if check_oracle else None
        for algo in ("minmax", "m4"):
            for bins in (1000, 100_000):
                n_out = bins * (2 if algo == "minmax" else 4)
                o = torch.empty(n_out, dtype=torch.int64, device=dev)
                c = torch.zeros(1, dtype=torch.int64, device=dev)
                ws = torch.empty(max(tsds.workspace_bytes(algo, yd, n_out), 256), dtype=torch.uint8, device=dev)
                fn = lambda: tsds.downsample_into(algo, yd, n_out, o, c, workspace=ws, stream=st)
                ms, ms_sync = time_calls(fn, st, reps)
                parity = None
                if check_oracle:
                    import oracle
                    ref = oracle.binned_parallel(algo, yh, n_out, threads=cpu_share())
                    parity = "bit-exact" if np.array_equal(o[: int(c.item())].cpu().numpy(), ref) else "MISMATCH"
                nbytes = n * yd.element_size()
                lines.append({"algo": algo, "dtype": name, "n": n, "n_out": n_out, "bins": bins, "ms": round(ms, 4),
                              "ms_single_call": round(ms_sync, 4),
                              "GBps": round(nbytes / ms / 1e6, 1), "frac_of_hbm_peak": round(nbytes / ms / 1e6 /
                                                                                          HBM_PEAK_GBS, 4),
                              "kernel": L.scan_config(yd.dtype, n, bins)[2], "parity_vs_oracle": parity})
                log(f"[bench] dtypes: {algo} {name} {bins} bins: {ms:.4f} ms ({nbytes / ms / 1e6:.0f} GB/s)")
                del ws
        del yd, yh
        torch.cuda.empty_cache()
    return {"workload": "uniform random values (the paper's Table 1 input), no x, 1 GB per series",
            "lines": lines}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the GPU reaches its steady clock after a few dozen 0.14 ms steps: the
    # default warm-up runs 100 of them (14 ms), then 100 are timed
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="m4x", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other configurations and the batched and served comparisons")
    ap.add_argument("--serve-full", action="store_true", help="served sweep at 100..20000 QPS, 10000 requests each")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of y (for counter calibration)")
    ap.add_argument("--batch-tuning", default=None,
                    help="chunk_bytes,small_bin,grid_blocks for the batched leg instead of autotuning, and no "
                         "plain comparison (for kernel traces of the batched replays alone)")
    ap.add_argument("--configs", default=None,
                    help="comma list of the configs leg's entries to run (minmax, minmaxlttb, lttb, everynth, "
                         "m4+gather, nan_m4; default all)")
    ap.add_argument("--legs", default="configs,dtypes,batched,served",
                    help="comma list of the extra legs to run after the headline: configs, dtypes, batched, served")
    args = ap.parse_args()
    legs = set(x for x in args.legs.split(",") if x)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a multi-GPU run would shard the series, or one series by index range, over the GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_05389_amd as tsds
    from paper_2307_05389_amd import _lib as L

    w = WORKLOADS[args.workload]
    log(f"[bench] generating {args.workload} ({w['n']:,} points)")
    dev = torch.device("cuda:0")
    if args.workload == "m4x":
        # generated on the GPU; host copies (for the oracle) are taken after
        # the timed region
        import synthetic as S
        xd, yd = S.device_m4_with_x(w["n"], seed=1, device=dev)
        x = y = None
    else:
        x, y = make_inputs(args.workload)
        yd = torch.from_numpy(y).to(dev)
        xd = torch.from_numpy(x).to(dev) if x is not None else None
    y_nbytes = yd.numel() * yd.element_size()
    out = torch.empty(w["n_out"], dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    st = torch.cuda.current_stream(dev)
    need = tsds.workspace_bytes(w["algo"], yd, w["n_out"], x=xd, minmax_ratio=4)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        tsds.downsample_into(w["algo"], yd, w["n_out"], out, cnt, x=xd, minmax_ratio=4, workspace=ws,
                             stream=st)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_calibration:
        tmp = torch.empty_like(yd)
        tmp.copy_(yd)
        torch.cuda.synchronize()
        del tmp

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in ev:  # torch creates the HIP events lazily, on first record
        a.record(st)
        b.record(st)
    lib = L.lib()
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        L.check(lib.ts_profile_scan_events(ev[k][0].cuda_event, ev[k][1].cuda_event))
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.check(lib.ts_profile_scan_events(None, None))
    ms_step = (t1 - t0) * 1e3 / args.steps
    scan_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    gbytes = y_nbytes / 1e9
    value = gbytes / (ms_step / 1e3)
    achieved = gbytes / (scan_ms / 1e3)
    got = out[: int(cnt.item())].cpu().numpy()
    log(f"[bench] {ms_step:.4f} ms/step, scan kernel {scan_ms:.4f} ms ({achieved:.0f} GB/s)")
    if y is None:
        x = xd.cpu().numpy() if xd is not None else None
        y = yd.cpu().numpy()

    nb = {"m4": w["n_out"] // 4, "minmax": w["n_out"] // 2, "minmaxlttb": w["n_out"] * 4 // 2}[w["algo"]]
    variant, chunk_bytes, kernel = L.scan_config(yd.dtype, w["n"] if w["algo"] != "minmaxlttb" else w["n"] - 2,
                                                 nb, None if xd is None else xd.dtype)
    traffic = load_traffic(kernel, args.workload)
    res = {
        "metric": "MinMax/M4 input GB/s vs HBM peak",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}[y.dtype],
        "data": "synthetic",
        "config": {"workload": w["desc"], "n": w["n"], "n_out": w["n_out"], "algo": w["algo"],
                   "bytes_per_step": int(y.nbytes), "parallelism": "single GPU"},
        "points_per_s": round(w["n"] / (ms_step / 1e3), 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel, "kernel_ms": round(scan_ms, 5), "chunk_bytes": chunk_bytes},
        "paper_context": "tsdownsample M4 float64 N=1e8 no x, 32-thread Xeon E5-2650 v2: 18.06 ms "
                         "(44.3 GB/s); different hardware and workload",
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on host)")
        cb, ref = cpu_baseline(args.workload, x, y, w)
        res["cpu_baseline"] = cb
        res["parity_vs_oracle"] = "bit-exact" if np.array_equal(ref, got) else "MISMATCH"
    if not args.no_extra:
        del yd, xd, ws
        torch.cuda.empty_cache()
        chk = not args.no_cpu_baseline
        if "configs" in legs:
            only = None if args.configs is None else set(args.configs.split(","))
            res["other_configs"] = bench_configs(check_oracle=chk, only=only)
        if "dtypes" in legs:
            res["narrow_dtypes"] = bench_dtypes(check_oracle=chk)
            torch.cuda.empty_cache()
        if "batched" in legs:
            bt = None if args.batch_tuning is None else tuple(int(v) for v in args.batch_tuning.split(","))
            res["batched"] = bench_batched(check_oracle=chk and bt is None, tuning=bt, plain=bt is None)
            torch.cuda.empty_cache()
        if "served" in legs:
            res["served"] = bench_served(full=args.serve_full, check_oracle=chk)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
