"""Benchmark of the sparse stress model's hot path on one MI355X.

One step = the whole path over one synthetic graph already resident in HBM:
max/min pivot selection, BFS from every pivot and regions, term set, PivotMDS
start layout, T Jacobi sweeps of Eq. 5, final stress.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload rgg|grid|ba|mesh]
    python bench.py --workload serve [--requests 4096] [--loads 0.5 0.8 0.95] [--pool-gib G]

The serve workload runs a stream of layout requests through the layout pool
(continuous batching); its step is the whole stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (description, builder, k, iters, precision)
    "rgg": ("random geometric graph, n=100000 uniform in the unit square, mean degree 8, largest "
            "component, seed 12345; k=200 maxmin pivots from node 0; 500 sweeps; FP32 coordinates",
            lambda G: G.rgg(100000, 12345, 8.0), 200, 500, "fp32"),
    "grid": ("grid 50x50, k=50 maxmin pivots from node 0, 200 sweeps, FP64",
             lambda G: G.grid(50, 50), 50, 200, "fp64"),
    "ba": ("Barabasi-Albert n=1000000, m0=5, seed 7; k=200; 300 sweeps; FP32 coordinates",
           lambda G: G.barabasi_albert(1000000, 5, 7), 200, 300, "fp32"),
    "mesh": ("triangulated 2000x2000 lattice minus 200 circular holes (radius 10-60), largest "
             "component, seed 12345; k=100; 300 sweeps; FP32 coordinates",
             lambda G: G.holed_mesh(2000, 2000, 200, 10, 60, 12345), 100, 300, "fp32"),
}

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# VALU issue capacity without packed FP32 (disabled in this build): 256 CUs x
# 64 lanes per clock x 2.4 GHz, in lane-slots per second
VALU_PEAK_TSLOTS = 256 * 64 * 2.4e9 / 1e12
# VALU lane-slots of the arithmetic one FP32 term needs: two subtractions,
# two FMAs for r^2, the reciprocal square root (a transcendental: measured on
# MI355X at half the FMA rate, 2 slots), one FMA for the coefficient and two
# FMAs into the sums -- addressing and unpacking excluded
SLOTS_PER_TERM = 9
PROFILE_LABEL = {"rgg": "rgg100k_k200", "ba": "ba1m_k200", "mesh": "mesh2000_k100", "grid": "grid50_k50"}


SWEEP_KERNEL_SRC = os.path.join(ROOT, "paper_1608_08909_amd", "csrc", "sweep_f32.h")


def kernel_source_sha256() -> str:
    """sha256 of the FP32 sweep's device code (host-side planning excluded)."""
    import hashlib
    return hashlib.sha256(open(SWEEP_KERNEL_SRC, "rb").read()).hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated by a copy kernel), or None when no
    summary exists or the sweep kernel's source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{PROFILE_LABEL.get(workload, workload)}_sweep_f32_hbm_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "-")):
            a, b = line.split(":", 1)
            fields[a.strip()] = b.strip()
    if fields.get("kernel_source_sha256") != kernel_source_sha256() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def sweep_bytes(n: int, m: int, k: int, dbytes: int, prec: str) -> int:
    """Algorithmic HBM bytes of one Jacobi sweep: every packed pivot distance
    once (k per node), every arc index once, per node its row pointer, its
    coordinates read and written once and its denominator."""
    xb = 8 if prec == "fp32" else 16
    denb = 4 if prec == "fp32" else 8
    return n * k * dbytes + 2 * m * 4 + n * (4 + 2 * xb + denb)


def percentile(a, q):
    return float(np.percentile(np.asarray(a), q))


def cpu_model() -> str:
    """The host CPU's model name, with its family and model numbers (a
    virtual machine may report only a generic name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                key, val = (x.strip() for x in line.split(":", 1))
                if key in ("model name", "cpu family", "model", "stepping") and key not in info:
                    info[key] = val
            if len(info) == 4:
                break
    except OSError:
        pass
    name = info.get("model name", "unknown")
    if "cpu family" in info and "model" in info:
        name += f" (family {info['cpu family']}, model {info['model']}, stepping {info.get('stepping', '?')})"
    return name


def usable_cores() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline(g, k, iters, sweeps_one=1, sweeps_all=3, pmds_work=1e9):
    """The CPU oracle on the same graph (the oracle as it stands, untuned).

    Preprocessing (max/min, BFS, regions, weights; serial in the oracle) runs
    once on the whole graph.  PivotMDS runs on the whole graph when n k^2 is
    at most `pmds_work`, else on the distance columns of the first
    pmds_work / k^2 nodes with its time scaled by n / (those nodes): that
    sample's centred matrix stays closer to the caches, so the scaled time is
    a lower bound.  The sweeps (OpenMP over nodes in the oracle; Jacobi, so
    the result does not depend on the thread count) are sampled on one
    thread and on every usable core and scaled to `iters` sweeps.  The value
    is end-to-end node-updates/s on all cores; `one_thread` repeats it on
    one."""
    import oracle

    cores = usable_cores()
    t0 = time.perf_counter()
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    t_pre = time.perf_counter() - t0
    if g.n * k * k <= pmds_work:
        t0 = time.perf_counter()
        x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
        t_pmds = time.perf_counter() - t0
        pmds_note = "PivotMDS on the whole graph"
    else:
        ns = max(1000, int(pmds_work / (k * k)))
        t0 = time.perf_counter()
        oracle.pivotmds(np.ascontiguousarray(T.dist[:, :ns]))
        t_pmds = (time.perf_counter() - t0) * g.n / ns
        pmds_note = f"PivotMDS on {ns} of {g.n} nodes, time scaled by n/{ns} (a lower bound)"
        # sweep timing needs a start layout only: a seeded one of the layout's scale
        x0 = np.random.default_rng(0).normal(size=(g.n, 2)) * np.sqrt(g.n)
    rates = {}
    for threads, count in ((1, sweeps_one), (cores, sweeps_all)):
        t0 = time.perf_counter()
        oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, count, threads=threads)
        rates[threads] = (time.perf_counter() - t0) / count
    step_1 = t_pre + t_pmds + iters * rates[1]
    step_n = t_pre + t_pmds + iters * rates[cores]
    sample = (f"{cpu_model()}: preprocessing once on one thread ({t_pre:.2f} s), {pmds_note} "
              f"({t_pmds:.2f} s), {sweeps_one} sweep(s) on 1 thread ({rates[1] * 1e3:.0f} ms each) and "
              f"{sweeps_all} on {cores} threads ({rates[cores] * 1e3:.0f} ms each), step time scaled to {iters} sweeps")
    return {"value": g.n * iters / step_n, "unit": "node-updates/s", "cores": cores, "kind": "oracle",
            "sample": sample, "cpu_model": cpu_model(), "step_s": step_n,
            "phase_s": {"preprocess": t_pre, "pivotmds": t_pmds, "sweep_all_cores": rates[cores],
                        "sweep_one_thread": rates[1]},
            "sweep_node_updates_per_s": g.n / rates[cores],
            "one_thread": {"value": g.n * iters / step_1, "cores": 1, "step_s": step_1,
                           "sweep_node_updates_per_s": g.n / rates[1]}}


SERVE_DESC = ("serving stream: {count} layout requests, all queued at once (closed-loop capacity), then with "
              "Poisson arrivals at fractions of that capacity; each graph drawn "
              "uniformly from grid a x b (a, b in [10,150]), random geometric graph (n in [200,20000], mean "
              "degree 6-10, largest component) and random tree + 5% extra edges (n in [200,20000]); "
              "k=min(100, n/10) maxmin pivots; {sweeps} sweeps each (the first FP64, the rest FP32); "
              "layout pool arena {pool_gib:g} GiB, sweep quantum {quantum}")


def _request_graph(spec):
    from paper_1608_08909_amd import graphs as G
    return G.make_request_graph(spec)


def _request_graphs(specs):
    """Generates the request graphs on the host cores (before any device use)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_request_graph, specs, chunksize=8))


def run_serve(args):
    """The serving stream through the layout pool.  First the closed-loop
    capacity: the whole stream queued at once (every request arrives at time
    0), whose layouts/s is the line's value.  Then the same stream with
    Poisson arrivals at `--loads` times that capacity (latency measured at a
    load the server sustains), and once at 0.8 x capacity with Algorithm 1's
    stop test (tolerance `--tol`) to count the sweeps it saves."""
    from paper_1608_08909_amd import graphs as G

    specs = G.serving_requests(args.requests, args.seed)
    warm_specs = G.serving_requests(args.warm_requests, args.seed + 1)
    t_gen = time.perf_counter()
    graphs = _request_graphs(specs)
    warm_graphs = _request_graphs(warm_specs)
    t_gen = time.perf_counter() - t_gen

    import torch

    from paper_1608_08909_amd import serve, ssm

    torch.cuda.set_device(0)
    pool_bytes = int(args.pool_gib * (1 << 30))

    def requests(gs, rate, seed, tol=0.0):
        arr = serve.poisson_arrivals(len(gs), rate, seed) if rate > 0 else np.zeros(len(gs))
        return [serve.Request(i, g, min(100, g.n // 10), float(a), sweeps=args.sweeps, tol=tol)
                for i, (g, a) in enumerate(zip(gs, arr))]

    def run(rate, tol=0.0, seed=args.seed):
        rep = serve.serve(requests(graphs, rate, seed, tol), pool_bytes, args.quantum, max_prepare=args.max_prepare,
                          first_prepare=args.first_prepare, prep_quantum=args.prep_quantum)
        done = rep.completed()
        lat = rep.latencies_ms()
        sweeps = np.array([r.sweeps_run for r in done])
        return rep, done, {
            "rate_per_s": rate, "tol": tol, "completed": len(done), "failed": len(rep.requests) - len(done),
            "wall_s": rep.wall_s, "layouts_per_s": len(done) / rep.wall_s,
            "node_updates_per_s": float(sum(r.graph.n * r.sweeps_run for r in done)) / rep.wall_s,
            "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "max": float(lat.max())},
            "sweeps_per_layout": {"mean": float(sweeps.mean()), "min": int(sweeps.min()), "max": int(sweeps.max())},
            "rounds": rep.rounds, "prepare_batches": rep.prepares, "peak_active_graphs": rep.peak_active,
            "peak_pool_bytes": rep.peak_bytes, "host_phase_s": rep.host_s}

    for _ in range(args.warmup):
        serve.serve(requests(warm_graphs, 0.0, args.seed + 2), pool_bytes, args.quantum, max_prepare=args.max_prepare,
                    first_prepare=args.first_prepare, prep_quantum=args.prep_quantum)
    torch.cuda.synchronize()
    rep, done, closed = run(0.0)
    capacity = closed["layouts_per_s"]
    loads = []
    for frac in args.loads:
        _, _, row = run(frac * capacity, seed=args.seed + 10)
        row["load"] = frac
        loads.append(row)
    # Algorithm 1's stop test per request, at 0.8 x capacity
    _, done_tol, early = run(0.8 * capacity, tol=args.tol, seed=args.seed + 10)
    early["load"] = 0.8
    early["sweeps_saved_fraction"] = 1.0 - early["sweeps_per_layout"]["mean"] / args.sweeps

    # equal final stress: the plain per-graph FP64 path on the same GPU, on a
    # sample spread over the stream (also timed: the plain form's layouts/s);
    # with the stop test, the plain FP64 path with the same stop test
    sample = done[:: max(1, len(done) // 16)][:16]
    rels, t_plain = [], 0.0
    for r in sample:
        dg = ssm.DeviceGraph.from_csr(r.graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, terms, *_ = ssm.layout(dg, r.k, r.sweeps, ssm.FP64)
        s64 = ssm.stress(dg, terms, x)
        t_plain += time.perf_counter() - t0
        rels.append(abs(r.stress - s64) / s64)
    by_id = {r.rid: r for r in done_tol}
    rels_tol = []
    for r in sample:
        rt = by_id.get(r.rid)
        if rt is None:
            continue
        dg = ssm.DeviceGraph.from_csr(rt.graph)
        x, terms, *_ = ssm.layout(dg, rt.k, 1, ssm.FP64)
        ssm.majorize(dg, terms, x, rt.sweeps - 1, tol=args.tol)
        s64 = ssm.stress(dg, terms, x)
        rels_tol.append(abs(rt.stress - s64) / s64)
    early["final_stress_rel_diff_vs_plain_fp64_same_stop"] = {"max": float(max(rels_tol)), "sample": len(rels_tol)}

    # roofline of the pooled FP32 sweep on a batch of the stream's graphs
    batch = graphs[:256]
    pool = ssm.Pool(pool_bytes)
    pairs = [(g, pool.add(g, min(100, g.n // 10), 0, 1 << 30)) for g in batch]
    pairs = [(g, s) for g, s in pairs if s is not None]
    slots = [s for _, s in pairs]
    pool.prepare(slots, 1)
    pool.sweep(slots, 5)
    stream = torch.cuda.current_stream()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    pool.sweep(slots, reps)
    e1.record(stream)
    torch.cuda.synchronize()
    launch_us = e0.elapsed_time(e1) * 1e3 / reps
    nbytes = 0
    for g, s in pairs:  # the graph's own k (the padding ranks are not counted)
        nbytes += g.n * pool.info(s)["k"] * 2 + g.col_idx.size * 4 + g.n * (4 + 8 + 8 + 4)
    batch_nodes = sum(g.n for g, _ in pairs)
    pool.close()
    achieved = nbytes / (launch_us * 1e-6) / 1e9

    out = {
        "metric": "node-updates/sec & layouts/sec (p50/p99) at equal final stress vs plain, 1 GPU",
        "value": capacity,
        "unit": "layouts/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.warmup,
        "ms_per_step": closed["wall_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SERVE_DESC.format(count=args.requests, sweeps=args.sweeps, pool_gib=args.pool_gib,
                                                 quantum=args.quantum),
                   "requests": args.requests, "seed": args.seed, "pool_bytes": pool_bytes, "quantum": args.quantum,
                   "max_prepare": args.max_prepare, "first_prepare": args.first_prepare,
                   "prep_quantum": args.prep_quantum, "sweeps": args.sweeps},
        "closed_loop": closed,
        "layouts_per_s": capacity,
        "latency_ms": closed["latency_ms"],
        "node_updates_per_s": closed["node_updates_per_s"],
        "poisson_loads": loads,
        "early_exit": early,
        "final_stress_rel_diff_vs_plain_fp64": {"max": float(max(rels)), "sample": len(rels)},
        "plain_fp64_layouts_per_s_sample": len(sample) / t_plain,
        "host_graph_generation_s": t_gen,
        "roofline": {"bound": "hbm", "kernel": "k_pool_sweep32", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": nbytes, "launch_us": launch_us, "batch_graphs": len(slots),
                     "batch_nodes": batch_nodes},
    }
    if not args.no_cpu_baseline:
        import oracle
        cs = sorted(done[:64], key=lambda r: r.graph.n)[len(done[:64]) // 2: len(done[:64]) // 2 + 2]
        t0 = time.perf_counter()
        for r in cs:
            oracle.layout(r.graph.n, r.graph.row_ptr, r.graph.col_idx, r.k, r.sweeps)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(cs) / dt, "unit": "layouts/s", "cores": 1, "kind": "oracle",
                               "sample": f"{cpu_model()}: {len(cs)} median-size requests of the stream (n = "
                                         f"{[r.graph.n for r in cs]}), full layouts with {args.sweeps} sweeps, "
                                         f"{dt:.1f} s on one core (the oracle lays out one request per call; "
                                         f"requests are independent, so {usable_cores()} cores would serve about "
                                         f"{usable_cores() * len(cs) / dt:.2f} layouts/s)",
                               "cpu_model": cpu_model()}
    print(json.dumps(out), flush=True)


def run_quality(args):
    """Section 4.1's quality measures on the 50 x 50 grid: the full-stress
    reference (k = n, 500 FP64 sweeps), then sparse layouts (k = 50, 100, 200;
    max/min and k-means sp sampling; 200 FP64 sweeps) scored by normalized
    stress and by the Procrustes statistic against the reference.  One step =
    the reference layout; `value` is its node-updates/s."""
    import torch

    from paper_1608_08909_amd import graphs as G
    from paper_1608_08909_amd import ssm

    torch.cuda.set_device(0)
    g = G.grid(50, 50)
    dg = ssm.DeviceGraph.from_csr(g)
    for _ in range(args.warmup):
        ssm.full_stress_layout(dg, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xr, _ = ssm.full_stress_layout(dg, 500)
    torch.cuda.synchronize()
    t_ref = (time.perf_counter() - t0) / args.steps
    ns_ref = ssm.normalized_stress(dg, xr)
    rows = []
    for sampling in ("maxmin", "kmeans"):
        for k in (50, 100, 200):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, *_ = ssm.layout(dg, k, 200, ssm.FP64, sampling=sampling)
            torch.cuda.synchronize()
            rows.append({"sampling": sampling, "k": k, "ms": (time.perf_counter() - t1) * 1e3,
                         "normalized_stress": ssm.normalized_stress(dg, x), "procrustes": ssm.procrustes(x, xr)})
    out = {
        "metric": "node-updates/sec & layouts/sec (p50/p99) at equal final stress vs plain, 1 GPU",
        "value": g.n * 500 / t_ref,
        "unit": "node-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_ref * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "quality report on the grid 50x50: full-stress reference (k = n = 2500 pivots, "
                               "start from PivotMDS on the first 1024, 500 FP64 sweeps) and sparse layouts (k = 50, 100, 200 by max/min and k-means sp, "
                               "200 FP64 sweeps) scored by normalized stress and the Procrustes statistic"},
        "reference_normalized_stress": ns_ref,
        "quality": rows,
    }
    print(json.dumps(out), flush=True)


def run_weighted(args):
    """Algorithm 1 with edge lengths on the random geometric graph (n =
    100,000, mean degree 8, lengths uniform in [0.5, 2)): one step = max/min
    on lengths, the k shortest-path rows, regions and per-term weights,
    PivotMDS, 500 sweeps (the first FP64, then FP32), stress."""
    import torch

    from paper_1608_08909_amd import graphs as G
    from paper_1608_08909_amd import ssm

    torch.cuda.set_device(0)
    g = G.rgg(100000, 12345, 8.0)
    ln = G.edge_lengths(g, 12345)
    k, iters = 200, 500
    dg = ssm.DeviceGraph.from_csr(g)
    lt = torch.from_numpy(ln).cuda()
    stream = torch.cuda.current_stream()
    phases = {}

    def step(record=False):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
        ev[0].record(stream)
        piv = ssm.select_pivots_w(dg, lt, k, 0)
        ev[1].record(stream)
        dist = ssm.sssp_pivots(dg, lt, piv)
        ev[2].record(stream)
        T = ssm.build_terms_w(dg, lt, piv, dist)
        ev[3].record(stream)
        x = ssm.pivotmds_init_w(dg, lt, T)
        ev[4].record(stream)
        x = ssm.majorize_mixed_w(dg, lt, T, x, iters)
        ev[5].record(stream)
        st = ssm.stress_w(dg, lt, T, x)
        ev[6].record(stream)
        if record:
            torch.cuda.synchronize()
            for a, name in enumerate(["select", "shortest_paths", "terms", "pivotmds", "sweeps", "stress"]):
                phases.setdefault(name, []).append(ev[a].elapsed_time(ev[a + 1]))
        return T, x, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T, x, s32 = step(record=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the FP32 sweep alone, events on its stream
    xs = x.clone()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ssm.majorize_w(dg, lt, T, xs, iters)
    e1.record(stream)
    torch.cuda.synchronize()
    sweep_us = e0.elapsed_time(e1) * 1e3 / (reps * iters)
    nbytes = g.n * k * 8 + g.col_idx.size * (4 + 8) + g.n * (4 + 8 + 8 + 4)
    achieved = nbytes / (sweep_us * 1e-6) / 1e9
    # equal final stress: the FP64 path on the same GPU
    x64 = ssm.pivotmds_init_w(dg, lt, T)
    ssm.majorize_w(dg, lt, T, x64, iters)
    s64 = ssm.stress_w(dg, lt, T, x64)
    out = {
        "metric": "node-updates/sec & layouts/sec (p50/p99) at equal final stress vs plain, 1 GPU",
        "value": g.n * iters * args.steps / elapsed, "unit": "node-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "random geometric graph n=100000 (largest component), mean degree 8, seed 12345, "
                               "edge lengths uniform in [0.5, 2) (seed 12345); k=200 max/min pivots on lengths; "
                               "500 sweeps (first FP64, then FP32)", "n": g.n, "m": g.m, "k": k, "iters": iters},
        "phases_ms": {a: float(np.median(b)) for a, b in phases.items()},
        "sweep_us": sweep_us,
        "final_stress": s32, "final_stress_fp64_plain": s64, "final_stress_rel_diff": abs(s32 - s64) / s64,
        "roofline": {"bound": "hbm", "kernel": "k_wsweep_f32", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": nbytes,
                     "launch_us": sweep_us},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mesh", choices=sorted(WORKLOADS) + ["serve", "quality", "weighted"])
    ap.add_argument("--requests", type=int, default=4096, help="serve: requests in the stream")
    ap.add_argument("--warm-requests", type=int, default=64, help="serve: requests of each warm-up stream")
    ap.add_argument("--loads", type=float, nargs="*", default=[0.5, 0.8, 0.95],
                    help="serve: Poisson arrival rates as fractions of the measured closed-loop capacity")
    ap.add_argument("--tol", type=float, default=1e-4, help="serve: stop-test tolerance of the early-exit stream")
    ap.add_argument("--pool-gib", type=float, default=32.0, help="serve: layout pool arena (GiB)")
    ap.add_argument("--quantum", type=int, default=25, help="serve: sweeps per scheduling round")
    ap.add_argument("--max-prepare", type=int, default=1024, help="serve: largest preparation batch")
    ap.add_argument("--first-prepare", type=int, default=128, help="serve: preparation batch while nothing runs")
    ap.add_argument("--prep-quantum", type=int, default=100, help="serve: sweeps queued in a round that prepares")
    ap.add_argument("--sweeps", type=int, default=200, help="serve: sweeps per request")
    ap.add_argument("--seed", type=int, default=4, help="serve: stream seed")
    ap.add_argument("--sampling", default="maxmin", choices=["maxmin", "kmeans"],
                    help="pivot sampling: max/min, or max/min refined by k-means sp")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(each graph's layout runs on a single device)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "quality":
        run_quality(args)
        return
    if args.workload == "weighted":
        run_weighted(args)
        return

    import torch

    from paper_1608_08909_amd import graphs as G
    from paper_1608_08909_amd import ssm

    desc, builder, k, iters, prec_name = WORKLOADS[args.workload]
    prec = ssm.FP32 if prec_name == "fp32" else ssm.FP64
    torch.cuda.set_device(0)
    g = builder(G)
    dg = ssm.DeviceGraph.from_csr(g)
    ssm.validate_csr(dg)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    phases = {}
    km_passes = []
    last_pivots = [None]
    kmeans = args.sampling == "kmeans"

    def step(record=False):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
        ev[0].record(stream)
        if kmeans:
            piv0, dist0 = ssm.select_pivots(dg, k, 0, with_dist=True)
            ev[7].record(stream)
            piv, _, passes = ssm.kmeans_pivots(piv0, dist0)
            del dist0
        else:
            piv = ssm.select_pivots(dg, k, 0)
        last_pivots[0] = piv
        ev[1].record(stream)
        dist, delta, region = ssm.bfs_pivots(dg, piv)
        ev[2].record(stream)
        terms = ssm.build_terms(dg, piv, dist, delta, region)
        ev[3].record(stream)
        x = ssm.pivotmds_init(dg, terms, ssm.FP64)
        ev[4].record(stream)
        if prec == ssm.FP32:
            x = ssm.majorize_mixed(dg, terms, x, iters, warm=1)
        else:
            ssm.majorize(dg, terms, x, iters)
        ev[5].record(stream)
        s = ssm.stress(dg, terms, x)
        ev[6].record(stream)
        if record:
            torch.cuda.synchronize()
            names = ["select", "bfs_regions", "terms", "pivotmds", "sweeps", "stress"]
            for a, name in enumerate(names):
                phases.setdefault(name, []).append(ev[a].elapsed_time(ev[a + 1]))
            if kmeans:
                phases["select"][-1] = ev[0].elapsed_time(ev[7])
                phases.setdefault("kmeans_sp", []).append(ev[7].elapsed_time(ev[1]))
                km_passes.append(passes)
        return terms, x, s

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    step_ms = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        terms, x, s32 = step(record=True)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = g.n * iters * args.steps / elapsed

    # Sweep kernel alone: events on the stream the sweeps run on.
    kdim, delta_max, dmax = terms.dims()
    dbytes = 1 if dmax <= 255 else 2
    xs = x.clone()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ssm.majorize(dg, terms, xs, iters)
    e1.record(stream)
    torch.cuda.synchronize()
    sweep_us = e0.elapsed_time(e1) * 1e3 / (reps * iters)
    nbytes = sweep_bytes(g.n, g.m, k, dbytes, prec_name)
    achieved = nbytes / (sweep_us * 1e-6) / 1e9
    # terms of one sweep: every (node, pivot) pair at distance >= 2 (all but
    # the pivot itself and its neighbours) and every arc
    deg = np.diff(g.row_ptr)
    pivots_np = last_pivots[0].cpu().numpy()
    n_terms = g.n * k - k - int(deg[pivots_np].sum()) + 2 * g.m
    alu = n_terms * SLOTS_PER_TERM / (sweep_us * 1e-6) / 1e12

    # Equal final stress versus the plain FP64 form on the same GPU.
    x64 = ssm.pivotmds_init(dg, terms, ssm.FP64)
    ssm.majorize(dg, terms, x64, iters)
    s64 = ssm.stress(dg, terms, x64)
    rel = abs(s32 - s64) / s64
    # The method's own sensitivity: FP64 sweeps from the start layout rounded
    # to FP32 once, against FP64 sweeps from the exact start.
    xr = ssm.pivotmds_init(dg, terms, ssm.FP64).float().double()
    ssm.majorize(dg, terms, xr, iters)
    band = abs(ssm.stress(dg, terms, xr) - s64) / s64

    out = {
        "metric": "node-updates/sec & layouts/sec (p50/p99) at equal final stress vs plain, 1 GPU",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == ssm.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "sampling": args.sampling, "n": g.n, "m": g.m, "k": k, "iters": iters,
                   "delta_max": delta_max, "dmax": dmax, "graph_sha256": g.sha256()},
        "layouts_per_s": args.steps / elapsed,
        "latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99)},
        "sweep_node_updates_per_s": g.n / (sweep_us * 1e-6),
        "sweep_us": sweep_us,
        "phases_ms": {kk: float(np.median(v)) for kk, v in phases.items()},
        "final_stress": s32,
        "final_stress_fp64_plain": s64,
        "final_stress_rel_diff": rel,
        "fp64_sensitivity_to_fp32_rounded_start": band,
        "roofline": {"bound": "hbm", "kernel": "k_sweep_f32" if prec == ssm.FP32 else "k_sweep_f64",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload) if prec == ssm.FP32 else None,
                     "bytes_per_launch": nbytes, "launch_us": sweep_us,
                     "alu": {"achieved": alu, "peak": VALU_PEAK_TSLOTS, "unit": "T VALU lane-slots/s",
                             "frac": alu / VALU_PEAK_TSLOTS, "terms_per_launch": n_terms,
                             "slots_per_term": SLOTS_PER_TERM}},
    }
    if args.workload == "rgg":
        out["roofline"]["note"] = ("the 45.5 MB working set of one sweep fits the 256 MB last-level cache (MALL): "
                                   "this fraction is of the HBM peak, the bytes are served from the MALL")
    if kmeans:
        # k-means sp: each pass's assignment is an n x k x k FP64 contraction
        # (B = Y S^T), 2 n k^2 flops; phase-level rate (all its kernels and
        # the per-pass host check included).
        ms = float(np.median(phases["kmeans_sp"]))
        p = int(np.median(km_passes))
        tf = 2 * g.n * k * k * p / (ms * 1e-3) / 1e12
        out["kmeans_sp"] = {"passes": p, "ms": ms, "assign_flops_per_pass": 2 * g.n * k * k,
                            "phase_tflops": tf, "phase_frac_fp64_peak": tf / FP64_PEAK_TFLOPS}
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads and writes 256 MiB
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, k, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
    # free the library's handles and cached scratch, and torch's cached device
    # memory, before interpreter teardown
    if "paper_1608_08909_amd.ssm" in sys.modules:
        sys.modules["paper_1608_08909_amd.ssm"].shutdown()
    if "torch" in sys.modules:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
