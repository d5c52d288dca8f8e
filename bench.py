"""Benchmark of the sparse stress model's hot path on one MI355X.

One step = the whole path over one synthetic graph already resident in HBM:
max/min pivot selection, BFS from every pivot and regions, term set, PivotMDS
start layout, T Jacobi sweeps of Eq. 5, final stress.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload rgg|grid|ba|mesh]
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
PROFILE_LABEL = {"rgg": "rgg100k_k200", "ba": "ba1m_k200", "mesh": "mesh2000_k100", "grid": "grid50_k50"}


def measured_traffic(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated by a copy kernel), or None when no
    summary exists or the sweep source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{PROFILE_LABEL.get(workload, workload)}_sweep_f32_hbm_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "-")):
            a, b = line.split(":", 1)
            fields[a.strip()] = b.strip()
    src = os.path.join(ROOT, "paper_1608_08909_amd", "csrc", "sweep.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("sweep_source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
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


def cpu_baseline(g, k, iters, sample_sweeps, threads=1):
    """The CPU oracle on the same graph: the full preprocessing and start
    layout once, then `sample_sweeps` sweeps; the step time is extrapolated to
    `iters` sweeps."""
    import oracle

    t0 = time.perf_counter()
    T = oracle.preprocess(g.n, g.row_ptr, g.col_idx, k)
    x0 = oracle.initial_layout(g.row_ptr, g.col_idx, T)
    t1 = time.perf_counter()
    oracle.majorize(g.row_ptr, g.col_idx, T.pivots, T.dist, T.wtab, T.den, x0, sample_sweeps, threads=threads)
    t2 = time.perf_counter()
    per_sweep = (t2 - t1) / sample_sweeps
    step = (t1 - t0) + iters * per_sweep
    return {"value": g.n * iters / step, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"preprocessing + PivotMDS once ({t1 - t0:.2f} s) and {sample_sweeps} of {iters} sweeps "
                      f"({per_sweep * 1e3:.1f} ms each), step time extrapolated to {iters} sweeps",
            "step_s": step, "sweep_node_updates_per_s": g.n / per_sweep}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rgg", choices=sorted(WORKLOADS))
    ap.add_argument("--sampling", default="maxmin", choices=["maxmin", "kmeans"],
                    help="pivot sampling: max/min, or max/min refined by k-means sp")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(each graph's layout runs on a single device)", file=sys.stderr)
        sys.exit(2)

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
                     "bytes_per_launch": nbytes, "launch_us": sweep_us},
    }
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
        out["cpu_baseline"] = cpu_baseline(g, k, iters, args.cpu_sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
