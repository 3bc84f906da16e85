"""Benchmark of the RAKS hot path on one MI355X.

A step is one pass over the workload's query set through the whole path
(activation levels resident; per query: both exploration runs, central-node
identification, top-w, recovery, RPG check with Theorem 4, ranking, marginal
recovery, results back on the host).  Prints one JSON line.

value = GTEPS: arcs scanned by the algorithm (E_arc of both runs, the count
the reference implementation also reports) per second of wall time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS + queries/s (batched vs single), bit-exact; p50/p99 query latency"
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "medium": "medium: 2M nodes, 20M directed edges (40M arcs), power-law 2.1, 100 labels, "
              "vocabulary 100k Zipf 1.1; 32 queries of 3 central + 3 marginal keywords, "
              "k = w = 20, level bound 20",
    "small": "small: 10k nodes, 50k directed edges; 64 queries of 2 + 2 keywords, k = w = 10",
    "large": "large: 20M nodes, 200M directed edges, power-law 2.0, hubs of 1.0-2.0M "
             "out-edges, vocabulary 1M; 8 queries of 5 + 5 keywords, k = w = 50, level bound 12",
    "batch": "batch: 20M nodes, 200M directed edges, power-law 2.1, vocabulary 100k; "
             "256 queries of 1-4 central + 1-4 marginal keywords, k = w = 20, level bound 20",
    "serve": "serve: 50M nodes, 500M directed edges, power-law 2.1, vocabulary 1M; "
             "queries of 2-10 keywords split into central/marginal, k = w = 20, level bound 20",
}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(g, qs, budget_s):
    import oracle
    o = oracle.Oracle(g, check=False)
    act = o.activation(g.abar, 0.5)
    arcs, n, t0 = 0, 0, time.perf_counter()
    for q in qs:
        r = o.query(act, q)
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": arcs / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"first {n} of the {len(qs)} workload queries, single thread, "
                      f"{dt:.1f} s; activation levels precomputed (not timed)",
            "qps": n / dt}


def traffic_for(args):
    """HBM bytes per k_expand launch from the committed profiler summary, or
    None when the summary is missing or was taken on other expansion code or
    another workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_expand_{args.workload}_traffic.json")
    if not os.path.exists(path) or args.path != "single" or args.mode != "edge":
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2001_06770_amd", "csrc", "explore.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if rec.get("explore_hip_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def cpu_parallel(g, qs, budget_s):
    """The paper's OpenMP CPU variant on all host cores, on the same leading
    queries as the single-core reference leg."""
    import baselines
    import oracle
    act = oracle.Oracle(g, check=False).activation(g.abar, 0.5)
    cpu = baselines.CpuRaks(g)
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    arcs, n, t0 = 0, 0, time.perf_counter()
    for q in qs:
        r = cpu.query(act, q, threads)
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": arcs / dt / 1e9, "unit": "GTEPS", "cores": threads,
            "kind": "paper CPU variant (OpenMP)", "qps": n / dt,
            "sample": f"first {n} of the {len(qs)} workload queries, {threads} threads, "
                      f"{dt:.1f} s; activation levels precomputed (not timed)"}


def run_single(ctx, qs, lat, dev_ms):
    arcs = 0
    for i, q in enumerate(qs):
        if i and i % 64 == 0:
            print(f"#   {i}/{len(qs)} queries", file=sys.stderr, flush=True)
        a = time.perf_counter()
        r = ctx.query(q, lean=True)
        lat.append((time.perf_counter() - a) * 1e3)
        dev_ms.append(r["device_ms"])
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
    return arcs


def run_batched(ctx, qs, lat, dev_ms):
    a = time.perf_counter()
    rs = ctx.query_batch(qs, lean=True)
    wall = (time.perf_counter() - a) * 1e3
    arcs = 0
    for r in rs:
        lat.append(wall)    # a query of a batch is done when its batch is
        dev_ms.append(r["device_ms"])
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
    return arcs


def serving_leg(ctx, qs, rate, n, seed):
    """Open-loop Poisson arrivals at ``rate`` queries/s into the serving loop.
    Latency runs from the scheduled arrival to results ready, so a late
    submission counts against the server (no coordinated omission)."""
    import random
    rng = random.Random(seed)
    ctx.serve_start(lanes=0)
    try:
        sub = []
        t0 = time.perf_counter()
        t_next = t0
        for i in range(n):
            t_next += rng.expovariate(rate)
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            late_ms = (time.perf_counter() - t_next) * 1e3
            sub.append((ctx.submit(qs[i % len(qs)]), late_ms))
        lat, qwait, arcs = [], [], 0
        for t, late_ms in sub:
            r = ctx.wait(t, lean=True)
            lat.append(late_ms + r["host_ms"])
            qwait.append(r["queue_ms"])
            arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
        dt = time.perf_counter() - t0
    finally:
        ctx.serve_stop()
    return {"rate_qps": rate, "queries": n, "achieved_qps": n / dt, "gteps": arcs / dt / 1e9,
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "queue_p50_ms": percentile(qwait, 50), "queue_p99_ms": percentile(qwait, 99)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="edge", choices=["edge", "node"])
    ap.add_argument("--path", default="single", choices=["single", "batched"],
                    help="path of the timed steps (value, roofline)")
    ap.add_argument("--lanes", type=int, default=4, help="lanes of the batched path")
    ap.add_argument("--only-timed", action="store_true",
                    help="skip the other path's leg and the serving leg (profiling runs)")
    ap.add_argument("--serve-rates", default="200,1000",
                    help="Poisson arrival rates (queries/s) of the serving leg; '' skips it")
    ap.add_argument("--queries", type=int, default=0,
                    help="use only the first N queries of the workload per step (0 = all)")
    ap.add_argument("--serve-queries", type=int, default=256,
                    help="arrivals per rate (at least; see --serve-seconds)")
    ap.add_argument("--serve-seconds", type=float, default=0.0,
                    help="if set, arrivals per rate = rate * seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "profiler's FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the search shards by query across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 5}))
        return
    import synth
    import paper_2001_06770_amd as raks

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    g = synth.make_graph(args.workload)
    qs = synth.make_queries(g, args.workload)
    if args.queries:
        qs = qs[:args.queries]
    mode = raks.RAKS_ACT_EDGE if args.mode == "edge" else raks.RAKS_ACT_NODE
    lanes = max(1, args.lanes)
    ctx = raks.Context(0, lanes=lanes)
    ctx.load_graph(g, alpha=0.5, mode=mode)
    from paper_2001_06770_amd import autotune
    tuned = autotune.load(args.workload)
    if tuned:
        ctx.set_tuning(**tuned)
    torch.cuda.synchronize()
    print(f"# graph loaded: {g.n_nodes} nodes, {g.n_arcs} arcs", file=sys.stderr, flush=True)
    legs = {"single": run_single, "batched": run_batched}

    step_fn = legs[args.path]
    for _ in range(args.warmup):
        step_fn(ctx, qs, [], [])
    torch.cuda.synchronize()

    # ---- timed steps
    ctx.set_timing(1 << raks.TIMER_EXPAND)   # events around the expansion launches only
    lat, dev_ms, arcs = [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        arcs += step_fn(ctx, qs, lat, dev_ms)
        print(f"# step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nq = len(qs) * args.steps
    texp = ctx.timing(raks.TIMER_EXPAND)
    ctx.set_timing(False)

    achieved = texp["bytes"] / (texp["ms"] * 1e-3) / 1e9 if texp["ms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": arcs / dt / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "activation": args.mode,
                   "queries_per_step": len(qs), "path": args.path,
                   "queries_used": "all" if not args.queries else f"first {len(qs)}",
                   "lanes": lanes if args.path == "batched" else 1,
                   "cohort_tuning": tuned},
        "qps": nq / dt,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "device_p50_ms": percentile(dev_ms, 50),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_for(args),
                     "kernel": "k_expand", "launches": texp["launches"],
                     "avg_launch_us": texp["ms"] * 1e3 / max(texp["launches"], 1),
                     "bytes_per_launch": texp["bytes"] / max(texp["launches"], 1)},
    }
    # algorithmic efficiency: algorithmic bytes per launch over measured HBM bytes
    rf = out["roofline"]
    rf["alg_efficiency"] = rf["bytes_per_launch"] / rf["traffic"] if rf["traffic"] else None

    # ---- the other path, same queries (not part of the timed steps)
    if not args.only_timed:
        other = "batched" if args.path == "single" else "single"
        fn = legs[other]
        fn(ctx, qs, [], [])
        olat, odev, oarcs = [], [], 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            oarcs += fn(ctx, qs, olat, odev)
        torch.cuda.synchronize()
        odt = time.perf_counter() - t1
        out[other] = {"lanes": lanes if other == "batched" else 1, "gteps": oarcs / odt / 1e9,
                      "qps": nq / odt, "ms_per_step": odt * 1e3 / args.steps,
                      "p50_ms": percentile(olat, 50), "p99_ms": percentile(olat, 99)}
        single_qps = out["qps"] if args.path == "single" else out["single"]["qps"]
        batched_qps = out["qps"] if args.path == "batched" else out["batched"]["qps"]
        out["batched_over_single"] = batched_qps / single_qps
        print(f"# {other} leg done", file=sys.stderr, flush=True)
        rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
        if rates:
            out["serving"] = [
                serving_leg(ctx, qs, r, max(args.serve_queries, int(r * args.serve_seconds)),
                            seed=int(r)) for r in rates]
            print("# serving leg done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("# cpu baseline (reference implementation) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, qs, args.cpu_seconds)
        print("# cpu parallel variant ...", file=sys.stderr, flush=True)
        out["cpu_parallel"] = cpu_parallel(g, qs, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
