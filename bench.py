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
              "k = w = 20, level bound 20; single-query path",
    "small": "small: 10k nodes, 50k directed edges; 64 queries of 2 + 2 keywords, k = w = 10",
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="edge", choices=["edge", "node"])
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
    mode = raks.RAKS_ACT_EDGE if args.mode == "edge" else raks.RAKS_ACT_NODE
    ctx = raks.Context(0)
    ctx.load_graph(g, alpha=0.5, mode=mode)
    torch.cuda.synchronize()
    print(f"# graph loaded: {g.n_nodes} nodes, {g.n_arcs} arcs", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        for q in qs:
            ctx.query(q, lean=True)
    torch.cuda.synchronize()

    ctx.set_timing(True)
    lat, dev_ms, arcs, nq = [], [], 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for q in qs:
            a = time.perf_counter()
            r = ctx.query(q, lean=True)
            lat.append((time.perf_counter() - a) * 1e3)
            dev_ms.append(r["device_ms"])
            arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
            nq += 1
        print(f"# step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    texp = ctx.timing(raks.TIMER_EXPAND)
    ctx.set_timing(False)
    timers = {name: ctx.timing(i) for i, name in
              enumerate(["expand", "scan", "control", "recover", "other"])}

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
                   "queries_per_step": len(qs), "path": "single"},
        "qps": nq / dt,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "device_p50_ms": percentile(dev_ms, 50),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "k_expand", "launches": texp["launches"],
                     "avg_launch_us": texp["ms"] * 1e3 / max(texp["launches"], 1),
                     "bytes_per_launch": texp["bytes"] / max(texp["launches"], 1)},
        "kernel_ms": {k: round(v["ms"], 3) for k, v in timers.items()},
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline (reference implementation) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, qs, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
