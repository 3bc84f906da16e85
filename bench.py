"""Benchmark of the RAKS hot path on one MI355X.

A step is one pass over the workload's timed query set through the whole path
(activation levels resident; per query: both exploration runs, central-node
identification, top-w, recovery, RPG check with Theorem 4, ranking, marginal
recovery, results back on the host).  The default workload is the largest
one, the serving graph (50M nodes, 1B arcs), with its 32 sampled queries; the
timed path is the batched one (cohorts: many queries per level loop).  Prints
one JSON line.

value = GTEPS: arcs scanned by the algorithm (E_arc of both runs, the count
the reference implementation also reports) per second of wall time.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS + queries/s (batched vs single), bit-exact; p50/p99 query latency"
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "serve": "serve: 50M nodes, 500M directed edges (1B arcs), power-law 2.1, 100 labels, "
             "vocabulary 1M Zipf 1.1; queries of 2-10 keywords split randomly into central/"
             "marginal, k = w = 20, level bound 20",
    "batch": "batch: 20M nodes, 200M directed edges (400M arcs), power-law 2.1, vocabulary 100k; "
             "queries of 1-4 central + 1-4 marginal keywords, k = w = 20, level bound 20",
    "large": "large: 20M nodes, 200M directed edges, power-law 2.0, hubs of 1.0-2.0M "
             "out-edges, vocabulary 1M; queries of 5 + 5 keywords, k = w = 50, level bound 12",
    "medium": "medium: 2M nodes, 20M directed edges (40M arcs), power-law 2.1, 100 labels, "
              "vocabulary 100k Zipf 1.1; queries of 3 central + 3 marginal keywords, "
              "k = w = 20, level bound 20",
    "small": "small: 10k nodes, 50k directed edges; queries of 2 + 2 keywords, k = w = 10",
}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[i]


def golden_set(workload):
    """The workload's sampled queries and the reference's counters for them
    (tests/golden, written by a script that runs only the reference)."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_queries.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def alg_bytes(stats, C, M, n):
    """Algorithmic bytes of one query's exploration from its work counters:
    per scanned arc its id and level (5), per arc passing the gate the
    neighbour's |T| hitting levels, one byte per written level (the
    expansion); per frontier node a queue entry, its row bounds and own row,
    per level a frontier bitmap, and the matrix init (the level loop)."""
    expand = loop = 0.0
    for st, T in zip(stats, (C, M)):
        if not st.get("levels"):
            continue
        e = 5.0 * st["e_arc"] + T * st["gate_pass"] + st["h_writes"]
        expand += e
        loop += e + (4 + 8 + T) * st["frontier"] + st["levels"] * n / 8.0 + n * T
    return expand, loop


def traffic_for(args):
    """HBM bytes per expansion launch from the committed profiler summary, or
    None when the summary is missing or was taken on other expansion code or
    another workload or path."""
    if args.mode != "edge":
        return None
    kern, src = (("k_expand", "explore.hip") if args.path == "single"
                 else ("k_co_expand", "cohort.hip"))
    path = os.path.join(ROOT, "profiles", f"{kern}_{args.workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2001_06770_amd", "csrc", src), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if rec.get(src.replace(".", "_") + "_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_legs(g, qs, budget_s):
    """The CPU baselines on the same graph: activation levels from the paper's
    OpenMP CPU variant (all cores; not part of the metric), the reference
    implementation's exploration (Algorithm 1, one thread) on query 0's
    central keywords with the level bound raised one level at a time while it
    fits the budget, the CPU variant's full queries, and its thread sweep on
    the reference's sample."""
    import baselines
    import oracle
    cores = host_cores()
    cpu = baselines.CpuRaks(g)
    t0 = time.perf_counter()
    act = cpu.activation(g.abar, 0.5, 0, cores)
    t_act = time.perf_counter() - t0
    o = oracle.Oracle(g, check=False)
    kws = list(qs[0].central)
    done = None
    for L in range(0, 21):
        t1 = time.perf_counter()
        _, st = o.explore(act, kws, block=True, max_level=L)
        dt = time.perf_counter() - t1
        done = (L, st, dt)
        if dt * 4 > budget_s or st["end"] != "level_bound":
            break
    L, st, dt = done
    base = {"value": st["e_arc"] / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"Algorithm 1 exploration of timed query 0's {len(kws)} central keywords, "
                      f"levels 0..{st['levels'] - 1} ({st['e_arc']} arcs scanned), one thread, "
                      f"{dt:.1f} s; activation levels from the CPU variant ({t_act:.1f} s on "
                      f"{cores} threads, not timed)"}
    # the paper's CPU variant: full queries on all cores, then its Tnum sweep
    arcs, n, t2 = 0, 0, time.perf_counter()
    for q in qs:
        r = cpu.query(act, q, cores)
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
        n += 1
        if time.perf_counter() - t2 > budget_s:
            break
    dq = time.perf_counter() - t2
    par = {"value": arcs / dq / 1e9, "unit": "GTEPS", "cores": cores,
           "kind": "paper CPU variant (OpenMP)", "qps": n / dq,
           "sample": f"first {n} of the {len(qs)} timed queries, {cores} threads, {dq:.1f} s",
           "activation_s": t_act}
    sweep = []
    for th in sorted({1, 2, 4, 8, cores}):
        t3 = time.perf_counter()
        s2 = cpu.explore(act, kws, block=True, max_level=L, threads=th)
        d3 = time.perf_counter() - t3
        sweep.append({"threads": th, "gteps": s2["e_arc"] / d3 / 1e9, "s": d3})
    par["tnum_sweep"] = {"sample": "the reference's exploration sample above", "points": sweep}
    return base, par


def run_single(ctx, qs, lat):
    arcs = 0
    for i, q in enumerate(qs):
        a = time.perf_counter()
        r = ctx.query(q, lean=True)
        lat.append((time.perf_counter() - a) * 1e3)
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
    return arcs


def run_batched(ctx, qs, lat):
    rs = ctx.query_batch(qs, lean=True)
    arcs = 0
    for r in rs:
        lat.append(r["host_ms"])   # from the batch call to the query's results
        arcs += r["stats"][0]["e_arc"] + r["stats"][1]["e_arc"]
    return arcs


def serving_leg(ctx, qs, rate, n, seed):
    """Open-loop Poisson arrivals at ``rate`` queries/s into the serving loop.
    Latency runs from the scheduled arrival to results ready, so a late
    submission counts against the server (no coordinated omission)."""
    import random
    rng = random.Random(seed)
    ctx.serve_start()
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


def leg(fn, ctx, qs, passes):
    import torch
    lat, arcs = [], 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(passes):
        arcs += fn(ctx, qs, lat)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return {"gteps": arcs / dt / 1e9, "qps": len(qs) * passes / dt,
            "ms_per_step": dt * 1e3 / passes, "p50_ms": percentile(lat, 50),
            "p99_ms": percentile(lat, 99)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="serve", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="edge", choices=["edge", "node"])
    ap.add_argument("--path", default="batched", choices=["single", "batched"],
                    help="path of the timed steps (value, roofline)")
    ap.add_argument("--lanes", type=int, default=4, help="lanes of the lanes-mode batch leg")
    ap.add_argument("--only-timed", action="store_true",
                    help="skip every leg but the timed one (profiling runs)")
    ap.add_argument("--serve-rates", default="200,1000",
                    help="Poisson arrival rates (queries/s) of the serving legs; '' skips them")
    ap.add_argument("--serve-queries", type=int, default=64, help="arrivals per rate")
    ap.add_argument("--queries", type=int, default=0,
                    help="time the first N queries of the workload (0: its sampled set "
                         "from tests/golden when there is one, else all)")
    ap.add_argument("--alphas", default="0.2,0.35,0.65,0.8",
                    help="alpha sweep of the batched path (Section 5.2 Exp-4); '' skips it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates the "
                         "profiler's FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(queries are independent: several GPUs would each hold the graph and take a "
              "share of the queries)", file=sys.stderr)
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
    from paper_2001_06770_amd import autotune

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    t_gen = time.perf_counter()
    g = synth.make_graph(args.workload)
    print(f"# graph generated: {g.n_nodes} nodes, {g.n_arcs} arcs "
          f"({time.perf_counter() - t_gen:.0f} s)", file=sys.stderr, flush=True)
    gold = golden_set(args.workload) if not args.queries else None
    if gold:
        qs = [synth.Query(tuple(e["central"]), tuple(e["marginal"]), e["k"], e["w"],
                          e["max_level"]) for e in gold["queries"]]
        qdesc = (f"the {len(qs)} sampled queries of tests/golden (indices "
                 f"{gold['queries'][0]['index']}, {gold['queries'][1]['index']}, ... of the "
                 f"seeded stream)")
    else:
        qs = synth.make_queries(g, args.workload)
        if args.queries:
            qs = qs[:args.queries]
        qdesc = f"the first {len(qs)} queries of the seeded stream"
    mode = raks.RAKS_ACT_EDGE if args.mode == "edge" else raks.RAKS_ACT_NODE
    ctx = raks.Context(0, lanes=max(1, args.lanes))
    ctx.load_graph(g, alpha=0.5, mode=mode)
    tuned = autotune.load(args.workload)
    if tuned:
        ctx.set_tuning(**tuned)
    torch.cuda.synchronize()
    print("# graph loaded", file=sys.stderr, flush=True)
    legs = {"single": run_single, "batched": run_batched}
    step_fn = legs[args.path]
    for _ in range(args.warmup):
        step_fn(ctx, qs, [])
    torch.cuda.synchronize()

    # ---- timed steps: events around the level kernels (expansion, scan, control)
    ctx.set_timing((1 << raks.TIMER_EXPAND) | (1 << raks.TIMER_SCAN) | (1 << raks.TIMER_CONTROL))
    lat, arcs = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        arcs += step_fn(ctx, qs, lat)
        print(f"# step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nq = len(qs) * args.steps
    tk = {k: ctx.timing(k) for k in (raks.TIMER_EXPAND, raks.TIMER_SCAN, raks.TIMER_CONTROL)}
    ctx.set_timing(False)

    # algorithmic bytes of the timed steps from the reference's counters
    # (stored with the sampled queries) or, without them, the library's own
    # counters, which the parity tests hold equal to the reference's
    exp_b = loop_b = 0.0
    if gold:
        for e in gold["queries"]:
            a, b = alg_bytes(e["stats"], len(e["central"]), len(e["marginal"]), g.n_nodes)
            exp_b, loop_b = exp_b + a, loop_b + b
        counters = "reference implementation (tests/golden)"
    else:
        for q in qs:
            r = ctx.query(q, lean=True)
            a, b = alg_bytes(r["stats"], len(q.central), len(q.marginal), g.n_nodes)
            exp_b, loop_b = exp_b + a, loop_b + b
        counters = "library counters (equal to the reference's in the parity tests)"
    exp_b *= args.steps
    loop_b *= args.steps
    te = tk[raks.TIMER_EXPAND]
    t_exp = te["ms"] * 1e-3
    t_loop = sum(t["ms"] for t in tk.values()) * 1e-3
    launches = max(te["launches"], 1)
    achieved = exp_b / t_exp / 1e9 if t_exp > 0 else 0.0
    loop_ach = loop_b / t_loop / 1e9 if t_loop > 0 else 0.0
    traffic = traffic_for(args)
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
                   "queries": qdesc, "queries_per_step": len(qs), "path": args.path,
                   "cohort_tuning": tuned},
        "qps": nq / dt,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "kernel": "k_expand" if args.path == "single" else "k_co_expand",
            "launches": te["launches"], "avg_launch_us": te["ms"] * 1e3 / launches,
            "bytes_per_launch": exp_b / launches,
            "bytes_model": "per query and run: 5 E_arc + |T| gate_pass + h_writes, counters "
                           "from the " + counters,
            "examined_bytes_per_launch": te["bytes"] / launches,
            "alg_efficiency": (exp_b / launches) / traffic if traffic else None,
            "level_loop": {"achieved": loop_ach, "frac": loop_ach / PEAK_HBM_GBS,
                           "kernels": "scan + control + expansion",
                           "ms_per_step": t_loop * 1e3 / args.steps},
        },
    }

    if not args.only_timed:
        other = "single" if args.path == "batched" else "batched"
        r = leg(legs[other], ctx, qs, 1)
        out[other] = r
        sq = out["qps"] if args.path == "single" else r["qps"]
        bq = out["qps"] if args.path == "batched" else r["qps"]
        out["batched_over_single"] = bq / sq
        print(f"# {other} leg done", file=sys.stderr, flush=True)
        ctx.set_batch_mode(raks.RAKS_BATCH_LANES)
        out["lanes_batch"] = dict(leg(run_batched, ctx, qs, 1), lanes=max(1, args.lanes))
        ctx.set_batch_mode(raks.RAKS_BATCH_COHORT)
        print("# lanes leg done", file=sys.stderr, flush=True)
        rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
        if rates:
            out["serving"] = [serving_leg(ctx, qs, rt, args.serve_queries, seed=int(rt))
                              for rt in rates]
            print("# serving legs done", file=sys.stderr, flush=True)
        alphas = [float(x) for x in args.alphas.split(",") if x.strip()]
        if alphas:
            base = out["value"] if args.path == "batched" else out["batched"]["gteps"]
            bq = out["qps"] if args.path == "batched" else out["batched"]["qps"]
            sweep = [{"alpha": 0.5, "gteps": base, "qps": bq}]
            for a in alphas:
                ctx.set_alpha(a)
                r = leg(run_batched, ctx, qs, 1)
                sweep.append({"alpha": a, "gteps": r["gteps"], "qps": r["qps"]})
            ctx.set_alpha(0.5)
            out["alpha_sweep"] = {"path": "batched", "points": sorted(sweep, key=lambda d: d["alpha"])}
            print("# alpha sweep done", file=sys.stderr, flush=True)
    ctx.close()
    if not args.no_cpu_baseline:
        print("# cpu legs ...", file=sys.stderr, flush=True)
        out["cpu_baseline"], out["cpu_parallel"] = cpu_legs(g, qs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
