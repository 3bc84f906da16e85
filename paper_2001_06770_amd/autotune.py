"""Autotuner of the cohort path.

Times one batch of a workload's queries on the GPU for settings of the cohort
path's parameters and keeps the fastest:

* ``admit_below`` -- a batch admits waiting queries only while at most this
  many of the cohort's queries are still exploring (0: level-aligned waves,
  32: whenever a query fits);
* ``expand_tile`` -- examined arcs per expansion tile (512, 1024, 2048);
* ``expand_wg_per_cu`` -- workgroups per compute unit of the expansion.

The objective is the device time of the level kernels (frontier scan, control
step, expansion) over the batch, from the library's event timers; the
batch's wall time is recorded beside it.  The search is coordinate descent in
the order above, starting from the library's defaults.  The result is a JSON
file (``tuning/<workload>.json`` in this package) that ``bench.py`` applies.

usage: python -m paper_2001_06770_amd.autotune --workload batch --queries 64 --out FILE
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SPACE = {"admit_below": (0, 4, 32), "expand_tile": (512, 1024, 2048),
         "expand_wg_per_cu": (4, 8, 16)}
DEFAULT = {"admit_below": 32, "expand_tile": 1024, "expand_wg_per_cu": 8}


def tuning_path(workload: str) -> str:
    return os.path.join(HERE, "tuning", f"{workload}.json")


def load(workload: str):
    """The tuned settings of a workload, or None."""
    p = tuning_path(workload)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)["choice"]


def measure(ctx, qs, setting, raks):
    ctx.set_tuning(**setting)
    ctx.set_timing(True)
    t0 = time.perf_counter()
    ctx.query_batch(qs, lean=True)
    wall = time.perf_counter() - t0
    ms = sum(ctx.timing(k)["ms"] for k in (raks.TIMER_EXPAND, 1, 2))
    ctx.set_timing(False)
    return ms, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--queries", type=int, default=64)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import synth
    import paper_2001_06770_amd as raks
    g = synth.make_graph(args.workload)
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_queries.json")
    if os.path.exists(gold):
        # the sampled queries the benchmark times
        with open(gold) as f:
            ent = json.load(f)["queries"]
        qs = [synth.Query(tuple(e["central"]), tuple(e["marginal"]), e["k"], e["w"],
                          e["max_level"]) for e in ent][:args.queries]
        qdesc = f"first {len(qs)} of the sampled queries (tests/golden)"
    else:
        qs = synth.make_queries(g, args.workload)[:args.queries]
        qdesc = f"first {len(qs)}"
    ctx = raks.Context(0)
    ctx.load_graph(g, alpha=0.5)
    ctx.query_batch(qs, lean=True)   # warm-up: lanes, buffers, code objects
    cur = dict(DEFAULT)
    best_ms, _ = measure(ctx, qs, cur, raks)
    trials = [{"setting": dict(cur), "level_kernel_ms": best_ms}]
    print(f"# default {cur}: {best_ms:.1f} ms", file=sys.stderr, flush=True)
    for key, values in SPACE.items():
        for val in values:
            if val == cur[key]:
                continue
            cand = dict(cur, **{key: val})
            ms, wall = measure(ctx, qs, cand, raks)
            trials.append({"setting": cand, "level_kernel_ms": ms, "wall_s": wall})
            print(f"# {cand}: {ms:.1f} ms ({wall:.2f} s wall)", file=sys.stderr, flush=True)
            if ms < best_ms:
                best_ms, cur = ms, cand
    ctx.close()
    out = {"workload": args.workload, "queries": qdesc,
           "objective": "device ms of the level kernels (scan, control, expansion) per batch",
           "choice": cur, "level_kernel_ms": best_ms, "trials": trials}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["choice"]))


if __name__ == "__main__":
    main()
