"""Writes expected results of the reference implementation for the full-size
workloads (large, batch, serve) to tests/golden/<workload>_queries.json.

Calls only the reference (``oracle``) and the seeded input generator
(``synth``).  It stores the SHA-256 of the activation levels (uint8 per arc)
and, for each sampled query, the status, the counters of both
runs and, per result, central node, scores, key, sizes and SHA-256 digests of
the node list (int32 little-endian) and of the arc list ((src, dst, label)
int32 triples), so the GPU tests can check full-size outputs without running
the reference at those sizes during the test.

usage: python tests/golden/make_golden.py large [n_queries] [--node] [--shard K/N PART_FILE]
       python tests/golden/make_golden.py merge large PART_FILE...

--node uses NODE activation (levels from the node weights) and writes
tests/golden/<workload>_node_queries.json.

With --shard, only every N-th sampled query starting at K is run and the
entries go to PART_FILE; merge combines the parts of all N shards into
tests/golden/<workload>_queries.json (the same file one unsharded run writes).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth   # noqa: E402


def digest(result: dict) -> dict:
    nodes = np.asarray(result["nodes"], np.int32).tobytes()
    arcs = np.asarray(result["arcs"], np.int32).reshape(-1, 3).tobytes()
    return {"central": result["central"], "score_c": result["score_c"],
            "score_m": result["score_m"], "key": result["key"],
            "n_nodes": len(result["nodes"]), "n_arcs": len(result["arcs"]),
            "nodes_sha256": hashlib.sha256(nodes).hexdigest(),
            "arcs_sha256": hashlib.sha256(arcs).hexdigest()}


def summarize(res: dict) -> dict:
    return {"status": res["status"], "n_cg": res["n_cg"], "stats": res["stats"],
            "results": [digest(r) for r in res["results"]]}


def write(name, out):
    path = os.path.join(HERE, f"{name}_queries.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    return path


def merge(name, parts):
    out = None
    entries = []
    for p in parts:
        with open(p) as f:
            d = json.load(f)
        if out is None:
            out = {k: v for k, v in d.items() if k != "queries"}
        assert all(d[k] == out[k] for k in out), "parts of different runs"
        entries += d["queries"]
    entries.sort(key=lambda e: e["index"])
    assert len({e["index"] for e in entries}) == len(entries)
    out["queries"] = entries
    print(f"wrote {write(name, out)} ({len(entries)} queries)")


def main():
    if sys.argv[1] == "merge":
        merge(sys.argv[2], sys.argv[3:])
        return
    name = sys.argv[1]
    count = int(sys.argv[2]) if len(sys.argv) > 2 and not sys.argv[2].startswith("--") else 8
    node = "--node" in sys.argv
    shard, part = None, None
    if "--shard" in sys.argv:
        i = sys.argv.index("--shard")
        k, n = (int(x) for x in sys.argv[i + 1].split("/"))
        shard, part = (k, n), sys.argv[i + 2]
    t0 = time.time()
    g = synth.make_graph(name)
    print(f"graph {name}: {g.n_nodes} nodes {g.n_arcs} arcs abar {g.abar} "
          f"({time.time() - t0:.0f} s)", flush=True)
    o = oracle.Oracle(g, check=False)
    if node:
        act = o.activation(g.abar, 0.5, oracle.MODE_NODE)[0]
    else:
        act = o.activation(g.abar, 0.5)
    act_sha = hashlib.sha256(np.ascontiguousarray(act, np.uint8).tobytes()).hexdigest()
    print(f"activation levels ({time.time() - t0:.0f} s)", flush=True)
    qs = synth.make_queries(g, name)
    stride = max(1, len(qs) // count)
    picked = list(range(0, len(qs), stride))[:count]
    if shard:
        picked = picked[shard[0]::shard[1]]
    out = {"workload": name, "alpha": 0.5, "abar_x100": g.abar_x100, "n_arcs": g.n_arcs,
           "act_sha256": act_sha, "queries": []}
    if node:
        out["mode"] = "node"
    for i in picked:
        q = qs[i]
        t1 = time.time()
        res = o.query(act, q, lean=True)
        entry = {"index": i, "central": list(q.central), "marginal": list(q.marginal),
                 "k": q.k, "w": q.w, "max_level": q.max_level}
        entry.update(summarize(res))
        out["queries"].append(entry)
        print(f"query {i}: {len(res['results'])} results, e_arc "
              f"{res['stats'][0]['e_arc'] + res['stats'][1]['e_arc']} ({time.time() - t1:.1f} s)",
              flush=True)
    if part:
        with open(part, "w") as f:
            json.dump(out, f)
        print(f"wrote {part}")
    else:
        print(f"wrote {write(name + ('_node' if node else ''), out)} ({time.time() - t0:.0f} s total)")


if __name__ == "__main__":
    main()
