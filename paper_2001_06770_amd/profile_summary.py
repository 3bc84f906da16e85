"""Summaries of rocprofv3 output for the committed profiles.

``stats``: the per-kernel table of a ``--kernel-trace --stats`` run
(``*_kernel_stats.csv``) as markdown, longest total first.

``traffic``: bytes per expansion launch from two ``--pmc`` runs of the same
benchmark command, one collecting FETCH_SIZE and one WRITE_SIZE (KiB per
dispatch, ``*_counter_collection.csv``).  Each counter is summed over every
dispatch of the kernel, scaled by the factor a plain device copy gives for it
(2.0 for FETCH_SIZE, 1.0 for WRITE_SIZE: a 1 GiB copy reads as 512 MiB of
FETCH_SIZE and writes as 1 GiB of WRITE_SIZE), and divided by the number of
launches the benchmark timed in that run (its JSON line, ``roofline.launches``),
so that it compares with the line's per-launch algorithmic bytes.  The record
carries the SHA-256 of the kernel's source file: the benchmark uses it only
while the source is unchanged.

usage:
  python -m paper_2001_06770_amd.profile_summary stats RUN_kernel_stats.csv [--top N]
  python -m paper_2001_06770_amd.profile_summary traffic --kernel NAME --source FILE.hip
      --workload W --fetch F.csv --write W.csv --bench-json B.json --out OUT.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
FETCH_SCALE = 2.0
WRITE_SCALE = 1.0


def _col(row: dict, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def stats_table(path: str, top: int) -> str:
    with open(path, newline="") as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(_col(r, "TotalDurationNs")))
    out = ["| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = _col(r, "Name", "Kernel_Name")
        out.append(f"| `{name[:90]}` | {int(_col(r, 'Calls'))} | "
                   f"{float(_col(r, 'TotalDurationNs')) / 1e6:.2f} | "
                   f"{float(_col(r, 'AverageNs')) / 1e3:.1f} | {float(_col(r, 'Percentage')):.1f} |")
    return "\n".join(out)


def counter_sum(path: str, kernel: str, counter: str):
    """Sum of a counter (KiB) over the dispatches of kernels whose name
    contains ``kernel``, and the number of those dispatches."""
    total, disp = 0.0, set()
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if kernel not in _col(r, "Kernel_Name"):
                continue
            if _col(r, "Counter_Name") != counter:
                continue
            total += float(_col(r, "Counter_Value"))
            disp.add(_col(r, "Dispatch_Id"))
    return total, len(disp)


def bench_line(path: str) -> dict:
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])


def traffic(args) -> dict:
    fetch, nf = counter_sum(args.fetch, args.kernel, "FETCH_SIZE")
    write, nw = counter_sum(args.write, args.kernel, "WRITE_SIZE")
    launches = bench_line(args.bench_json)["roofline"]["launches"]
    with open(os.path.join(HERE, "csrc", args.source), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    fb = FETCH_SCALE * fetch * 1024.0 / launches
    wb = WRITE_SCALE * write * 1024.0 / launches
    return {"kernel": args.kernel, "workload": args.workload,
            "bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb,
            "write_bytes_per_launch": wb, "dispatches": [nf, nw], "timed_launches": launches,
            "fetch_scale": FETCH_SCALE, "write_scale": WRITE_SCALE,
            args.source.replace(".", "_") + "_sha256": sha}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--top", type=int, default=14)
    t = sub.add_parser("traffic")
    for k in ("kernel", "source", "workload", "fetch", "write", "bench_json", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.csv, args.top))
    else:
        rec = traffic(args)
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))


if __name__ == "__main__":
    sys.exit(main())
