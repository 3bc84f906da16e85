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
so that it compares with the line's per-launch algorithmic bytes.  The profiled
command runs without warm-up, so every dispatch belongs to the timed steps;
dispatches that are not timed are expansion launches queued past a run's end,
which exit at once.  The record
carries the SHA-256 of the kernel's source file: the benchmark uses it only
while the source is unchanged.

``table``: every kernel's FETCH_SIZE and WRITE_SIZE bytes (scaled as above)
and its summed dispatch time in the two counter runs, as markdown.

usage:
  python -m paper_2001_06770_amd.profile_summary stats RUN_kernel_stats.csv [--top N]
  python -m paper_2001_06770_amd.profile_summary table --fetch F.csv --write W.csv [--top N]
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


def traffic_table(fetch_csv: str, write_csv: str, top: int) -> str:
    agg = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if _col(r, "Counter_Name") != counter:
                    continue
                name = _col(r, "Kernel_Name").split("(")[0].replace("void ", "")
                d = agg.setdefault(name, {}).setdefault(counter, [0.0, set(), 0.0])
                d[0] += float(_col(r, "Counter_Value"))
                if _col(r, "Dispatch_Id") not in d[1]:
                    d[1].add(_col(r, "Dispatch_Id"))
                    d[2] += (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-6
    rows = []
    for name, d in agg.items():
        fk, fd, fms = d.get("FETCH_SIZE", [0.0, set(), 0.0])
        wk, wd, wms = d.get("WRITE_SIZE", [0.0, set(), 0.0])
        fb, wb = FETCH_SCALE * fk * 1024.0, WRITE_SCALE * wk * 1024.0
        ms = (fms + wms) / 2.0
        rows.append((ms, name, len(fd), fb, wb))
    rows.sort(key=lambda r: -r[0])
    out = ["| kernel | dispatches | ms | fetched GB | written GB | GB/s |",
           "|---|---:|---:|---:|---:|---:|"]
    for ms, name, nd, fb, wb in rows[:top]:
        gbs = (fb + wb) / 1e9 / (ms * 1e-3) if ms > 0 else 0.0
        out.append(f"| `{name[:60]}` | {nd} | {ms:.1f} | {fb / 1e9:.1f} | {wb / 1e9:.1f} | {gbs:.0f} |")
    return "\n".join(out)


def bench_line(path: str) -> dict:
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])


def traffic(args) -> dict:
    fetch, nf = counter_sum(args.fetch, args.kernel, "FETCH_SIZE")
    write, nw = counter_sum(args.write, args.kernel, "WRITE_SIZE")
    if nf != nw or nf == 0:
        raise SystemExit(f"{args.kernel}: {nf} FETCH_SIZE and {nw} WRITE_SIZE dispatches")
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
    tb = sub.add_parser("table")
    tb.add_argument("--fetch", required=True)
    tb.add_argument("--write", required=True)
    tb.add_argument("--top", type=int, default=14)
    t = sub.add_parser("traffic")
    for k in ("kernel", "source", "workload", "fetch", "write", "bench_json", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats_table(args.csv, args.top))
    elif args.cmd == "table":
        print(traffic_table(args.fetch, args.write, args.top))
    else:
        rec = traffic(args)
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))


if __name__ == "__main__":
    sys.exit(main())
