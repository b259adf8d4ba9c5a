"""Summarise a rocprofv3 kernel trace (CSV) of bench.py into a short text table.

Dispatches are grouped by (kernel, grid size, workgroup size), which
identifies one call of the benchmark step, and reported with their count and
mean / median duration; the benchmark's own per-call event timings (its
--detail JSONL) are placed beside them when given.

    python -m paper_2310_16214_amd.prof_summary TRACE.csv [--detail bench_detail.jsonl]
        [--stats KERNEL_STATS.csv] [--command "..."] [--top 20]
"""
from __future__ import annotations

import argparse
import csv
import json
import re
import statistics

from paper_2310_16214_amd.traffic import kernel_name_prefix


def short(name):
    name = re.sub(r"HIP_vector_type<float, 2u>", "float2", name)
    return re.sub(r"\(.*\)$", "", name).replace("void ", "")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--detail", default="")
    ap.add_argument("--stats", default="")
    ap.add_argument("--command", default="")
    ap.add_argument("--top", type=int, default=25)
    args = ap.parse_args()
    groups = {}
    with open(args.trace) as f:
        for r in csv.DictReader(f):
            if "ppx::" not in r["Kernel_Name"]:
                continue
            key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]),
                   int(r["LDS_Block_Size"]), int(r["VGPR_Count"]))
            groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    detail = []
    if args.detail:
        detail = [json.loads(x) for x in open(args.detail)]
    lines = []
    if args.command:
        lines.append(f"command: {args.command}")
    lines.append("per call of the step (rocprofv3 kernel trace; 'events' = bench.py's HIP-event mean)")
    lines.append(f"{'kernel':34s} {'grid':>9s} {'L':>5s} {'LDS':>7s} {'VGPR':>5s} {'n':>4s} "
                 f"{'mean_us':>9s} {'med_us':>9s}  call / events_us")
    rows = sorted(groups.items(), key=lambda kv: -statistics.mean(kv[1]))[:args.top]
    for (k, grid, wg, lds, vgpr), ts in rows:
        calls = []
        for d in detail:
            c = d["cfg"]
            if not k.startswith("ppx::" + kernel_name_prefix(d)) or c["threads_per_block"] != wg:
                continue
            persistent = "_np<" in k or "_pipe<" in k  # launched with the resident grid
            if persistent or grid // wg == -(-d["batch"] // c["problems_per_block"]):
                calls.append(f"{d['op']} n={d['n']} {d['dtype']} / {d['us']:.1f}")
        match = "; ".join(calls)
        lines.append(f"{k[:34]:34s} {grid // wg:9d} {wg:5d} {lds:7d} {vgpr:5d} {len(ts):4d} "
                     f"{statistics.mean(ts):9.2f} {statistics.median(ts):9.2f}  {match}")
    if args.stats:
        lines.append("")
        lines.append("rocprofv3 --stats (all calls of a kernel instantiation pooled)")
        with open(args.stats) as f:
            for i, r in enumerate(csv.DictReader(f)):
                if i >= 12:
                    break
                lines.append(f"{short(r['Name'])[:40]:40s} calls={r['Calls']:>5s} "
                             f"avg_us={float(r['AverageNs']) / 1e3:9.2f} pct={float(r['Percentage']):6.2f}")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
