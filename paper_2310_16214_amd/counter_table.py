"""Summarise rocprofv3 counter runs (CSV) of ``one_call`` into a short table.

Each counter CSV is one pass of ``rocprofv3 --pmc ... --output-format csv``
over the same ``one_call`` command; rows are per (dispatch, counter).  The
dispatches of the library's kernels are grouped by (kernel, grid, workgroup)
in the order they first run, which is the order of the shapes in the calls
file that ``one_call --out`` wrote, and each counter is averaged over a
group's dispatches.  FETCH_SIZE / WRITE_SIZE (KiB) are scaled to bytes by
what they read for the 256 MiB reference copy (``one_call --copy-ref``).

Derived columns, per call:
  traffic / algorithmic -- counted HBM bytes over the call's inputs read once
      and outputs written once;
  VALU floor us -- SQ_INSTS_VALU wave instructions at four cycles each, the
      transcendental ones among them (SQ_INSTS_VALU_TRANS_F, quarter rate) at
      sixteen, spread evenly over the 1024 SIMDs at 2.4 GHz: the time the
      vector ALUs alone would need;
  wait LDS / wave cycles and wait any / wave cycles -- the share of the waves'
      lifetime spent waiting on LDS instructions, and on anything.

    python -m paper_2310_16214_amd.counter_table CALLS.jsonl PASS.csv [PASS.csv ...]
        [--trace KERNEL_TRACE.csv] [--command "..."]
"""
from __future__ import annotations

import argparse
import csv
import json
import re
from collections import OrderedDict

SIMDS, CLOCK_MHZ = 1024, 2400.0
COPY_BYTES = 256 * 2 ** 20


def _short(name):
    name = re.sub(r"\(.*\)$", "", name).replace("void ", "")
    return name.replace("HIP_vector_type<float, 2u>", "float2")


def load(paths):
    """{(kernel, grid, wg): {counter: [values per dispatch]}} in first-run
    order, and the reference copy's readings."""
    groups = OrderedDict()
    copy = {}
    for p in paths:
        with open(p) as f:
            for r in csv.DictReader(f):
                name, val = r["Kernel_Name"], float(r["Counter_Value"])
                key = (_short(name), int(r["Grid_Size"]), int(r["Workgroup_Size"]))
                if "copyBuffer" in name:
                    big = copy.setdefault(r["Counter_Name"], [0.0])
                    big[0] = max(big[0], val)
                    continue
                if not name.startswith("ppx::") and "ppx::" not in name:
                    continue
                groups.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(val)
    return groups, copy


def trace_means(path):
    """Mean kernel duration (us) per (kernel, grid, wg) from a kernel trace."""
    acc = OrderedDict()
    with open(path) as f:
        for r in csv.DictReader(f):
            key = (_short(r["Kernel_Name"]), int(r.get("Grid_Size") or r["Grid_Size_X"]),
                   int(r.get("Workgroup_Size") or r["Workgroup_Size_X"]))
            if "ppx::" not in key[0]:
                continue
            acc.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("calls")
    ap.add_argument("passes", nargs="+")
    ap.add_argument("--trace", default="")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    calls = [json.loads(x) for x in open(args.calls) if x.strip()]
    groups, copy = load(args.passes)
    durs = trace_means(args.trace) if args.trace else {}
    fs = COPY_BYTES / (copy["FETCH_SIZE"][0] * 1024) if "FETCH_SIZE" in copy else None
    ws = COPY_BYTES / (copy["WRITE_SIZE"][0] * 1024) if "WRITE_SIZE" in copy else None
    keys = list(groups)
    if len(keys) != len(calls):
        raise SystemExit(f"{len(keys)} kernel groups for {len(calls)} calls: run one kernel per shape")
    if args.command:
        print(f"command: `{args.command}`\n")
    if fs:
        print(f"FETCH_SIZE scale {fs:.4f}, WRITE_SIZE scale {ws:.4f} (256 MiB reference copy)\n")
    print("| call | kernel | grid | L | us | GB/s (frac of 8 TB/s) | traffic / algorithmic | VALU insts per wave |"
          " of which transcendental | VALU floor us | LDS insts per wave | wait LDS / wave cycles |"
          " wait any / wave cycles | LDS bank conflicts per LDS inst |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for call, key in zip(calls, keys):
        c = {k: sum(v) / len(v) for k, v in groups[key].items()}
        us = durs.get(key)
        alg = call["algorithmic_bytes"]
        gbs = f"{alg / us / 1e3:.0f} ({alg / us / 8e6:.3f})" if us else "-"
        traffic = "-"
        if fs and "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            traffic = f"{(c['FETCH_SIZE'] * fs + c['WRITE_SIZE'] * ws) * 1024 / alg:.3f}"
        waves = c.get("SQ_WAVES")
        per_wave = lambda k: f"{c[k] / waves:.0f}" if waves and k in c else "-"  # noqa: E731
        trans = c.get("SQ_INSTS_VALU_TRANS_F", 0.0)
        floor = (f"{((c['SQ_INSTS_VALU'] - trans) * 4 + trans * 16) / SIMDS / CLOCK_MHZ:.1f}"
                 if "SQ_INSTS_VALU" in c else "-")
        wc = c.get("SQ_WAVE_CYCLES")
        frac = lambda k: f"{c[k] / wc:.2f}" if wc and k in c else "-"  # noqa: E731
        bank = (f"{c['SQ_LDS_BANK_CONFLICT'] / c['SQ_INSTS_LDS']:.2f}"
                if c.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in c else "-")
        cfg = call.get("cfg") or {}
        label = f"{call['op']} {call['dtype']} n={call['n']} x {call['batch']}"
        if call["op"] == "tridiag":
            label += f" {call['shape'].split(':')[3] if call['shape'].count(':') >= 3 else 'cr'} (algo {cfg.get('algo')})"
        print(f"| {label} | `{key[0]}` | {key[1] // key[2]} | {key[2]} | {us:.2f} |" if us else
              f"| {label} | `{key[0]}` | {key[1] // key[2]} | {key[2]} | - |", end="")
        print(f" {gbs} | {traffic} | {per_wave('SQ_INSTS_VALU')} | {per_wave('SQ_INSTS_VALU_TRANS_F')} | {floor} |"
              f" {per_wave('SQ_INSTS_LDS')} |"
              f" {frac('SQ_WAIT_INST_LDS')} | {frac('SQ_WAIT_ANY')} | {bank} |")


if __name__ == "__main__":
    main()
