"""Summarise rocprofv3 counter runs (CSV) of ``one_call`` into a short table.

Each counter CSV is one pass of ``rocprofv3 --pmc ... --output-format csv``
over the same ``one_call`` command; rows are per (dispatch, counter).  The
library's dispatches, in dispatch order, are assigned to the calls of the
calls file that ``one_call --out`` wrote: each call ran its ``reps`` times,
launching ``kernels`` kernels each time (a two-pass FFT call: pass A then
pass B, one table row per pass, each with the call's algorithmic bytes, since
both passes read and write every value once).  Each counter is averaged over
a row's dispatches.  FETCH_SIZE / WRITE_SIZE (KiB) are scaled to bytes by
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


def _rows(calls):
    """The (call index, kernel index) of each library dispatch, in order."""
    out = []
    for ci, call in enumerate(calls):
        for _ in range(call.get("reps", 5)):
            out += [(ci, k) for k in range(call.get("kernels", 1))]
    return out


def _dispatches(path, value_of):
    """{dispatch id: (key, name, row value)} of one CSV."""
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            key = (_short(name), int(r.get("Grid_Size") or r["Grid_Size_X"]),
                   int(r.get("Workgroup_Size") or r["Workgroup_Size_X"]))
            per.setdefault(int(r["Dispatch_Id"]), (key, name, []))[2].append(value_of(r))
    return per


def load(paths, calls):
    """({(call, kernel): (key, {counter: [values per dispatch]})}, the
    reference copy's readings)."""
    rows = _rows(calls)
    groups = OrderedDict()
    copy = {}
    for p in paths:
        per = _dispatches(p, lambda r: (r["Counter_Name"], float(r["Counter_Value"])))
        lib = [d for d in sorted(per) if "ppx::" in per[d][1]]
        if len(lib) != len(rows):
            raise SystemExit(f"{p}: {len(lib)} library dispatches for {len(rows)} expected (calls x reps x kernels)")
        for d in sorted(per):
            key, name, vals = per[d]
            if "copyBuffer" in name:
                for cn, v in vals:
                    big = copy.setdefault(cn, [0.0])
                    big[0] = max(big[0], v)
        for row, d in zip(rows, lib):
            key, _, vals = per[d]
            g = groups.setdefault(row, (key, {}))[1]
            for cn, v in vals:
                g.setdefault(cn, []).append(v)
    return groups, copy


def trace_means(path, calls):
    """Mean kernel duration (us) per (call, kernel) from a kernel trace."""
    rows = _rows(calls)
    per = _dispatches(path, lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lib = [d for d in sorted(per) if "ppx::" in per[d][1]]
    if len(lib) != len(rows):
        raise SystemExit(f"{path}: {len(lib)} library dispatches for {len(rows)} expected")
    acc = OrderedDict()
    for row, d in zip(rows, lib):
        acc.setdefault(row, []).append(per[d][2][0])
    return {k: sum(v) / len(v) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("calls")
    ap.add_argument("passes", nargs="+")
    ap.add_argument("--trace", default="")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    calls = [json.loads(x) for x in open(args.calls) if x.strip()]
    groups, copy = load(args.passes, calls)
    durs = trace_means(args.trace, calls) if args.trace else {}
    fs = COPY_BYTES / (copy["FETCH_SIZE"][0] * 1024) if "FETCH_SIZE" in copy else None
    ws = COPY_BYTES / (copy["WRITE_SIZE"][0] * 1024) if "WRITE_SIZE" in copy else None
    if args.command:
        print(f"command: `{args.command}`\n")
    if fs:
        print(f"FETCH_SIZE scale {fs:.4f}, WRITE_SIZE scale {ws:.4f} (256 MiB reference copy)\n")
    print("| call | kernel | grid | L | us | GB/s (frac of 8 TB/s) | traffic / algorithmic | VALU insts per wave |"
          " of which transcendental | VALU floor us | LDS insts per wave | wait LDS / wave cycles |"
          " wait any / wave cycles | LDS bank conflicts per LDS inst |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for row, (key, vals) in groups.items():
        call = calls[row[0]]
        tag = "" if call.get("kernels", 1) == 1 else f" pass {'AB'[row[1]]}"
        c = {k: sum(v) / len(v) for k, v in vals.items()}
        us = durs.get(row)
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
        if "plan" in call:
            pl = call["plan"]
            label += (f" (n1 = 2^{pl['log2_n1']}, A r{pl['radix_a']}/t{pl['tile_a']},"
                      f" B r{pl['radix_b']}/t{pl['tile_b']}){tag}")
        print(f"| {label} | `{key[0]}` | {key[1] // key[2]} | {key[2]} | {us:.2f} |" if us else
              f"| {label} | `{key[0]}` | {key[1] // key[2]} | {key[2]} | - |", end="")
        print(f" {gbs} | {traffic} | {per_wave('SQ_INSTS_VALU')} | {per_wave('SQ_INSTS_VALU_TRANS_F')} | {floor} |"
              f" {per_wave('SQ_INSTS_LDS')} |"
              f" {frac('SQ_WAIT_INST_LDS')} | {frac('SQ_WAIT_ANY')} | {bank} |")


if __name__ == "__main__":
    main()
