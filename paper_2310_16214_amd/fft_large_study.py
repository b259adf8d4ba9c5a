"""Large-N FFT study on the current GPU: the two-pass plans of
fft_batched_large for N = 2^15 .. 2^23 at 256 MiB per call (2^25 / N
problems), each method of tune_fft_large (exhaustive, analytical, learned)
against the exhaustive best, the Phi metric of Sec. VI over the sizes, the
default plan, and the best plan's throughput against the 8 TB/s HBM peak and
against the library's streaming reference for one pass's bytes.

Each plan is timed as the median of `reps` whole two-pass calls on rotating
buffer sets (no launch reads data a previous one left in the caches).  HBM
bytes: each pass reads and writes every element once, 32 B per element for
the call; the FFT's algorithmic minimum is 16 B per element (one read, one
write), the figure `frac_alg` is against.

    python -m paper_2310_16214_amd.fft_large_study --out-dir profiles
    rocprofv3 --kernel-trace --stats ... -- python3 -m paper_2310_16214_amd.fft_large_study \
        --replay profiles/fft_large_study.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0


def stream_gbs(ppx, torch, nbytes, dev, reps=10):
    """Streaming reference for one pass: nbytes in, nbytes out (median)."""
    sets = [[torch.empty(nbytes // 4, dtype=torch.float32, device=dev) for _ in range(2)] for _ in range(3)]
    ts = []
    for r in range(reps + 2):
        a, b = sets[r % 3]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ppx.stream_reference([a], b, nbytes)
        e1.record()
        e1.synchronize()
        if r >= 2:
            ts.append(e0.elapsed_time(e1) * 1e3)
    ts.sort()
    return 2 * nbytes / ts[len(ts) // 2] / 1e3


def traffic_table(fetch_csv, write_csv):
    """Per-kernel HBM traffic of a --replay run from two rocprofv3 counter
    CSVs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what it
    reads for the replay's first dispatch, a plain 256 MiB device copy."""
    import csv
    from collections import OrderedDict
    per, copy = OrderedDict(), {}
    for path in (fetch_csv, write_csv):
        for r in csv.DictReader(open(path)):
            name, cn, v = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
            if "copyBuffer" in name:
                copy[cn] = max(copy.get(cn, 0.0), v)
            elif "k_fft_tile" in name:
                per.setdefault(name.split("(")[0].replace("void ", ""), {}).setdefault(cn, []).append(v)
    mib = 256.0
    fs, ws = mib * 1024 / copy["FETCH_SIZE"], mib * 1024 / copy["WRITE_SIZE"]
    out = [f"Calibration: the replay's first dispatch is a plain 256 MiB device copy; it reads FETCH_SIZE "
           f"{copy['FETCH_SIZE']:.0f} KiB and WRITE_SIZE {copy['WRITE_SIZE']:.0f} KiB, so the counters are scaled "
           f"by x{fs:.3f} (reads) and x{ws:.3f} (writes). Each pass moves 256 MiB in each direction (algorithmic).",
           "", "| kernel | dispatches | read MiB | write MiB | read / 256 MiB | write / 256 MiB |",
           "|---|---|---|---|---|---|"]
    for k, c in per.items():
        rd = sum(c["FETCH_SIZE"]) / len(c["FETCH_SIZE"]) * fs / 1024
        wr = sum(c["WRITE_SIZE"]) / len(c["WRITE_SIZE"]) * ws / 1024
        out.append(f"| `{k}` | {len(c['FETCH_SIZE'])} | {rd:.1f} | {wr:.1f} | {rd / mib:.3f} | {wr / mib:.3f} |")
    return out


def report(study_json, stats_csv="", fetch_csv="", write_csv=""):
    """Markdown summary of a study JSON (and of a rocprofv3 kernel-stats CSV
    and FETCH_SIZE / WRITE_SIZE counter CSVs of a --replay run, when given)."""
    import csv
    d = json.load(open(study_json))
    plan = lambda p: f"n1=2^{p[0]} A:r{p[1]}/t{p[3]} B:r{p[2]}/t{p[4]}"  # noqa: E731
    out = ["| N | plans | exhaustive best | us | GElem/s | HBM GB/s (32 B/elem) | of peak | of stream | "
           "analytical (e) | learned (e, evals) | default us |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in d["records"]:
        out.append(f"| 2^{r['n'].bit_length() - 1} | {r['plans']} | {plan(r['exhaustive']['plan'])} | "
                   f"{r['exhaustive']['us']:.1f} | {r['gelem_s']:.0f} | {r['gbs_hbm']:.0f} | {r['frac_hbm']:.2f} | "
                   f"{r['hbm_frac_of_stream_ref']:.2f} | {plan(r['analytical']['plan'])} ({r['e_analytical']:.2f}) | "
                   f"{plan(r['learned']['plan'])} ({r['e_learned']:.2f}, {r['learned']['evals']}) | "
                   f"{r['default']['us']:.1f} |")
    sm = d["summary"]
    out += ["", f"Phi analytical {sm['phi_analytical']:.3f}, Phi learned {sm['phi_learned']:.3f} "
                f"(mean {sm['mean_learned_evals']:.1f} timed plans per size); {sm['reps']} timed calls per plan."]
    if stats_csv:
        out += ["", "Per-pass kernel times of the exhaustive-best plans (rocprofv3 --stats, 10 calls per size):", "",
                "| kernel | calls | mean us |", "|---|---|---|"]
        for r in csv.DictReader(open(stats_csv)):
            if "k_fft_tile" in r["Name"]:
                name = r["Name"].split("(")[0].replace("void ", "")
                out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} |")
    if fetch_csv and write_csv:
        out += [""] + traffic_table(fetch_csv, write_csv)
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--sizes", default="15,16,17,18,19,20,21,22,23")
    ap.add_argument("--report", nargs="+", default=None,
                    metavar=("STUDY_JSON", "KERNEL_STATS_CSV [FETCH_CSV WRITE_CSV]"),
                    help="print the markdown summary of a study (no GPU)")
    ap.add_argument("--plans", default="", metavar="STUDY_JSON",
                    help="print the exhaustive-best plans of a study as tune-cache lines")
    ap.add_argument("--replay", default="",
                    help="a study JSON: only run the exhaustive-best plan of each size in --sizes 10 times, "
                         "after one 256 MiB copy (for a kernel trace or counter runs)")
    args = ap.parse_args()
    if args.plans:
        for r in json.load(open(args.plans))["records"]:
            p = r["exhaustive"]["plan"]
            print(f"gfx950 plan {r['n']} {p[0]} {p[1]} {p[2]} {p[3]} {p[4]} {r['exhaustive']['us']:.3f} 0")
        return
    if args.report:
        report(*args.report)
        return
    import torch
    from paper_2310_16214_amd import ppx
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    if args.replay:
        # a plain 256 MiB device copy first: the calibration dispatch for
        # FETCH_SIZE / WRITE_SIZE counter runs of the replay
        a = torch.zeros(1 << 25, dtype=torch.complex64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        sizes = {int(v) for v in args.sizes.split(",")}
        for rec in json.load(open(args.replay))["records"]:
            n, batch = rec["n"], rec["batch"]
            if n.bit_length() - 1 not in sizes:
                continue
            plan = ppx.make_plan(*rec["exhaustive"]["plan"])
            x = torch.zeros(n * batch, dtype=torch.complex64, device=dev)
            y = torch.empty_like(x)
            for _ in range(10):
                ppx.fft_batched_large(x, y, n, batch, -1, plan)
            torch.cuda.synchronize()
            print(f"replayed n={n} plan={plan}", flush=True)
            del x, y
        return
    records = []
    for ln in (int(v) for v in args.sizes.split(",")):
        n = 1 << ln
        batch = (1 << 25) >> ln
        t0 = time.time()
        ex, ex_us, ex_ev, trace = ppx.tune_fft_large(n, batch, 0, reps=args.reps)
        times = {p.as_tuple(): us for p, us in trace}
        an, _, _, _ = ppx.tune_fft_large(n, batch, 1, reps=args.reps)
        le, _, le_ev, _ = ppx.tune_fft_large(n, batch, 2, reps=args.reps)
        d = ppx.default_fft_plan(n)
        best = min(times.values())
        rec = dict(n=n, batch=batch, plans=len(times),
                   exhaustive=dict(plan=ex.as_tuple(), us=times[ex.as_tuple()]),
                   analytical=dict(plan=an.as_tuple(), us=times[an.as_tuple()]),
                   learned=dict(plan=le.as_tuple(), us=times[le.as_tuple()], evals=le_ev),
                   default=dict(plan=d.as_tuple(), us=times[d.as_tuple()]),
                   all=[[list(k), v] for k, v in sorted(times.items())])
        rec["e_analytical"] = best / rec["analytical"]["us"]
        rec["e_learned"] = best / rec["learned"]["us"]
        rec["tuned_vs_default"] = rec["default"]["us"] / best
        elems = n * batch
        rec["gelem_s"] = elems / best / 1e3
        rec["gbs_alg"] = 16 * elems / best / 1e3
        rec["gbs_hbm"] = 32 * elems / best / 1e3
        rec["frac_alg"] = rec["gbs_alg"] / PEAK_GBS
        rec["frac_hbm"] = rec["gbs_hbm"] / PEAK_GBS
        rec["stream_ref_gbs"] = stream_gbs(ppx, torch, 8 * elems, dev)
        rec["hbm_frac_of_stream_ref"] = rec["gbs_hbm"] / rec["stream_ref_gbs"]
        rec["seconds"] = time.time() - t0
        records.append(rec)
        print(json.dumps({k: v for k, v in rec.items() if k != "all"}), flush=True)
    phi = lambda es: len(es) / sum(1.0 / e for e in es)  # noqa: E731
    summary = dict(phi_analytical=phi([r["e_analytical"] for r in records]),
                   phi_learned=phi([r["e_learned"] for r in records]),
                   mean_learned_evals=sum(r["learned"]["evals"] for r in records) / len(records),
                   reps=args.reps)
    print(json.dumps(summary), flush=True)
    os.makedirs(args.out_dir, exist_ok=True)
    with open(os.path.join(args.out_dir, "fft_large_study.json"), "w") as f:
        json.dump(dict(records=records, summary=summary), f)


if __name__ == "__main__":
    main()
