"""Tuning study on the current GPU: exhaustive vs analytical vs learned.

For every operation and size of the benchmark sweeps it runs the three tuning
methods of the library (each candidate timed as the median of `reps`
launches, rotating buffer sets so that no launch reads cached data), times
the plain default configuration, and reports per size the efficiency of each
method against the exhaustive best and, over all sizes, the harmonic-mean
Phi metric of Sec. VI of arXiv:2310.16214.  It also measures "batched vs
plain": the batched launch against one launch per problem.

The exhaustive winners are written to a tune cache file (loaded by the
benchmark and usable through ppx.load_tune_cache) and the full record to a
JSON report.

    python -m paper_2310_16214_amd.tune_sweep --ops fft --out-dir profiles
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

METHOD_NAMES = {0: "exhaustive", 1: "analytical", 2: "learned"}


def sweeps(ops):
    from paper_2310_16214_amd import ppx
    out = []
    if "fft" in ops:
        for ln in range(4, 15):
            out.append(("fft", ppx.OP_FFT, ppx.C64, 1 << ln, (1 << 25) >> ln, -1))
    if "scan" in ops:
        for code in (ppx.I32, ppx.F32, ppx.F64):
            for ln in range(5, 14):
                out.append(("scan", ppx.OP_SCAN, code, 1 << ln, (1 << 24) >> ln, -1))
    if "tridiag" in ops:
        for code in (ppx.F32, ppx.F64):
            for algo in (ppx.TRI_CR, ppx.TRI_PCR, ppx.TRI_CR_PCR, ppx.TRI_WM, ppx.TRI_LF):
                for ln in range(5, 11):
                    out.append(("tridiag", ppx.OP_TRIDIAG, code, 1 << ln, (1 << 22) >> ln, algo))
    return out


def scan_forms_us(ppx, dtype, n, batch, cfg, reps, dev):
    """Median microseconds of the inclusive and of the exclusive scan with one
    configuration, each launch timed with events on the current stream and
    reading a different input set (>= 1 GiB rotated, so no launch reads
    cached data)."""
    import statistics

    import torch
    t = {ppx.I32: torch.int32, ppx.F32: torch.float32, ppx.F64: torch.float64}[dtype]
    set_bytes = 2 * n * batch * (8 if dtype == ppx.F64 else 4)
    nsets = max(2, min(16, -(-(1 << 30) // set_bytes)))
    xs = [torch.ones((batch, n), dtype=t, device=dev) for _ in range(nsets)]
    ys = [torch.empty_like(x) for x in xs]
    out = {}
    for excl in (False, True):
        f = ppx.scan_exclusive_batched if excl else ppx.scan_batched
        for w in range(3):
            f(xs[w % nsets], ys[w % nsets], n, batch, dtype, cfg)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for r in range(reps):
            i = (r + 3) % nsets
            ev[r][0].record()
            f(xs[i], ys[i], n, batch, dtype, cfg)
            ev[r][1].record()
        torch.cuda.synchronize()
        out["excl" if excl else "incl"] = statistics.median(a.elapsed_time(b) * 1e3 for a, b in ev)
    del xs, ys
    torch.cuda.empty_cache()
    return out


def plain_time_us(ppx, op, dtype, n, launches, dev):
    """Per-problem time of one launch per problem with the default config."""
    import torch
    cfg = ppx.default_config(op, dtype, n)
    if op == ppx.OP_FFT:
        x = torch.zeros((launches, n), dtype=torch.complex64, device=dev)
        y = torch.empty_like(x)
        run = lambda i: ppx.fft_batched(x[i], y[i], n, 1, -1, cfg)  # noqa: E731
    elif op == ppx.OP_SCAN:
        t = {ppx.I32: torch.int32, ppx.F32: torch.float32, ppx.F64: torch.float64}[dtype]
        x = torch.zeros((launches, n), dtype=t, device=dev)
        y = torch.empty_like(x)
        run = lambda i: ppx.scan_batched(x[i], y[i], n, 1, dtype, cfg)  # noqa: E731
    else:
        t = torch.float32 if dtype == ppx.F32 else torch.float64
        a = torch.zeros((launches, n), dtype=t, device=dev)
        b = torch.ones_like(a)
        y = torch.empty_like(a)
        run = lambda i: ppx.tridiag_batched(a[i], b[i], a[i], b[i], y[i], n, 1, dtype, cfg)  # noqa
    for i in range(min(20, launches)):
        run(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(launches):
        run(i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e6 / launches


def restricted_study(ppx, records, max_gb):
    """The three methods over a smaller search space, from the exhaustive
    run's timings: candidates with at most max_gb problems per workgroup
    (the benchmark configuration's "problems/block 1..16").  Exhaustive is
    the best timed candidate of the subset; analytical the library's
    selection rule applied to the subset (ppx_analytical_select); learned the
    library's Bayesian search (same stopping rule, seed and features as
    tune()) run over the subset with the measured times as its evaluations.
    Returns per-size records and Phi per group."""
    out, groups = [], {}
    for r in records:
        sub = [(c, us) for c, us in r["all"] if c[3] <= max_gb]
        if not sub:
            continue
        cands = [ppx.Config(*c) for c, _ in sub]
        times = {tuple(c): us for c, us in sub}
        best = min(times.values())
        ka = ppx.analytical_select(r["op_code"], r["dtype"], r["n"], r["batch"], cands)
        kb, order, _ = ppx.bo_search(cands, lambda c: times[tuple(c.as_tuple())], patience=5,
                                     min_rel=0.01, seed=0x231016214)
        rec = dict(op=r["op"], dtype=r["dtype"], algo=r["algo"], n=r["n"], space=len(sub),
                   best_cfg=min(sub, key=lambda t: t[1])[0], best_us=best,
                   analytical_cfg=sub[ka][0], e_analytical=best / sub[ka][1],
                   learned_cfg=sub[kb][0], e_learned=best / sub[kb][1], learned_evals=len(order),
                   e_full_space_best=r["exhaustive"]["us"] / best)
        out.append(rec)
        groups.setdefault((r["op"], r["dtype"], r["algo"]), []).append(rec)
    summary = [dict(op=k[0], dtype=k[1], algo=k[2], max_problems_per_block=max_gb,
                    sizes=[x["n"] for x in v], phi_analytical=ppx.phi([x["e_analytical"] for x in v]),
                    phi_learned=ppx.phi([x["e_learned"] for x in v]),
                    evals_learned=[x["learned_evals"] for x in v])
               for k, v in groups.items()]
    return out, summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ops", default="fft,scan,tridiag")
    ap.add_argument("--reps", type=int, default=100)
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--cache", default=os.path.join(ROOT, "paper_2310_16214_amd", "tuned",
                                                     "mi355x.txt"))
    ap.add_argument("--plain-launches", type=int, default=2000)
    ap.add_argument("--max-gb", type=int, default=16,
                    help="also report the methods over candidates with at most this many problems "
                         "per workgroup (0: skip)")
    args = ap.parse_args()
    import torch

    from paper_2310_16214_amd import ppx
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    ops = set(args.ops.split(","))
    if os.path.exists(args.cache):
        ppx.load_tune_cache(args.cache)
    records = []
    for name, op, dtype, n, batch, algo in sweeps(ops):
        rec = dict(op=name, op_code=op, dtype=dtype, n=n, batch=batch, algo=algo)
        t0 = time.time()
        for method in (ppx.TUNE_ANALYTICAL, ppx.TUNE_LEARNED, ppx.TUNE_EXHAUSTIVE):
            rep, trace = ppx.tune_ex(op, dtype, n, batch, method, algo=algo, reps=args.reps)
            rec[METHOD_NAMES[method]] = dict(cfg=rep.best.as_dict(), us=rep.best_us,
                                             evals=rep.evals_used, space=rep.ncands)
            if method == ppx.TUNE_EXHAUSTIVE:
                rec["all"] = [(c.as_tuple(), us) for c, us in trace]
        dflt = ppx.default_config(op, dtype, n)
        if algo >= 0:
            dflt.algo = algo
            dflt.lds_elems = 0
            if not ppx.config_valid(op, dtype, n, dflt):
                # in-wave only (Wang & Mou): one system per workgroup with the
                # fewest equations per lane
                dflt = min((c for c in ppx.enumerate_configs(op, dtype, n)
                            if c.algo == algo and c.problems_per_block == 1),
                           key=lambda c: c.elems_per_thread)
        rec["default"] = dict(cfg=dflt.as_dict(), us=ppx.time_config(op, dtype, n, batch, dflt,
                                                                     args.reps))
        # efficiency as the paper defines it: performance of the method's
        # configuration as a fraction of the best observed, both read from the
        # exhaustive run's timings; the re-timed ratio is kept beside it
        table = {tuple(c): us for c, us in rec["all"]}
        best = min(table.values())
        rec["exhaustive"]["us"] = best
        for m in ("analytical", "learned"):
            key = tuple(rec[m]["cfg"][f] for f in ("radix", "elems_per_thread", "threads_per_block",
                                                   "problems_per_block", "lds_elems", "algo"))
            rec["e_" + m] = best / table[key]
            rec["e_" + m + "_retimed"] = best / rec[m]["us"]
        rec["tuned_vs_default"] = rec["default"]["us"] / best
        rec["gelem_s"] = n * batch / best / 1e3
        if op == ppx.OP_SCAN:
            c = rec["exhaustive"]["cfg"]
            cfg = ppx.make_config(c["radix"], c["threads_per_block"], c["problems_per_block"], c["algo"])
            rec["forms_us"] = scan_forms_us(ppx, dtype, n, batch, cfg, args.reps, dev)
        if args.plain_launches > 0:
            k = min(args.plain_launches, batch)
            per = plain_time_us(ppx, op, dtype, n, k, dev)
            rec["plain_us_per_problem"] = per
            rec["batched_vs_plain"] = per * batch / best
        rec["seconds"] = time.time() - t0
        records.append(rec)
        print(json.dumps({k: v for k, v in rec.items() if k != "all"}), flush=True)
    ppx.save_tune_cache(args.cache)

    # Phi per (op, dtype, algo) group over its sizes
    groups = {}
    for r in records:
        groups.setdefault((r["op"], r["dtype"], r["algo"]), []).append(r)
    summary = []
    for (opname, dtype, algo), rs in groups.items():
        summary.append(dict(op=opname, dtype=dtype, algo=algo, sizes=[r["n"] for r in rs],
                            phi_analytical=ppx.phi([r["e_analytical"] for r in rs]),
                            phi_learned=ppx.phi([r["e_learned"] for r in rs]),
                            evals_learned=[r["learned"]["evals"] for r in rs],
                            space=[r["exhaustive"]["space"] for r in rs],
                            tuned_vs_default=[r["tuned_vs_default"] for r in rs],
                            batched_vs_plain=[r.get("batched_vs_plain") for r in rs]))
        print(json.dumps(summary[-1]), flush=True)
    restricted = None
    if args.max_gb > 0:
        rrec, rsum = restricted_study(ppx, records, args.max_gb)
        for x in rsum:
            print(json.dumps(x), flush=True)
        restricted = dict(records=rrec, summary=rsum)
    os.makedirs(args.out_dir, exist_ok=True)
    tag = "_".join(sorted(ops))
    with open(os.path.join(args.out_dir, f"tuning_{tag}.json"), "w") as f:
        json.dump(dict(records=records, summary=summary, reps=args.reps, restricted=restricted), f)


if __name__ == "__main__":
    main()
