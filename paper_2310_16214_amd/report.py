"""Markdown summaries of the tuning study (tune_sweep JSON) and of the serving
benchmark (serve_bench JSON).

    python -m paper_2310_16214_amd.report tuning tuning_fft_scan_tridiag.json
    python -m paper_2310_16214_amd.report serving serve.json
"""
from __future__ import annotations

import json
import sys

DT = {0: "int32", 1: "f32", 2: "f64", 3: "c64"}
ALGO = {-1: "", 0: " CR", 1: " PCR", 2: " CR-PCR", 6: " WM", 7: " LF"}


def cfg_str(c):
    return f"r{c['radix']} P{c['elems_per_thread']} L{c['threads_per_block']} G{c['problems_per_block']}" \
           + (f" a{c['algo']}" if c['algo'] else "")


def paper_unit(r):
    """The paper's own figure for the record: GFlop/s for the FFT (5 N log2 N
    flops per problem), MData/s for the scan and MRows/s for the tridiagonal
    solvers (N * batch * 1e-6 / t)."""
    import math
    elems_per_us = r["n"] * r["batch"] / r["exhaustive"]["us"]
    if r["op"] == "fft":
        return f"{5 * math.log2(r['n']) * elems_per_us / 1e3:.0f} GFlop/s"
    return f"{elems_per_us:.0f} {'MData/s' if r['op'] == 'scan' else 'MRows/s'}"


def tuning(path):
    d = json.load(open(path))
    out = ["| op | N | exhaustive best | us | GElem/s | paper unit | analytical (e) | learned (e, evals/space) | default us | tuned/default | batched/plain |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in d["records"]:
        name = r["op"] + " " + DT[r["dtype"]] + ALGO[r["algo"]]
        out.append(f"| {name} | {r['n']} | {cfg_str(r['exhaustive']['cfg'])} | {r['exhaustive']['us']:.1f} | "
                   f"{r['gelem_s']:.0f} | {paper_unit(r)} | {cfg_str(r['analytical']['cfg'])} ({r['e_analytical']:.2f}) | "
                   f"{cfg_str(r['learned']['cfg'])} ({r['e_learned']:.2f}, {r['learned']['evals']}/{r['exhaustive']['space']}) | "
                   f"{r['default']['us']:.1f} | {r['tuned_vs_default']:.2f} | {r.get('batched_vs_plain', float('nan')):.0f} |")
    forms = [r for r in d["records"] if "forms_us" in r]
    if forms:
        out += ["", "Scan forms with the exhaustive-best configuration (events per launch, median, input sets rotated "
                    "over >= 1 GiB); algorithmic bytes = one read and one write of every element; HBM peak 8 TB/s.", "",
                "| scan | N | inclusive us | exclusive us | excl/incl | inclusive GB/s | % of HBM peak |",
                "|---|---|---|---|---|---|---|"]
        for r in forms:
            es = 8 if r["dtype"] == 2 else 4
            f = r["forms_us"]
            gbs = 2 * es * r["n"] * r["batch"] / f["incl"] / 1e3
            out.append(f"| {DT[r['dtype']]} | {r['n']} | {f['incl']:.1f} | {f['excl']:.1f} | "
                       f"{f['excl'] / f['incl']:.3f} | {gbs:.0f} | {100 * gbs / 8000:.1f} |")
    out += ["", "| group | sizes | Phi analytical | Phi learned | mean learned evals | geo-mean tuned/default |",
            "|---|---|---|---|---|---|"]
    for s in d["summary"]:
        import math
        g = math.exp(sum(math.log(v) for v in s["tuned_vs_default"]) / len(s["tuned_vs_default"]))
        out.append(f"| {s['op']} {DT[s['dtype']]}{ALGO[s['algo']]} | {s['sizes'][0]}..{s['sizes'][-1]} | "
                   f"{s['phi_analytical']:.3f} | {s['phi_learned']:.3f} | "
                   f"{sum(s['evals_learned']) / len(s['evals_learned']):.1f} | {g:.2f} |")
    rs = d.get("restricted")
    if rs:
        gb = rs["summary"][0]["max_problems_per_block"] if rs["summary"] else 16
        out += ["", f"Restricted space: candidates with at most {gb} problems per workgroup (the benchmark "
                    "configuration's problems/block 1..16), from the same exhaustive timings; analytical = the "
                    "library's selection rule over the subset, learned = its Bayesian search over the subset "
                    "with the measured times as evaluations.", "",
                "| group | sizes | Phi analytical | Phi learned | mean learned evals | subset best / full-space best |",
                "|---|---|---|---|---|---|"]
        for sm in rs["summary"]:
            recs = [x for x in rs["records"] if (x["op"], x["dtype"], x["algo"]) == (sm["op"], sm["dtype"], sm["algo"])]
            worst = min(x["e_full_space_best"] for x in recs)
            out.append(f"| {sm['op']} {DT[sm['dtype']]}{ALGO[sm['algo']]} | {sm['sizes'][0]}..{sm['sizes'][-1]} | "
                       f"{sm['phi_analytical']:.3f} | {sm['phi_learned']:.3f} | "
                       f"{sum(sm['evals_learned']) / len(sm['evals_learned']):.1f} | min {worst:.3f} |")
    print("\n".join(out))


def serving(path):
    d = json.load(open(path))
    out = [f"jobs per trace: {d['njobs']}; budget {d['budget_bytes'] / 2**30:.1f} GiB; "
           f"max launches in flight {d['max_inflight']}; mix: {d['mix']}", "",
           "| load (of fused saturation) | mode | p50 ms | p99 ms | GElem/s | % HBM peak | launches |",
           "|---|---|---|---|---|---|---|"]
    for m, r in d["saturation"].items():
        out.append(f"| burst (saturation) | {m} | {r['p50_ms']:.2f} | {r['p99_ms']:.2f} | {r['gelem_s']:.1f} | "
                   f"{100 * r['hbm_frac']:.1f} | {r['launches']} |")
    for r in d["points"]:
        out.append(f"| {r['load']:.2f} ({r['offered_jobs_per_s']:.0f} jobs/s) | {r['mode']} | {r['p50_ms']:.2f} | "
                   f"{r['p99_ms']:.2f} | {r['gelem_s']:.1f} | {100 * r['hbm_frac']:.1f} | {r['launches']} |")
    b = d["backpressure_half_budget"]
    out.append(f"| {b['load']:.2f}, half budget | fused | {b['p50_ms']:.2f} | {b['p99_ms']:.2f} | "
               f"{b['gelem_s']:.1f} | {100 * b['hbm_frac']:.1f} | {b['launches']} |")
    if "online" in d:
        o = d["online"]
        out += ["", f"Online learned tuning (one launch per request; {o['jobs']} jobs of the classes "
                    f"{', '.join(o['classes'])}, batch giving 2^21..2^22 elements, all arriving at t = 0):", "",
                "| configurations | pass | GElem/s | % HBM peak | p50 ms | p99 ms | evaluation launches so far |",
                "|---|---|---|---|---|---|---|"]
        rows = [("analytical model", 1, o["analytical"], "-")]
        for k, p in enumerate(o["online"].get("passes", [o["online"]])):
            rows.append(("online BO", k + 1, p, f"{p['online']['evaluations']} (converged "
                                                f"{p['online']['converged']}/{p['online']['sessions']})"))
        if "offline_exhaustive" in o:
            rows.append(("offline exhaustive cache", 1, o["offline_exhaustive"], "-"))
        for name, k, r, ev in rows:
            out.append(f"| {name} | {k} | {r['gelem_s']:.1f} | {100 * r['hbm_frac']:.1f} | {r['p50_ms']:.2f} | "
                       f"{r['p99_ms']:.2f} | {ev} |")
    print("\n".join(out))


if __name__ == "__main__":
    {"tuning": tuning, "serving": serving}[sys.argv[1]](sys.argv[2])
