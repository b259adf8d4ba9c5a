"""Serving benchmark: continuous batching into mixed persistent launches vs one
launch per request, on the same GPU and the same arrival trace.

Requests are whole batched jobs: operation FFT (complex FP32), inclusive scan
(FP32) or tridiagonal solve (FP32, the CR -> PCR hybrid family, which holds
every size in registers), equiprobable; per-job N log-uniform on 2^4..2^14;
batch count uniform on 1..4096; Poisson arrivals.  Job inputs are
windows into resident, seeded device pools; outputs are allocated by the
server from its HBM budget and released when the job completes.

The saturation throughput of each mode comes from a burst (every request
arriving at t = 0); the load points are fractions of the fused mode's
saturation arrival rate.  Reported per point: p50 / p99 latency (arrival to
observed completion, host clock), throughput in GElem/s and the fraction of
HBM peak the jobs' algorithmic bytes represent.  A last study serves a trace
of repeated job classes one launch per request with analytical
configurations, with online learned tuning, and with the offline exhaustive
cache.

    python -m paper_2310_16214_amd.serve_bench --jobs 2000 --out serve.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
OPS = ("fft", "scan", "tridiag")
TRI_FAMILY = 2  # PPX_TRI_CR_PCR, the CR -> PCR hybrid family


class Pools:
    """Seeded device input pools that job inputs are windows of."""

    def __init__(self, dev, seed=0):
        import torch

        from paper_2310_16214_amd import inputs
        self.fft = torch.from_numpy(inputs.fft_input(1 << 14, 4096, seed=seed).reshape(-1)).to(dev)
        self.scan = torch.from_numpy(inputs.scan_input(1 << 14, 4096, np.float32, seed=seed + 1)
                                     .reshape(-1)).to(dev)
        a, b, c, d, _ = inputs.tridiag_input(1 << 14, 4096, np.float32, seed=seed + 2)
        self.tri = [torch.from_numpy(v.reshape(-1)).to(dev) for v in (a, b, c, d)]


def _make_job(op, n, batch, rng, pools):
    """A job whose inputs are a random window of the pools, with its meta."""
    from paper_2310_16214_amd import ppx
    elems = n * batch
    if op == "fft":
        off = int(rng.integers(0, pools.fft.numel() - elems + 1)) & ~1
        job = ppx.make_job(ppx.OP_FFT, ppx.C64, n, batch, pools.fft.data_ptr() + 8 * off, None)
        bpe = 16
    elif op == "scan":
        off = int(rng.integers(0, pools.scan.numel() - elems + 1)) & ~3
        job = ppx.make_job(ppx.OP_SCAN, ppx.F32, n, batch, pools.scan.data_ptr() + 4 * off, None)
        bpe = 8
    else:
        off = int(rng.integers(0, pools.tri[0].numel() - elems + 1)) & ~3
        p = [v.data_ptr() + 4 * off for v in pools.tri]
        job = ppx.make_job(ppx.OP_TRIDIAG, ppx.F32, n, batch, p[0], None, algo=TRI_FAMILY,
                           b=p[1], c=p[2], d=p[3])
        bpe = 20
    return job, dict(op=op, n=n, batch=batch, elems=elems, bytes=bpe * elems, offset=off)


def make_trace(njobs, rate_per_s, seed, pools):
    """List of (Job, arrival_us, meta).  rate_per_s = inf: all at t = 0."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for _ in range(njobs):
        op = OPS[rng.integers(0, 3)]
        ln = int(rng.integers(4, 15))
        n = 1 << ln
        batch = int(rng.integers(1, 4097))
        if np.isfinite(rate_per_s):
            t += rng.exponential(1e6 / rate_per_s)
        job, meta = _make_job(op, n, batch, rng, pools)
        out.append((job, t, meta))
    return out


def _summary(trace, comps, mode):
    lat = np.array([c.complete_us - c.arrival_us for c in comps]) / 1e3
    first = min(c.arrival_us for c in comps)
    last = max(c.complete_us for c in comps)
    span_s = (last - first) / 1e6
    elems = sum(m["elems"] for _, _, m in trace)
    byts = sum(m["bytes"] for _, _, m in trace)
    return dict(mode=mode, jobs=len(trace), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()),
                gelem_s=elems / span_s / 1e9, hbm_frac=byts / span_s / 1e9 / HBM_PEAK_GBS,
                span_ms=span_s * 1e3)


def run_trace(trace, mode, budget, max_inflight, passes=1):
    """Replays the trace `passes` times on one server (online tuning keeps its
    sessions across passes); the first pass's record, with the later passes
    under "passes"."""
    from paper_2310_16214_amd import ppx
    flags = {"fused": ppx.SERVE_FUSED, "per_request": ppx.SERVE_PER_REQUEST,
             "online": ppx.SERVE_PER_REQUEST | ppx.SERVE_ONLINE_TUNE}[mode]
    srv = ppx.Server(budget, max_inflight=max_inflight, flags=flags)
    recs = []
    for _ in range(passes):
        t0 = time.perf_counter()
        comps = srv.replay([(j, t) for j, t, _ in trace], auto_release=True)
        r = _summary(trace, comps, mode)
        r["wall_s"] = time.perf_counter() - t0
        if mode == "online":
            r["online"] = srv.online_stats()
        recs.append(r)
    stats = srv.stats()
    srv.close()
    out = dict(recs[0])
    out.update(launches=stats["launches"], peak_used_gib=stats["peak_used_bytes"] / 2 ** 30,
               max_inflight_seen=stats["max_inflight_seen"])
    if passes > 1:
        out["passes"] = recs
    return out


# The online-tuning study: repeated job classes, each large enough (>= 2^21
# elements) for its launches to be timed.
ONLINE_CLASSES = (("fft", 256), ("fft", 4096), ("scan", 1024), ("scan", 8192), ("tridiag", 64),
                  ("tridiag", 512))


def online_study(pools, njobs, seed, budget, max_inflight, cache):
    """Per-request serving of one trace three ways: configurations from the
    analytical model (empty tune cache), online learned tuning (sessions
    start empty, the trace is replayed twice on the same server), and the
    offline exhaustive cache."""
    from paper_2310_16214_amd import ppx
    rng = np.random.default_rng(seed)
    trace = []
    for _ in range(njobs):
        op, n = ONLINE_CLASSES[rng.integers(0, len(ONLINE_CLASSES))]
        batch = int(rng.integers((1 << 21) // n, (1 << 22) // n + 1))
        job, meta = _make_job(op, n, batch, rng, pools)
        trace.append((job, 0.0, meta))
    ppx.clear_tune_cache()
    run_trace(trace[:60], "per_request", budget, max_inflight)  # warm-up
    res = dict(classes=[f"{o} n={n}" for o, n in ONLINE_CLASSES], jobs=njobs)
    res["analytical"] = run_trace(trace, "per_request", budget, max_inflight)
    res["online"] = run_trace(trace, "online", budget, max_inflight, passes=2)
    if os.path.exists(cache):
        ppx.load_tune_cache(cache)
        res["offline_exhaustive"] = run_trace(trace, "per_request", budget, max_inflight)
    return res


def run(njobs=10000, loads=(0.25, 0.5, 0.75, 0.9), budget=4 << 30, max_inflight=2, seed=0,
        quick=False):
    import torch

    from paper_2310_16214_amd import ppx
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    cache = os.path.join(ROOT, "paper_2310_16214_amd", "tuned", "mi355x.txt")
    if os.path.exists(cache):
        ppx.load_tune_cache(cache)
    pools = Pools(dev, seed)
    torch.cuda.synchronize()
    # warm-up (code objects, graphs, arena)
    warm = make_trace(50, float("inf"), seed + 99, pools)
    run_trace(warm, "fused", budget, max_inflight)
    run_trace(warm, "per_request", budget, max_inflight)
    burst = make_trace(njobs, float("inf"), seed, pools)
    sat = {m: run_trace(burst, m, budget, max_inflight) for m in ("fused", "per_request")}
    jobs_per_s = njobs / (sat["fused"]["span_ms"] / 1e3)
    points = []
    for f in loads:
        trace = make_trace(njobs, f * jobs_per_s, seed + 1, pools)
        for m in ("fused", "per_request"):
            r = run_trace(trace, m, budget, max_inflight)
            r["load"] = f
            r["offered_jobs_per_s"] = f * jobs_per_s
            points.append(r)
            print(json.dumps(r), flush=True)
    # back-pressure: half the budget at the highest load
    bp = make_trace(njobs, loads[-1] * jobs_per_s, seed + 1, pools)
    back = run_trace(bp, "fused", budget // 2, max_inflight)
    back["load"] = loads[-1]
    online = online_study(pools, njobs, seed + 7, budget, max_inflight, cache)
    print(json.dumps(online), flush=True)
    return dict(online=online, saturation=sat, saturation_jobs_per_s=jobs_per_s, points=points,
                backpressure_half_budget=back, budget_bytes=budget, max_inflight=max_inflight,
                njobs=njobs, mix="ops equiprobable {fft c64, scan f32, tridiag f32 (CR->PCR hybrid family)}; "
                               "log2 N uniform 4..14; batch uniform 1..4096; Poisson arrivals")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=10000)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--max-inflight", type=int, default=2)
    ap.add_argument("--out", default="")
    ap.add_argument("--online-only", action="store_true", help="run only the online-tuning study")
    args = ap.parse_args()
    budget = int(args.budget_gib * 2 ** 30)
    if args.online_only:
        import torch
        dev = torch.device("cuda:0")
        torch.zeros(1, device=dev)
        pools = Pools(dev, 0)
        cache = os.path.join(ROOT, "paper_2310_16214_amd", "tuned", "mi355x.txt")
        res = dict(online=online_study(pools, args.jobs, 7, budget, args.max_inflight, cache))
        print(json.dumps(res), flush=True)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        return
    res = run(njobs=args.jobs, budget=budget, max_inflight=args.max_inflight)
    print(json.dumps({k: v for k, v in res.items() if k != "points"}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
