"""GPU tests of the mixed launch with the shipped tune cache loaded: every
job's tiles run its tuned configuration, and its output is bit-identical to
the single call with the configuration ppx_mixed_tile_config reports (the
tuned one, persistent flag cleared), whatever else shares the launch; the
NULL-config single call agrees bitwise too wherever the tuned configuration is
not a persistent variant, and to the operation's tolerance where it is."""
import os

import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, fft_tol, scan_bound, to_dev, to_host

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(ppx.__file__), "tuned", "mi355x.txt")
PIPE = {ppx.OP_FFT: 2, ppx.OP_SCAN: 2, ppx.OP_TRIDIAG: 8}

# (kind, dtype code, n, batch, algo / direction); ragged batches
MIX = ([("fft", ppx.C64, 1 << k, b, d) for k, b, d in
        [(4, 3001, -1), (5, 777, 1), (6, 501, -1), (7, 129, -1), (8, 97, 1), (9, 65, -1), (10, 37, -1),
         (11, 19, 1), (12, 9, -1), (13, 5, -1), (14, 3, 1)]]
       + [("scan", dt, 1 << k, b, form) for dt, k, b, form in
          [(ppx.I32, 5, 1001, 0), (ppx.F32, 6, 333, 1), (ppx.F32, 9, 77, 0), (ppx.I32, 11, 21, 1),
           (ppx.F32, 12, 13, 0), (ppx.F32, 13, 7, 0), (ppx.F64, 10, 33, 1), (ppx.I32, 14, 3, 0)]]
       + [("tri", dt, 1 << k, b, fam) for dt, k, b, fam in
          [(ppx.F32, 5, 999, ppx.TRI_CR), (ppx.F32, 7, 201, ppx.TRI_PCR), (ppx.F32, 10, 37, ppx.TRI_CR),
           (ppx.F32, 10, 23, ppx.TRI_PCR), (ppx.F64, 6, 300, ppx.TRI_WM), (ppx.F64, 9, 41, ppx.TRI_LF),
           (ppx.F64, 10, 17, ppx.TRI_CR), (ppx.F32, 8, 61, ppx.TRI_LF), (ppx.F32, 12, 3, ppx.TRI_CR),
           (ppx.F64, 11, 5, ppx.TRI_PCR), (ppx.F32, 13, 3, ppx.TRI_CR_PCR), (ppx.F64, 12, 3, ppx.TRI_CR_PCR),
           (ppx.F32, 10, 37, ppx.TRI_CR_PCR), (ppx.F32, 14, 2, ppx.TRI_CR_PCR)]]
       # jobs of at least 2^22 elements with persistent tuned configurations:
       # their own tuned calls inside the launch
       + [("fft", ppx.C64, 1 << 14, 300, -1), ("scan", ppx.F32, 1 << 13, 600, 0)])


@pytest.fixture(scope="module")
def tuned():
    ppx.clear_tune_cache()
    ppx.load_tune_cache(CACHE)
    yield
    ppx.clear_tune_cache()


def _build(cuda, seed):
    import torch
    jobs, recs = [], []
    for k, (kind, dt, n, batch, extra) in enumerate(MIX):
        s = seed * 1000 + k
        if kind == "fft":
            x = inputs.fft_input(n, batch, seed=s)
            xd = to_dev(x, cuda)
            y = torch.empty_like(xd)
            jobs.append(ppx.make_job(ppx.OP_FFT, ppx.C64, n, batch, xd, y, direction=extra))
            recs.append((kind, dt, n, batch, extra, (x,), (xd,), y))
        elif kind == "scan":
            npdt = {ppx.I32: np.int32, ppx.F32: np.float32, ppx.F64: np.float64}[dt]
            x = (inputs.scan_input_normal(n, batch, npdt, seed=s) if dt != ppx.I32
                 else inputs.scan_input(n, batch, np.int32, seed=s))
            xd = to_dev(x, cuda)
            y = torch.empty_like(xd)
            jobs.append(ppx.make_job(ppx.OP_SCAN, dt, n, batch, xd, y, algo=extra))
            recs.append((kind, dt, n, batch, extra, (x,), (xd,), y))
        else:
            npdt = np.float32 if dt == ppx.F32 else np.float64
            a, b, c, d, _ = inputs.tridiag_input(n, batch, npdt, seed=s)
            dev = [to_dev(v, cuda) for v in (a, b, c, d)]
            y = torch.empty_like(dev[3])
            jobs.append(ppx.make_job(ppx.OP_TRIDIAG, dt, n, batch, dev[0], y, algo=extra, b=dev[1], c=dev[2],
                                     d=dev[3]))
            recs.append((kind, dt, n, batch, extra, (a, b, c, d), dev, y))
    return jobs, recs


def _single(rec, cfg, out):
    kind, dt, n, batch, extra, _, dev, _ = rec
    if kind == "fft":
        ppx.fft_batched(dev[0], out, n, batch, extra, cfg)
    elif kind == "scan":
        f = ppx.scan_exclusive_batched if extra == ppx.JOB_SCAN_EXCLUSIVE else ppx.scan_batched
        f(dev[0], out, n, batch, dt, cfg)
    else:
        if cfg is None:  # the family's configuration, as the per-request path resolves it
            cfg = ppx.tuned_config(ppx.OP_TRIDIAG, dt, n, extra)
        ppx.tridiag_batched(*dev, out, n, batch, dt, cfg)
    return to_host(out).copy()


def _oracle_ok(rec, out):
    kind, dt, n, batch, extra, host, _, _ = rec
    if kind == "fft":
        return oracle.rel_l2(out, oracle.dft(host[0], inverse=extra == 1)).max() <= fft_tol(n)
    if kind == "scan":
        ref = oracle.scan(host[0], exclusive=extra == ppx.JOB_SCAN_EXCLUSIVE)
        if dt == ppx.I32:
            return np.array_equal(out, ref)
        unit = 2.0 ** -24 if dt == ppx.F32 else 2.0 ** -53
        b = scan_bound(host[0], unit, exclusive=extra == ppx.JOB_SCAN_EXCLUSIVE, oracle_unit=2.0 ** -53)
        return np.all(np.abs(out.astype(np.float64) - ref) <= b)
    tol = 1e-4 if dt == ppx.F32 else 1e-12
    return oracle.tridiag_residual(*host, out).max() <= tol


def test_each_job_runs_its_tuned_configuration(cuda, tuned):
    import torch
    jobs, recs = _build(cuda, seed=1)
    for job, rec in zip(jobs, recs):
        kind, dt, n, batch, extra = rec[:5]
        per, cfg = ppx.mixed_tile_config(job)
        op = {"fft": ppx.OP_FFT, "scan": ppx.OP_SCAN, "tri": ppx.OP_TRIDIAG}[kind]
        ref = ppx.tuned_config(op, dt, n, extra) if kind == "tri" else ppx.resolve_config(op, dt, n, batch)
        if ref is None:  # no tuned entry (n > 1024): the family's analytical choice
            assert ppx.tri_family(cfg.algo) == ppx.tri_family(extra), (rec[:5], cfg)
        elif ppx.mixed_job_is_direct(op, n, batch, ref):  # runs as its own tuned call
            assert cfg.as_tuple() == ref.as_tuple(), (rec[:5], cfg, ref)
        else:
            assert cfg.as_tuple() == ref.as_tuple()[:5] + (ref.algo & ~PIPE[op],), (rec[:5], cfg, ref)
        print(f"{rec[:5]}: tile = {per} problems, config {cfg}")
    banner(f"mixed tuned launch of {len(jobs)} jobs")
    ppx.launch_mixed(jobs)
    outs = [to_host(r[7]).copy() for r in recs]
    for job, rec, out in zip(jobs, recs, outs):
        assert _oracle_ok(rec, out), rec[:5]
        _, cfg = ppx.mixed_tile_config(job)
        banner(f"single call {rec[:5]} {cfg}")
        z = torch.empty_like(rec[7])
        single = _single(rec, cfg, z)
        assert np.array_equal(single, out), f"{rec[:5]}: mixed != single call with {cfg}"
        op = {"fft": ppx.OP_FFT, "scan": ppx.OP_SCAN, "tri": ppx.OP_TRIDIAG}[rec[0]]
        tuned_cfg = (ppx.tuned_config(op, rec[1], rec[2], rec[4]) if rec[0] == "tri"
                     else ppx.resolve_config(op, rec[1], rec[2], rec[3]))
        if tuned_cfg is None:
            continue
        null = _single(rec, None, z)
        if not tuned_cfg.algo & PIPE[op] or ppx.mixed_job_is_direct(op, rec[2], rec[3], tuned_cfg):
            assert np.array_equal(null, out), f"{rec[:5]}: mixed != NULL-config single call"
        else:
            assert _oracle_ok(rec, null), rec[:5]
            print(f"{rec[:5]}: persistent tuned config; NULL-config call bit-identical: "
                  f"{np.array_equal(null, out)}")


def test_alone_equals_in_the_mix(cuda, tuned):
    jobs, recs = _build(cuda, seed=2)
    banner("mixed tuned launch, whole mix")
    ppx.launch_mixed(jobs)
    outs = [to_host(r[7]).copy() for r in recs]
    # the mix in reverse order, and each job alone
    for r in recs:
        r[7].zero_()
    banner("mixed tuned launch, reversed")
    ppx.launch_mixed(jobs[::-1])
    for r, o in zip(recs, outs):
        assert np.array_equal(to_host(r[7]), o), r[:5]
    for i, job in enumerate(jobs):
        recs[i][7].zero_()
        banner(f"mixed tuned alone {recs[i][:5]}")
        ppx.launch_mixed([job])
        assert np.array_equal(to_host(recs[i][7]), outs[i]), recs[i][:5]
