"""Runs batched call shapes a few times each on resident inputs, for
rocprofv3 kernel traces and counter runs of one kernel at a time.

Each shape is ``op:dtype:n[:family]`` (family: the tridiagonal family, cr,
pcr, crpcr, wm or lf; FFT and scan use the configuration their call takes
with cfg = NULL, tridiagonal the tuned one of the family), run with batch =
elems // n.  FFT sizes above 16384 run the two-pass transform with its tuned
(else default) plan: two kernels per call, pass A then pass B, each moving
every value once in each direction.  One JSON line per shape gives its
configuration (or plan), the kernels one call launches and the algorithmic
bytes of each (inputs read once, outputs written once), in the order the
kernels run.  ``--copy-ref`` first runs a 256 MiB device-to-device
copy, whose counter readings scale FETCH_SIZE / WRITE_SIZE to bytes.

    python -m paper_2310_16214_amd.one_call tridiag:f32:1024:pcr tridiag:f64:1024:cr \\
        [--elems 4194304] [--reps 5] [--copy-ref] [--out calls.jsonl]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from paper_2310_16214_amd import inputs, ppx

PKG = os.path.dirname(os.path.abspath(__file__))
FAMILIES = {"cr": ppx.TRI_CR, "pcr": ppx.TRI_PCR, "crpcr": ppx.TRI_CR_PCR, "wm": ppx.TRI_WM, "lf": ppx.TRI_LF}
DTYPES = {"i32": (ppx.I32, np.int32), "f32": (ppx.F32, np.float32), "f64": (ppx.F64, np.float64),
          "c64": (ppx.C64, np.complex64)}
COPY_BYTES = 256 * 2 ** 20


def _cfg_dict(c):
    return None if c is None else dict(zip(("radix", "elems_per_thread", "threads_per_block", "problems_per_block",
                                            "lds_elems", "algo"), c.as_tuple()))


def prepare(spec, elems, dev):
    """A zero-argument callable running one call of the shape, and its record."""
    import torch
    parts = spec.split(":")
    op, dt, n = parts[0], parts[1], int(parts[2])
    code, npdt = DTYPES[dt]
    batch = max(1, elems // n)
    kernels = 1
    if op == "fft" and n > 16384:
        x = torch.from_numpy(inputs.fft_input(n, batch, seed=1)).to(dev)
        y = torch.empty_like(x)
        plan = ppx.tuned_fft_plan(n) or ppx.default_fft_plan(n)
        run = lambda: ppx.fft_batched_large(x, y, n, batch, -1, plan)  # noqa: E731
        cfg = None
        nbytes, kernels = 16 * n * batch, 2
        rec_plan = dict(zip(("log2_n1", "radix_a", "radix_b", "tile_a", "tile_b"),
                            (plan.log2_n1, plan.radix_a, plan.radix_b, plan.tile_a, plan.tile_b)))
    elif op == "fft":
        x = torch.from_numpy(inputs.fft_input(n, batch, seed=1)).to(dev)
        y = torch.empty_like(x)
        cfg = ppx.resolve_config(ppx.OP_FFT, ppx.C64, n, batch)
        run = lambda: ppx.fft_batched(x, y, n, batch, -1)  # noqa: E731
        nbytes = 16 * n * batch
    elif op == "scan":
        x = torch.from_numpy(inputs.scan_input(n, batch, npdt, seed=1)).to(dev)
        y = torch.empty_like(x)
        cfg = ppx.resolve_config(ppx.OP_SCAN, code, n, batch)
        run = lambda: ppx.scan_batched(x, y, n, batch, code)  # noqa: E731
        nbytes = 2 * np.dtype(npdt).itemsize * n * batch
    elif op == "tridiag":
        fam = FAMILIES[parts[3] if len(parts) > 3 else "cr"]
        t = [torch.from_numpy(v).to(dev) for v in inputs.tridiag_input(n, batch, npdt, seed=1)[:4]]
        y = torch.empty_like(t[3])
        cfg = ppx.tuned_config(ppx.OP_TRIDIAG, code, n, fam)
        run = lambda: ppx.tridiag_batched(*t, y, n, batch, code, cfg)  # noqa: E731
        nbytes = 5 * np.dtype(npdt).itemsize * n * batch
    else:
        raise SystemExit(f"unknown op in {spec!r}")
    rec = dict(shape=spec, op=op, dtype=dt, n=n, batch=batch, cfg=_cfg_dict(cfg), kernels=kernels,
               algorithmic_bytes=nbytes)
    if kernels == 2:
        rec["plan"] = rec_plan
    return run, rec


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("shapes", nargs="+")
    ap.add_argument("--elems", type=int, default=1 << 22)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-ref", action="store_true")
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    torch.zeros(1, device=dev)
    cache = os.path.join(PKG, "tuned", "mi355x.txt")
    if os.path.exists(cache):
        ppx.load_tune_cache(cache)
    if args.copy_ref:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    recs = []
    for spec in args.shapes:
        run, rec = prepare(spec, args.elems, dev)
        rec["reps"] = args.reps
        for _ in range(args.reps):
            run()
        torch.cuda.synchronize()
        recs.append(rec)
        print(json.dumps(rec), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            for r in recs:
                f.write(json.dumps(r) + "\n")


if __name__ == "__main__":
    main()
