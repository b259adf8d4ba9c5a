"""HBM traffic per call of the benchmark step from two rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for a plain device-to-device copy of known size (the 256 MiB
copy that `bench.py --copy-ref` runs first), then matched to the step's calls
by grid and workgroup size.  The record carries a hash of the kernel sources
so that the benchmark drops the figure once the kernels change.

    python -m paper_2310_16214_amd.traffic FETCH.csv WRITE.csv DETAIL.jsonl OUT.json
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SOURCES = {
    "fft": ["fft_device.h", "device.h", "fft.hip", "fft_spec4.hip", "fft_spec8.hip", "fft_spec16.hip"],
    "scan": ["scan_device.h", "device.h", "scan.hip"],
    "tridiag": ["tridiag_device.h", "tridiag_wave_device.h", "device.h", "tridiag.hip"],
}
COPY_BYTES = 256 * 2 ** 20


def sources_sha(op):
    h = hashlib.sha256()
    for f in SOURCES["tridiag" if op.startswith("tridiag") else op]:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_name_prefix(d):
    """The demangled name prefix (kernel and template arguments) of a call."""
    c = d["cfg"]
    if d["op"] == "fft":
        split = "true" if c["algo"] & 1 else "false"
        log2n = d["n"].bit_length() - 1
        if c["radix"] == c["elems_per_thread"] and (c["radix"] in (8, 16) or (c["radix"] == 4 and log2n <= 6)):
            # specialised on log2 n
            name = "k_fft_np" if c["algo"] & 2 else "k_fft_n"
            return f"{name}<{c['radix']}, {c['elems_per_thread']}, {split}, {log2n}>"
        return f"k_fft<{c['radix']}, {c['elems_per_thread']}, {split}>"
    if d["op"] == "scan":
        t = {"int32": "int", "float32": "float", "float64": "double"}[d["dtype"]]
        name = "k_scan_pipe" if c["algo"] & 2 else "k_scan"
        excl = "true" if d.get("exclusive") else "false"
        return f"{name}<{t}, {c['elems_per_thread']}, {c['algo'] & 1}, {excl}>"
    t = "double" if d["dtype"] == "float64" else "float"
    if c["algo"] & 7 == 2 and d["n"] // c["elems_per_thread"] > 64:  # the hybrid across waves
        return f"k_tridiag_blk<{t}, {c['elems_per_thread']}>"
    if c["algo"] & 7 >= 2:
        name = "k_tridiag_wave_pipe" if c["algo"] & 8 else "k_tridiag_wave"
        return f"{name}<{t}, {c['algo'] & 7}, {c['elems_per_thread']}>"
    return f"k_tridiag<{t}, {c['algo']}>"


def _load(path):
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]),
                        int(r["Workgroup_Size"]), float(r["Counter_Value"])))
    return sorted(out)


def main(fetch_csv, write_csv, detail_jsonl, out_json):
    F, W = _load(fetch_csv), _load(write_csv)
    copies = [(f, w) for f, w in zip(F, W) if "copyBuffer" in f[1]]
    if not copies:
        raise SystemExit("no reference copy in the counter runs (run bench.py --copy-ref)")
    # the reference copies are the largest copy dispatches (small ones, such
    # as table uploads, also use the copy kernel)
    gmax = max(f[2] for f, _ in copies)
    copies = [(f, w) for f, w in copies if f[2] == gmax]
    f_scale = COPY_BYTES / 1024 / (sum(f[4] for f, _ in copies) / len(copies))
    w_scale = COPY_BYTES / 1024 / (sum(w[4] for _, w in copies) / len(copies))
    detail = [json.loads(x) for x in open(detail_jsonl)]
    records = []
    for d in detail:
        c = d["cfg"]
        grid = -(-d["batch"] // c["problems_per_block"]) * c["threads_per_block"]
        name = kernel_name_prefix(d)
        hits = [(f, w) for f, w in zip(F, W) if name in f[1] and f[3] == c["threads_per_block"]]
        exact = [h for h in hits if h[0][2] == grid]  # persistent kernels launch fewer workgroups
        hits = exact or hits
        if not hits:
            continue
        f, w = hits[-1]
        bpe = d.get("bpe") or (16 if d["op"] == "fft" else 8 if d["op"] == "scan"
                               else 5 * (8 if d["dtype"] == "float64" else 4))
        algo = bpe * d["n"] * d["batch"]
        records.append(dict(call=f"{d['op']} n={d['n']} {d['dtype']}", cfg=c,
                            fetch_kib=f[4], write_kib=w[4], fetch_scale=f_scale,
                            write_scale=w_scale,
                            traffic_bytes=(f[4] * f_scale + w[4] * w_scale) * 1024,
                            algorithmic_bytes=algo, sources_sha256=sources_sha(d["op"])))
    with open(out_json, "w") as fh:
        fh.write(json.dumps(dict(fetch_scale=f_scale, write_scale=w_scale,
                                 command="rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) "
                                         "--output-format csv -d DIR -o step -- python -u bench.py "
                                         "--steps 1 --warmup 0 --no-cpu-baseline --copy-ref")) + "\n")
        fh.write(json.dumps({"calls": records}, separators=(",", ":")) + "\n")
    print(f"fetch scale {f_scale:.4f}, write scale {w_scale:.4f}, {len(records)} calls")


if __name__ == "__main__":
    main(*sys.argv[1:5])
