"""CPU tests of the measurement tooling: the kernel names that the traffic
record and the kernel-trace summary match calls by are names of kernels the
library actually contains, for every shape the launchers dispatch to a
specialised, persistent or in-wave kernel."""
import os
import shutil
import subprocess

import pytest

from paper_2310_16214_amd import ppx
from paper_2310_16214_amd.traffic import kernel_name_prefix


def _call(op, n, radix, P, L, G, algo, dtype="c64"):
    cfg = dict(radix=radix, elems_per_thread=P, threads_per_block=L, problems_per_block=G,
               lds_elems=0, algo=algo)
    return dict(op=op, n=n, dtype=dtype, batch=1 << 10, cfg=cfg)


CASES = [
    (_call("fft", 16, 4, 4, 256, 64, 0), "k_fft_n<4, 4, false, 4>"),
    (_call("fft", 64, 4, 4, 64, 4, 1), "k_fft_n<4, 4, true, 6>"),
    (_call("fft", 128, 4, 4, 64, 2, 0), "k_fft<4, 4, false>"),
    (_call("fft", 256, 8, 8, 256, 8, 1), "k_fft_n<8, 8, true, 8>"),
    (_call("fft", 16384, 16, 16, 1024, 1, 2), "k_fft_np<16, 16, false, 14>"),
    (_call("fft", 8192, 16, 16, 512, 1, 3), "k_fft_np<16, 16, true, 13>"),
    (_call("fft", 1024, 8, 16, 512, 8, 0), "k_fft<8, 16, false>"),
    (_call("scan", 4096, 2, 4, 1024, 1, 2, "int32"), "k_scan_pipe<int, 4, 0, false>"),
    (_call("scan", 8192, 2, 8, 1024, 1, 3, "float32"), "k_scan_pipe<float, 8, 1, false>"),
    (_call("scan", 64, 2, 4, 64, 4, 1, "float32"), "k_scan<float, 4, 1, false>"),
    (dict(_call("scan", 1024, 2, 16, 64, 1, 0, "float64"), exclusive=True), "k_scan<double, 16, 0, true>"),
    (_call("tridiag_cr", 256, 2, 8, 128, 4, 2, "float32"), "k_tridiag_wave<float, 2, 8>"),
    (_call("tridiag_cr", 128, 2, 8, 128, 8, 10, "float32"), "k_tridiag_wave_pipe<float, 2, 8>"),
    (_call("tridiag_pcr", 1024, 2, 16, 256, 4, 4, "float64"), "k_tridiag_wave<double, 4, 16>"),
    (_call("tridiag_cr", 64, 2, 2, 64, 2, 0, "float64"), "k_tridiag<double, 0>"),
]


@pytest.mark.parametrize("d,name", CASES, ids=[c[1] for c in CASES])
def test_kernel_name_prefix(d, name):
    assert kernel_name_prefix(d) == name


@pytest.mark.skipif(shutil.which("nm") is None, reason="nm not available")
def test_names_are_kernels_of_the_library():
    ppx.lib()  # raises if the library is not built
    out = subprocess.run(["nm", "-C", ppx.LIB_PATH], capture_output=True, text=True, check=True).stdout
    for _, name in CASES:
        assert f"ppx::{name}(" in out, name


def test_counter_table_assigns_dispatches_to_calls_in_order(tmp_path):
    """counter_table maps the library's dispatches, in dispatch order, onto
    the calls file's calls x reps x kernels (a two-pass FFT call gives two
    rows, even where two calls share a kernel instantiation and grid); other
    kernels (the reference copy, torch's fills) are skipped, the copy's
    readings calibrate FETCH_SIZE."""
    import csv

    from paper_2310_16214_amd import counter_table
    calls = [dict(shape="fft:c64:4194304", op="fft", dtype="c64", n=1 << 22, batch=8, cfg=None, kernels=2,
                  reps=2, algorithmic_bytes=1 << 29),
             dict(shape="fft:c64:8388608", op="fft", dtype="c64", n=1 << 23, batch=4, cfg=None, kernels=2,
                  reps=2, algorithmic_bytes=1 << 29)]
    fields = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value",
              "Start_Timestamp", "End_Timestamp"]
    rows, did = [], 0

    def disp(name, grid, value):
        nonlocal did
        did += 1
        rows.append(dict(Dispatch_Id=did, Kernel_Name=name, Grid_Size=grid, Workgroup_Size=1024,
                         Counter_Name="FETCH_SIZE", Counter_Value=value, Start_Timestamp=0, End_Timestamp=1000))

    disp("__amd_rocclr_copyBuffer", 4096, 131072.0)
    disp("void at::native::fill", 256, 5.0)
    shared = "void ppx::k_fft_tile_p<16, 12, true, 4>(float2 const*)"
    for ci, (b_name, vals) in enumerate((("void ppx::k_fft_tile_p<16, 10, false, 16>(float2 const*)", (10.0, 20.0)),
                                         ("void ppx::k_fft_tile_p<16, 11, false, 8>(float2 const*)", (30.0, 40.0)))):
        for _ in range(2):
            disp(shared, 262144, vals[0])
            disp(b_name, 262144, vals[1])
    path = tmp_path / "pass.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)
    groups, copy = counter_table.load([str(path)], calls)
    assert copy["FETCH_SIZE"] == [131072.0]
    assert list(groups) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert [groups[k][1]["FETCH_SIZE"] for k in groups] == [[10.0, 10.0], [20.0, 20.0], [30.0, 30.0], [40.0, 40.0]]
    assert groups[(0, 0)][0][0] == groups[(1, 0)][0][0]  # one kernel instantiation, two calls
