"""GPU tests of the mixed launch: every job of a mix of operations, sizes and
batch counts against the oracle (each operation's tolerance), bit-identical
to the same job launched alone, stable across repeated launches with other
work in between, and the same whether the records travel in the kernel
arguments or in the device tables (persistent kernels)."""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, fft_tol, scan_bound, scan_f32_bound, to_dev, to_host

pytestmark = pytest.mark.gpu

# (op, dtype, n, batch, algo/direction)
MIX = [("fft", 16, 1000, -1), ("fft", 1024, 37, -1), ("fft", 16384, 3, 1), ("fft", 128, 129, 1),
       ("scan_i32", 32, 700, 0), ("scan_f32", 4096, 9, 0), ("scan_i32", 8192, 5, 0),
       ("scan_f32", 16384, 3, 0), ("tri_f32", 64, 300, ppx.TRI_CR), ("tri_f32", 1024, 7, ppx.TRI_PCR),
       ("tri_f64", 256, 33, ppx.TRI_CR), ("tri_f32", 8192, 2, ppx.TRI_CR), ("fft", 2048, 1, -1),
       ("scan_excl_i32", 256, 300, 1), ("scan_f64", 1024, 40, 0), ("scan_excl_f64", 16384, 3, 1),
       ("scan_excl_f32", 2048, 20, 1)]


def _build(cuda, seed=0):
    import torch
    jobs, checks = [], []
    for k, (kind, n, batch, extra) in enumerate(MIX):
        s = seed * 100 + k
        if kind == "fft":
            x = inputs.fft_input(n, batch, seed=s)
            xd = to_dev(x, cuda)
            y = torch.empty_like(xd)
            jobs.append(ppx.make_job(ppx.OP_FFT, ppx.C64, n, batch, xd, y, direction=extra))
            checks.append((kind, n, batch, (x, extra), (xd,), y))
        elif kind.startswith("scan"):
            code = {"i32": ppx.I32, "f32": ppx.F32, "f64": ppx.F64}[kind[-3:]]
            if code == ppx.F64:  # dyadic values: every partial sum exact
                _, x = inputs.scan_input_dyadic(n, batch, seed=s)
            else:
                x = inputs.scan_input(n, batch, np.int32 if code == ppx.I32 else np.float32, seed=s)
            xd = to_dev(x, cuda)
            y = torch.empty_like(xd)
            jobs.append(ppx.make_job(ppx.OP_SCAN, code, n, batch, xd, y, algo=extra))
            checks.append((kind, n, batch, (x,), (xd,), y))
        else:
            dt = np.float32 if kind.endswith("f32") else np.float64
            a, b, c, d, _ = inputs.tridiag_input(n, batch, dt, seed=s)
            dev = [to_dev(v, cuda) for v in (a, b, c, d)]
            y = torch.empty_like(dev[3])
            jobs.append(ppx.make_job(ppx.OP_TRIDIAG, ppx.F32 if dt == np.float32 else ppx.F64, n,
                                     batch, dev[0], y, algo=extra, b=dev[1], c=dev[2], d=dev[3]))
            checks.append((kind, n, batch, (a, b, c, d), dev, y))
    return jobs, checks


def _check_oracle(kind, n, host, out):
    if kind == "fft":
        x, direction = host
        err = oracle.rel_l2(out, oracle.dft(x, inverse=direction == 1)).max()
        assert err <= fft_tol(n), (kind, n, err)
    elif kind.startswith("scan"):
        x, excl = host[0], "excl" in kind
        ref = oracle.scan(x, exclusive=excl)
        if kind.endswith("f32"):
            bound = scan_bound(x, 2.0 ** -24, exclusive=True) if excl else scan_f32_bound(x)
            assert np.all(np.abs(out.astype(np.float64) - ref) <= bound), kind
        else:  # int32, and float64 on dyadic values: exact
            assert np.array_equal(out, ref), kind
    else:
        tol = 1e-4 if kind.endswith("f32") else 1e-12
        assert oracle.tridiag_residual(*host, out).max() <= tol


def test_mixed_launch_matches_oracle_and_alone(cuda):
    import torch
    jobs, checks = _build(cuda)
    banner(f"mixed launch of {len(jobs)} jobs")
    ppx.launch_mixed(jobs)
    outs = [to_host(c[5]).copy() for c in checks]
    for (kind, n, batch, host, _, _), out in zip(checks, outs):
        _check_oracle(kind, n, host, out)
    # each job alone in its own mixed launch gives the same bits
    for i, job in enumerate(jobs):
        banner(f"mixed alone job {i} {MIX[i]}")
        checks[i][5].zero_()
        ppx.launch_mixed([job])
        assert np.array_equal(to_host(checks[i][5]), outs[i]), MIX[i]


def test_replays_are_stable_with_eager_work_between(cuda):
    import torch
    jobs, checks = _build(cuda, seed=3)
    ref = None
    for rep in range(6):
        banner(f"mixed replay {rep}")
        for c in checks:
            c[5].fill_(float("nan") if c[5].dtype.is_floating_point or c[5].is_complex() else -7)
        ppx.launch_mixed(jobs)
        scratch = torch.randn(1 << 20, device=cuda).sum()  # eager work between replays
        torch.cuda.synchronize()
        outs = [to_host(c[5]).copy() for c in checks]
        if ref is None:
            ref = outs
            for (kind, n, batch, host, _, _), out in zip(checks, outs):
                _check_oracle(kind, n, host, out)
        else:
            for a, b, m in zip(ref, outs, MIX):
                assert np.array_equal(a, b), m
        del scratch


def test_mixed_matches_single_calls_within_tolerance(cuda):
    import torch
    jobs, checks = _build(cuda, seed=5)
    ppx.launch_mixed(jobs)
    torch.cuda.synchronize()
    for (kind, n, batch, host, dev, y), m in zip(checks, MIX):
        if kind != "fft":
            continue
        z = torch.empty_like(y)
        ppx.fft_batched(dev[0], z, n, batch, m[3])
        rel = oracle.rel_l2(to_host(y), to_host(z).astype(np.complex128)).max()
        assert rel <= 2 * fft_tol(n)


def test_mixed_rejects_bad_jobs(cuda):
    import torch
    x = torch.zeros(64, dtype=torch.float64, device=cuda)
    bad = ppx.make_job(ppx.OP_TRIDIAG, ppx.F64, 16384, 1, x, x, algo=ppx.TRI_PCR, b=x, c=x, d=x)
    with pytest.raises(ppx.PpxError):
        ppx.launch_mixed([bad])
    with pytest.raises(ppx.PpxError):
        ppx.launch_mixed([ppx.make_job(ppx.OP_FFT, ppx.C64, 100, 1, x, x)])
    with pytest.raises(ppx.PpxError):  # scan form must be inclusive or exclusive
        ppx.launch_mixed([ppx.make_job(ppx.OP_SCAN, ppx.F64, 64, 1, x, x, algo=2)])


def test_table_launch_equals_argument_launch(cuda):
    import torch
    jobs, checks = _build(cuda, seed=7)
    assert ppx.mixed_argument_launch(jobs)
    banner("mixed launch, records in the kernel arguments")
    ppx.launch_mixed(jobs)
    outs = [to_host(c[5]).copy() for c in checks]
    # more than PPX_MIXED_ARG_JOBS jobs of one family: the whole launch goes
    # through the device tables and the persistent kernels
    fill_in, fill_out, fill_host = [], [], []
    for k in range(ppx.MIXED_ARG_JOBS + 1):
        x = inputs.scan_input(32, 1 + 7 * k, np.int32, seed=700 + k)
        xd = to_dev(x, cuda)
        y = torch.full_like(xd, -5)
        fill_in.append(ppx.make_job(ppx.OP_SCAN, ppx.I32, 32, x.shape[0], xd, y, algo=k % 2))
        fill_out.append(y)
        fill_host.append((x, xd))
    mix = jobs[:5] + fill_in + jobs[5:]
    assert not ppx.mixed_argument_launch(mix)
    for c in checks:
        c[5].fill_(float("nan") if c[5].dtype.is_floating_point or c[5].is_complex() else -7)
    banner("mixed launch, device tables")
    ppx.launch_mixed(mix)
    for c, o, m in zip(checks, outs, MIX):
        assert np.array_equal(to_host(c[5]), o), m
    for k, (y, (x, _)) in enumerate(zip(fill_out, fill_host)):
        assert np.array_equal(to_host(y), oracle.scan(x, exclusive=k % 2 == 1)), k
