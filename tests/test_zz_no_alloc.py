"""GPU test of launch_mixed_noalloc (the mixed launch whose tables live in the
library's static device array): through the C ABI, its outputs are
bit-identical to launch_mixed's on the same jobs, on two calls in a row, the
second with fewer and smaller jobs (so any state the first call left in the
shared array must not leak into the second).  The first call has too many
jobs of one family for the kernel arguments, so its tables go through the
array; the second passes its records in the kernel arguments.  The refusal of calls larger
than the array is tested on the CPU (tests/test_mixed_plan_cpu.py)."""
import numpy as np
import pytest

from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

# (kind, dtype code, n, batch, algo / direction)
FIRST = [("fft", ppx.C64, 1024, 40, -1), ("fft", ppx.C64, 16384, 3, 1), ("fft", ppx.C64, 64, 300, -1),
         ("scan", ppx.F32, 4096, 17, 0), ("scan", ppx.I32, 128, 500, 1), ("scan", ppx.F64, 8192, 5, 0),
         ("tri", ppx.F32, 256, 90, ppx.TRI_CR), ("tri", ppx.F64, 1024, 9, ppx.TRI_PCR),
         ("tri", ppx.F32, 4096, 3, ppx.TRI_CR), ("tri", ppx.F32, 64, 200, ppx.TRI_WM),
         ("tri", ppx.F32, 8192, 2, ppx.TRI_CR_PCR), ("tri", ppx.F64, 2048, 3, ppx.TRI_CR_PCR),
         ("fft", ppx.C64, 16384, 300, -1)]  # a job that runs as its own tuned call
# more than PPX_MIXED_ARG_JOBS jobs of one family: the first call keeps its
# tables in the static array; the second passes its few records in the
# kernel arguments
FIRST += [("scan", ppx.I32, 32, 1 + 5 * k, k % 2) for k in range(ppx.MIXED_ARG_JOBS + 2)]
SECOND = [("scan", ppx.F32, 256, 7, 1), ("fft", ppx.C64, 32, 11, 1), ("tri", ppx.F64, 32, 5, ppx.TRI_LF)]


def _jobs(cuda, mix, seed):
    import torch
    jobs, outs = [], []
    for k, (kind, dt, n, batch, extra) in enumerate(mix):
        s = seed * 100 + k
        if kind == "fft":
            xd = to_dev(inputs.fft_input(n, batch, seed=s), cuda)
            jobs.append(lambda y, xd=xd, n=n, b=batch, e=extra: ppx.make_job(ppx.OP_FFT, ppx.C64, n, b, xd, y,
                                                                              direction=e))
            outs.append(lambda xd=xd: torch.empty_like(xd))
        elif kind == "scan":
            npdt = {ppx.I32: np.int32, ppx.F32: np.float32, ppx.F64: np.float64}[dt]
            xd = to_dev(inputs.scan_input(n, batch, npdt, seed=s), cuda)
            jobs.append(lambda y, xd=xd, n=n, b=batch, e=extra, dt=dt: ppx.make_job(ppx.OP_SCAN, dt, n, b, xd, y,
                                                                                     algo=e))
            outs.append(lambda xd=xd: torch.empty_like(xd))
        else:
            npdt = np.float32 if dt == ppx.F32 else np.float64
            dev = [to_dev(v, cuda) for v in inputs.tridiag_input(n, batch, npdt, seed=s)[:4]]
            jobs.append(lambda y, dev=dev, n=n, b=batch, e=extra, dt=dt: ppx.make_job(
                ppx.OP_TRIDIAG, dt, n, b, dev[0], y, algo=e, b=dev[1], c=dev[2], d=dev[3]))
            outs.append(lambda dev=dev: torch.empty_like(dev[3]))
    return jobs, outs


def _run_both(cuda, mix, seed, argument_launch):
    import torch
    make, alloc = _jobs(cuda, mix, seed)
    ya = [a() for a in alloc]
    yb = [a() for a in alloc]
    assert ppx.mixed_argument_launch([m(y) for m, y in zip(make, ya)]) == argument_launch
    for y in yb:  # stale values in the no-alloc outputs: every element must be written
        y.fill_(float("nan") if y.dtype.is_floating_point or y.is_complex() else -9)
    banner(f"launch_mixed, {len(mix)} jobs (seed {seed})")
    ppx.launch_mixed([m(y) for m, y in zip(make, ya)])
    banner(f"launch_mixed_noalloc, {len(mix)} jobs (seed {seed})")
    ppx.launch_mixed_noalloc([m(y) for m, y in zip(make, yb)])
    torch.cuda.synchronize()
    for item, a, b in zip(mix, ya, yb):
        assert np.array_equal(to_host(a), to_host(b)), item


def test_noalloc_matches_launch_mixed_twice(cuda):
    _run_both(cuda, FIRST, seed=1, argument_launch=False)
    _run_both(cuda, SECOND, seed=2, argument_launch=True)
