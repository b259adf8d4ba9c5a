"""GPU parity of the float64 scan and of the exclusive scan (Sec. III, "Scan
Operator", and its exclusive form) against the sequential oracle.

Bars: int32 bit-exact; float64 on dyadic inputs (every partial sum exact)
bit-exact, for every configuration; float64 on uniform[0,1) inputs within the
blocked-tree bound plus the oracle's own left-to-right rounding; float32
exclusive within the float32 blocked-tree bound (the oracle is exact for the
float32 recipe).
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, scan_bound, to_dev, to_host

pytestmark = pytest.mark.gpu

NS = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
U64, U32 = 2.0 ** -53, 2.0 ** -24


def _run(xd, n, batch, dtype, cfg=None, out=None, exclusive=False):
    import torch
    y = torch.empty_like(xd) if out is None else out
    f = ppx.scan_exclusive_batched if exclusive else ppx.scan_batched
    f(xd, y, n, batch, dtype, cfg)
    return to_host(y)


@pytest.mark.parametrize("n", NS)
def test_float64_dyadic_every_config_bit_exact(cuda, n):
    batch = 23
    _, x = inputs.scan_input_dyadic(n, batch, seed=n + 3)
    xd = to_dev(x, cuda)
    refs = {e: oracle.scan(x, exclusive=e) for e in (False, True)}
    for cfg in ppx.enumerate_configs(ppx.OP_SCAN, ppx.F64, n):
        for e in (False, True):
            banner(f"scan f64 dyadic n={n} excl={e} {cfg}")
            y = _run(xd, n, batch, ppx.F64, cfg, exclusive=e)
            assert np.array_equal(y, refs[e]), f"{cfg} excl={e}: {np.count_nonzero(y != refs[e])} mismatches"


@pytest.mark.parametrize("n", [16, 256, 2048, 16384])
def test_float64_uniform_every_config(cuda, n):
    batch = 11
    x = inputs.scan_input(n, batch, np.float64, seed=n + 5)
    xd = to_dev(x, cuda)
    for e in (False, True):
        ref = oracle.scan(x, exclusive=e)
        bound = scan_bound(x, U64, exclusive=e, oracle_unit=U64)
        for cfg in ppx.enumerate_configs(ppx.OP_SCAN, ppx.F64, n):
            banner(f"scan f64 n={n} excl={e} {cfg}")
            y = _run(xd, n, batch, ppx.F64, cfg, exclusive=e)
            err = np.abs(y - ref)
            assert np.all(err <= bound), f"{cfg} excl={e}: max err {err.max():.3e}"


@pytest.mark.parametrize("n", NS)
def test_exclusive_int32_every_config_bit_exact(cuda, n):
    batch = 29
    x = inputs.scan_input(n, batch, np.int32, seed=n + 11)
    ref = oracle.scan(x, exclusive=True)
    xd = to_dev(x, cuda)
    for cfg in ppx.enumerate_configs(ppx.OP_SCAN, ppx.I32, n):
        banner(f"scan excl i32 n={n} {cfg}")
        y = _run(xd, n, batch, ppx.I32, cfg, exclusive=True)
        assert np.array_equal(y, ref), f"{cfg}: {np.count_nonzero(y != ref)} mismatches"


@pytest.mark.parametrize("n", [16, 128, 1024, 4096, 16384])
def test_exclusive_float32_every_config(cuda, n):
    batch = 13
    x = inputs.scan_input(n, batch, np.float32, seed=n + 13)
    ref = oracle.scan(x, exclusive=True)
    bound = scan_bound(x, U32, exclusive=True)
    xd = to_dev(x, cuda)
    for cfg in ppx.enumerate_configs(ppx.OP_SCAN, ppx.F32, n):
        banner(f"scan excl f32 n={n} {cfg}")
        y = _run(xd, n, batch, ppx.F32, cfg, exclusive=True).astype(np.float64)
        assert np.all(y[:, 0] == 0.0)
        err = np.abs(y - ref)
        assert np.all(err <= bound), f"{cfg}: max err {err.max():.3e}"


def test_exclusive_wraps_and_in_place(cuda):
    n, batch = 2048, 5
    x = np.full((batch, n), 2 ** 30, dtype=np.int32)
    x[1] = -(2 ** 31)
    x[2, ::2] = 2 ** 31 - 1
    x[3:] = inputs.scan_input(n, 2, np.int32, seed=17)
    xd = to_dev(x, cuda)
    banner("scan excl i32 wrap + in place")
    y1 = _run(xd.clone(), n, batch, ppx.I32, exclusive=True)
    y2 = _run(xd, n, batch, ppx.I32, out=xd, exclusive=True)
    ref = oracle.scan(x, exclusive=True)
    assert np.array_equal(y1, ref) and np.array_equal(y2, ref)


@pytest.mark.parametrize("n", [32, 1024, 8192])
def test_full_size(cuda, n):
    """Benchmark sweep size: 2^24 elements per call, configuration from a
    NULL config; every element compared with the oracle."""
    batch = (1 << 24) // n
    _, xd64 = inputs.scan_input_dyadic(n, batch, seed=31)
    xi = inputs.scan_input(n, batch, np.int32, seed=32)
    for e in (False, True):
        banner(f"scan full f64 dyadic n={n} excl={e}")
        y = _run(to_dev(xd64, cuda), n, batch, ppx.F64, exclusive=e)
        assert np.array_equal(y, oracle.scan(xd64, exclusive=e))
    banner(f"scan full excl i32 n={n}")
    assert np.array_equal(_run(to_dev(xi, cuda), n, batch, ppx.I32, exclusive=True),
                          oracle.scan(xi, exclusive=True))


# (n, L, G_b, algo): persistent variants with batches that make every
# workgroup loop several times and leave a ragged last round
PERSISTENT = [(8192, 1024, 1, ppx.SCAN_LF_PIPE), (4096, 1024, 1, ppx.SCAN_KS_PIPE),
              (256, 128, 1, ppx.SCAN_LF_PIPE), (64, 256, 16, ppx.SCAN_KS_PIPE)]


@pytest.mark.parametrize("n,L,G,algo", PERSISTENT)
def test_persistent_variants_loop_and_tail(cuda, n, L, G, algo):
    batch = {8192: 2048 + 5, 4096: 4096 + 3, 256: 100000 + 3, 64: (1 << 18) + 7}[n]
    cfg = ppx.make_config(2, L, G, algo)
    assert ppx.config_valid(ppx.OP_SCAN, ppx.F64, n, cfg)
    _, x = inputs.scan_input_dyadic(n, batch, seed=n + 9)
    xi = inputs.scan_input(n, batch, np.int32, seed=n + 10)
    xd, xid = to_dev(x, cuda), to_dev(xi, cuda)
    for e in (False, True):
        banner(f"scan persistent f64 n={n} batch={batch} excl={e} {cfg}")
        assert np.array_equal(_run(xd, n, batch, ppx.F64, cfg, exclusive=e), oracle.scan(x, exclusive=e))
    banner(f"scan persistent excl i32 n={n} batch={batch} {cfg}")
    assert np.array_equal(_run(xid, n, batch, ppx.I32, cfg, exclusive=True), oracle.scan(xi, exclusive=True))
