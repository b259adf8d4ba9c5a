"""GPU parity of the batched inclusive scan against the sequential oracle.

Bar: int32 bit-exact (sums wrap modulo 2^32); float32 elementwise within
(ceil(log2 N) + 32) * 2^-23 * sum_{j<=i} |x_j| of the float64 oracle, which is
the exact sum for the uniform[0,1) float32 recipe.
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, scan_f32_bound, to_dev, to_host

pytestmark = pytest.mark.gpu

NS = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]


def _run(xd, n, batch, dtype, cfg=None, out=None):
    import torch
    y = torch.empty_like(xd) if out is None else out
    ppx.scan_batched(xd, y, n, batch, dtype, cfg)
    return to_host(y)


@pytest.mark.parametrize("n", NS)
def test_int32_every_config_bit_exact(cuda, n):
    cfgs = ppx.enumerate_configs(ppx.OP_SCAN, ppx.I32, n)
    batch = 37
    x = inputs.scan_input(n, batch, np.int32, seed=n)
    ref = oracle.scan(x)
    xd = to_dev(x, cuda)
    for cfg in cfgs + [ppx.default_config(ppx.OP_SCAN, ppx.I32, n)]:
        banner(f"scan i32 n={n} {cfg}")
        y = _run(xd, n, batch, ppx.I32, cfg)
        assert np.array_equal(y, ref), f"{cfg}: {np.count_nonzero(y != ref)} mismatches"


@pytest.mark.parametrize("n", NS)
def test_float32_every_config(cuda, n):
    cfgs = ppx.enumerate_configs(ppx.OP_SCAN, ppx.F32, n)
    batch = 19
    x = inputs.scan_input(n, batch, np.float32, seed=n + 1)
    ref = oracle.scan(x)
    bound = scan_f32_bound(x)
    xd = to_dev(x, cuda)
    worst = 0.0
    for cfg in cfgs:
        banner(f"scan f32 n={n} {cfg}")
        y = _run(xd, n, batch, ppx.F32, cfg).astype(np.float64)
        err = np.abs(y - ref)
        worst = max(worst, float(np.max(err / np.maximum(np.abs(ref), 1e-30))))
        assert np.all(err <= bound), f"{cfg}: max err {err.max():.3e}"
    print(f"n={n}: worst relative error {worst:.3e}")


def test_int32_wraps_modulo_2_32(cuda):
    n, batch = 1024, 3
    x = np.full((batch, n), 2 ** 30, dtype=np.int32)
    x[1] = -(2 ** 31)
    x[2, ::2] = 2 ** 31 - 1
    banner("scan i32 wrap")
    y = _run(to_dev(x, cuda), n, batch, ppx.I32)
    assert np.array_equal(y, oracle.scan(x))


def test_in_place_and_repeatable(cuda):
    n, batch = 2048, 33
    x = inputs.scan_input(n, batch, np.int32, seed=9)
    xd = to_dev(x, cuda)
    banner("scan i32 in place + repeat")
    y1 = _run(xd.clone(), n, batch, ppx.I32)
    y2 = _run(xd, n, batch, ppx.I32, out=xd)
    assert np.array_equal(y1, y2) and np.array_equal(y1, oracle.scan(x))


@pytest.mark.parametrize("n", [32, 256, 1024, 8192])
@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_full_size(cuda, n, dtype):
    """Benchmark sweep size: 2^24 elements per call, configuration from a
    NULL config; every element compared with the oracle."""
    batch = (1 << 24) // n
    code = ppx.I32 if dtype == np.int32 else ppx.F32
    banner(f"scan full n={n} dtype={np.dtype(dtype).name}")
    x = inputs.scan_input(n, batch, dtype, seed=21)
    y = _run(to_dev(x, cuda), n, batch, code)
    ref = oracle.scan(x)
    if dtype == np.int32:
        assert np.array_equal(y, ref)
    else:
        assert np.all(np.abs(y.astype(np.float64) - ref) <= scan_f32_bound(x))


# (n, P, L, G_b, algo): persistent variants with batches that make every
# workgroup loop several times and leave a ragged last round
PERSISTENT = [(8192, 8, 1024, 1, ppx.SCAN_LF_PIPE), (4096, 4, 1024, 1, ppx.SCAN_KS_PIPE),
              (256, 2, 128, 1, ppx.SCAN_LF_PIPE), (64, 4, 256, 16, ppx.SCAN_KS_PIPE)]


@pytest.mark.parametrize("n,P,L,G,algo", PERSISTENT)
@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_persistent_variants_loop_and_tail(cuda, n, P, L, G, algo, dtype):
    batch = {8192: 2048 + 5, 4096: 4096 + 3, 256: 100000 + 3, 64: (1 << 18) + 7}[n]
    code = ppx.I32 if dtype == np.int32 else ppx.F32
    cfg = ppx.make_config(2, L, G, algo)
    assert ppx.config_valid(ppx.OP_SCAN, code, n, cfg) and n * G // L == P
    x = inputs.scan_input(n, batch, dtype, seed=n + 7)
    banner(f"scan persistent n={n} batch={batch} {np.dtype(dtype).name} {cfg}")
    y = _run(to_dev(x, cuda), n, batch, code, cfg)
    ref = oracle.scan(x)
    if dtype == np.int32:
        assert np.array_equal(y, ref)
    else:
        assert np.all(np.abs(y.astype(np.float64) - ref) <= scan_f32_bound(x))
