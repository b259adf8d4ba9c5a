"""GPU parity of the batched FFT against the O(N^2) DFT oracle.

Bar: per-problem relative L2 <= 1e-5 * log2 N (FP32), max over the batch;
the oracle's own error against the float64 library FFT is reported alongside.
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, fft_tol, to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(x_dev, n, batch, cfg=None, direction=-1, out=None):
    import torch
    y = torch.empty_like(x_dev) if out is None else out
    ppx.fft_batched(x_dev, y, n, batch, direction, cfg)
    return to_host(y)


def test_c1_plain_radix2_64x1024(cuda):
    """The small benchmark case: 64 signals of N = 1024, seed 0, plain kernel."""
    n, batch = 1024, 64
    banner(f"fft c1 n={n} batch={batch} default config")
    x = inputs.fft_input(n, batch, seed=0)
    ref = oracle.dft(x)
    cfg = ppx.default_config(ppx.OP_FFT, ppx.C64, n)
    assert (cfg.radix, cfg.problems_per_block, cfg.threads_per_block) == (2, 1, 512)
    y = _run(to_dev(x, cuda), n, batch, cfg)
    err = oracle.rel_l2(y, ref)
    oracle_err = oracle.rel_l2(ref, np.fft.fft(x.astype(np.complex128), axis=1))
    print(f"c1 rel-L2 max {err.max():.3e} median {np.median(err):.3e}; "
          f"oracle vs float64 FFT {oracle_err.max():.3e}")
    assert err.max() <= fft_tol(n)


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384])
def test_every_config_matches_oracle(cuda, n):
    """Every valid (radix, L, G_b, algo) of the search space, ragged batch."""
    cfgs = ppx.enumerate_configs(ppx.OP_FFT, ppx.C64, n)
    assert cfgs, "no valid configuration"
    batch = 37 if n <= 1024 else 5  # not a multiple of any G_b > 1: ragged last workgroup
    x = inputs.fft_input(n, batch, seed=n)
    ref = oracle.dft(x)
    xd = to_dev(x, cuda)
    worst = 0.0
    for cfg in cfgs:
        banner(f"fft n={n} batch={batch} {cfg}")
        err = oracle.rel_l2(_run(xd, n, batch, cfg), ref)
        worst = max(worst, err.max())
        assert err.max() <= fft_tol(n), f"{cfg}: rel-L2 {err.max():.3e}"
    oracle_err = oracle.rel_l2(ref, np.fft.fft(x.astype(np.complex128), axis=1)).max()
    print(f"n={n}: {len(cfgs)} configs, worst rel-L2 {worst:.3e} (bound {fft_tol(n):.1e}); "
          f"oracle vs float64 FFT {oracle_err:.3e}")


@pytest.mark.parametrize("n", [16, 256, 2048, 16384])
def test_inverse_and_roundtrip(cuda, n):
    import torch
    batch = 6
    x = inputs.fft_input(n, batch, seed=3)
    banner(f"fft inverse n={n}")
    xd = to_dev(x, cuda)
    yi = _run(xd, n, batch, direction=+1)
    assert oracle.rel_l2(yi, oracle.dft(x, inverse=True)).max() <= fft_tol(n)
    fwd = torch.empty_like(xd)
    ppx.fft_batched(xd, fwd, n, batch, -1)
    back = _run(fwd, n, batch, direction=+1) / n
    assert oracle.rel_l2(back, x).max() <= 2 * fft_tol(n)


def test_in_place(cuda):
    n, batch = 4096, 9
    x = inputs.fft_input(n, batch, seed=5)
    xd = to_dev(x, cuda)
    banner("fft in place")
    y = _run(xd, n, batch, out=xd)
    assert oracle.rel_l2(y, oracle.dft(x)).max() <= fft_tol(n)


@pytest.mark.parametrize("n,radix,L,G", [(16, 4, 256, 64), (32, 4, 128, 16), (64, 8, 256, 32), (64, 4, 64, 4)])
def test_staged_io_in_place(cuda, n, radix, L, G):
    """Small n, where the specialised kernel reads and writes its workgroup's
    block as 16-byte words through LDS: in place with a ragged last
    workgroup, against the oracle; an 8-byte aligned buffer is refused."""
    import torch
    batch = 3 * G + 5
    x = inputs.fft_input(n, batch, seed=n + 7)
    ref = oracle.dft(x)
    cfg = ppx.make_config(radix, L, G, 0)
    banner(f"fft staged io n={n} {cfg}")
    xd = to_dev(x, cuda)
    y = _run(xd, n, batch, cfg, out=xd)
    assert oracle.rel_l2(y, ref).max() <= fft_tol(n)
    src = torch.zeros(batch * n + 1, dtype=torch.complex64, device=cuda)
    with pytest.raises(ppx.PpxError) as e:
        ppx.fft_batched(src[1:], src[1:], n, batch, -1, cfg)
    assert e.value.code == ppx.EINVAL


def test_single_problem_and_closed_forms(cuda):
    # impulse -> constant spectrum; constant -> N * delta (exact in FP32)
    n = 512
    x = np.zeros((2, n), np.complex64)
    x[0, 0] = 1.0
    x[1, :] = 1.0
    banner("fft closed forms")
    y = _run(to_dev(x, cuda), n, 2)
    assert np.allclose(y[0], 1.0, atol=1e-6)
    ref = np.zeros(n)
    ref[0] = n
    assert np.allclose(y[1], ref, atol=1e-3)


@pytest.mark.parametrize("n", [16, 1024, 16384])
def test_full_size_sampled(cuda, n):
    """Tuner-sweep size (256 MiB per call) with the configuration a NULL
    config resolves to; checked on sampled problems against the oracle."""
    import torch
    batch = (1 << 25) // n
    banner(f"fft full size n={n} batch={batch}")
    x = inputs.fft_input(n, batch, seed=11)
    xd = to_dev(x, cuda)
    y = torch.empty_like(xd)
    ppx.fft_batched(xd, y, n, batch, -1)
    idx = np.unique(np.array([0, 1, batch // 2, batch - 2, batch - 1]))
    ys = to_host(y[torch.from_numpy(idx).to(cuda)])
    err = oracle.rel_l2(ys, oracle.dft(x[idx]))
    assert err.max() <= fft_tol(n)


def test_rejects_bad_arguments(cuda):
    import torch
    x = torch.zeros(64, dtype=torch.complex64, device=cuda)
    with pytest.raises(ppx.PpxError) as e:
        ppx.fft_batched(x, x, 48, 1)
    assert e.value.code == ppx.EINVAL
    with pytest.raises(ppx.PpxError) as e:
        ppx.fft_batched(x, x, 64, 1, cfg=ppx.make_config(16, 64, 1))  # P = 1 < radix
    assert e.value.code == ppx.ECONFIG


# (n, radix, L, G_b, algo): the persistent (prefetching) variants with batches
# that make every workgroup loop several times and leave a ragged last round
# Covers mixed-radix first stages of every radix below R, full-radix first
# stages (4096 with R = 16, 512 with R = 8), two to five stages (so one to
# four chunks of prefetched loads), both exchanges and several problems per
# workgroup.
PERSISTENT = [(16384, 16, 1024, 1, ppx.FFT_LDS_PIPE), (8192, 16, 512, 1, ppx.FFT_LDS_SPLIT_PIPE),
              (8192, 8, 1024, 1, ppx.FFT_LDS_PIPE), (4096, 16, 512, 2, ppx.FFT_LDS_PIPE),
              (2048, 16, 128, 1, ppx.FFT_LDS_PIPE), (1024, 8, 128, 1, ppx.FFT_LDS_PIPE),
              (512, 8, 128, 2, ppx.FFT_LDS_SPLIT_PIPE), (128, 16, 64, 8, ppx.FFT_LDS_SPLIT_PIPE),
              (64, 16, 64, 16, ppx.FFT_LDS_SPLIT_PIPE), (32, 16, 64, 32, ppx.FFT_LDS_PIPE),
              (16, 8, 64, 32, ppx.FFT_LDS_PIPE)]


@pytest.mark.parametrize("n,radix,L,G,algo", PERSISTENT)
def test_persistent_variants_loop_and_tail(cuda, n, radix, L, G, algo):
    """Several problems per workgroup (grid = resident workgroups) and a ragged
    last round: sampled problems against the oracle (forward and inverse), and
    every problem against the plain kernel of the same shape, which runs the
    same stages (agreement to the FFT bound, not bitwise: the compiler may
    contract multiply-adds differently in the two kernels)."""
    import torch
    batch = {16384: 2048 + 37, 8192: 4096 + 21, 4096: 8192 + 3, 2048: 9000 + 11, 1024: 12000 + 5,
             512: 30000 + 1, 128: 100000 + 3, 64: 300000 + 7, 32: 400000 + 9, 16: 500000 + 13}[n]
    cfg = ppx.make_config(radix, L, G, algo)
    plain = ppx.make_config(radix, L, G, algo & ppx.FFT_LDS_SPLIT)
    assert ppx.config_valid(ppx.OP_FFT, ppx.C64, n, cfg)
    x = inputs.fft_input(n, batch, seed=n + 1)
    xd = to_dev(x, cuda)
    idx = np.unique(np.array([0, 1, G, batch // 3, batch // 2, batch - G - 1, batch - 2, batch - 1]))
    for direction in (-1, +1):
        banner(f"fft persistent n={n} batch={batch} {cfg} direction={direction}")
        y = torch.empty_like(xd)
        ppx.fft_batched(xd, y, n, batch, direction, cfg)
        ys = to_host(y[torch.from_numpy(idx).to(cuda)])
        err = oracle.rel_l2(ys, oracle.dft(x[idx], inverse=direction > 0))
        assert err.max() <= fft_tol(n), f"rel-L2 {err.max():.3e}"
        y2 = torch.empty_like(xd)
        ppx.fft_batched(xd, y2, n, batch, direction, plain)
        d = oracle.rel_l2(to_host(y), to_host(y2))
        print(f"n={n} direction={direction}: max rel-L2 persistent vs plain {d.max():.2e}")
        assert d.max() <= fft_tol(n)


@pytest.mark.parametrize("batch", [1, 7, 300, 1500, 2600, 4100, 6001])
def test_persistent_radix8_every_exit(cuda, batch):
    """Batches that end after one, two, three or more iterations per
    workgroup of the persistent kernel (every early exit of its peeled and
    unrolled loop), each problem against the plain kernel and a few against
    the oracle."""
    import torch
    n = 4096
    cfg = ppx.make_config(8, 512, 1, ppx.FFT_LDS_PIPE)
    plain = ppx.make_config(8, 512, 1, 0)
    x = inputs.fft_input(n, batch, seed=batch)
    xd = to_dev(x, cuda)
    banner(f"fft persistent radix 8 n={n} batch={batch}")
    y, y2 = torch.empty_like(xd), torch.empty_like(xd)
    ppx.fft_batched(xd, y, n, batch, -1, cfg)
    ppx.fft_batched(xd, y2, n, batch, -1, plain)
    assert oracle.rel_l2(to_host(y), to_host(y2)).max() <= fft_tol(n)
    idx = np.unique(np.array([0, batch // 2, batch - 1]))
    ys = to_host(y[torch.from_numpy(idx).to(cuda)])
    assert oracle.rel_l2(ys, oracle.dft(x[idx])).max() <= fft_tol(n)


def test_persistent_needs_radix_equal_p(cuda):
    import torch
    x = torch.zeros(1024, dtype=torch.complex64, device=cuda)
    with pytest.raises(ppx.PpxError) as e:
        ppx.fft_batched(x, x, 1024, 1, cfg=ppx.make_config(4, 64, 1, ppx.FFT_LDS_PIPE))  # P = 16, radix 4
    assert e.value.code == ppx.ECONFIG
