"""GPU parity of the batched CR / PCR / CR -> PCR hybrid / Wang & Mou /
Ladner-Fischer tridiagonal solvers against the FP64 Thomas oracle.

Bar: per-system relative residual ||A x - d|| / ||d|| (float64, on the stored
coefficients) <= 1e-4 for float32 and <= 1e-12 for float64, and the forward
error against the float64 oracle within the diagonal-dominance bound
||A^-1||_inf * ||A x - d||_inf (so also <= kappa_inf * 1e-4 relative, with
kappa_inf <= 6 for this recipe); the forward errors against the oracle and
against the known solution are reported.
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, to_dev, to_host, tridiag_forward_check

pytestmark = pytest.mark.gpu

TOL = {np.float32: 1e-4, np.float64: 1e-12}
CODE = {np.float32: ppx.F32, np.float64: ppx.F64}


def _solve(arrs_dev, n, batch, dtype, cfg=None, x=None):
    import torch
    a, b, c, d = arrs_dev
    x = torch.empty_like(d) if x is None else x
    ppx.tridiag_batched(a, b, c, d, x, n, batch, CODE[dtype], cfg)
    return to_host(x)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384])
def test_every_config(cuda, n, dtype):
    batch = 37 if n <= 1024 else 5 if n <= 4096 else 3
    a, b, c, d, xt = inputs.tridiag_input(n, batch, dtype, seed=n)
    dev = [to_dev(v, cuda) for v in (a, b, c, d)]
    ref = oracle.thomas(a, b, c, d)
    cfgs = ppx.enumerate_configs(ppx.OP_TRIDIAG, CODE[dtype], n)
    if not cfgs:
        assert dtype == np.float64 and n == 16384  # the only size with no configuration
        return
    worst_fe = 0.0
    for cfg in cfgs:
        banner(f"tridiag n={n} {np.dtype(dtype).name} {cfg}")
        x = _solve(dev, n, batch, dtype, cfg)
        r = oracle.tridiag_residual(a, b, c, d, x)
        assert r.max() <= TOL[dtype], f"{cfg}: residual {r.max():.3e}"
        fe, fb = tridiag_forward_check(a, b, c, d, x, ref)
        assert np.all(fe <= fb), f"{cfg}: forward error {fe.max():.3e} over its bound"
        worst_fe = max(worst_fe, float(fe.max()))
    print(f"n={n} {np.dtype(dtype).name}: {len(cfgs)} configs, last residual {r.max():.2e}, "
          f"worst |x-oracle| {worst_fe:.2e}, |x-x_true| {np.max(np.abs(x - xt)):.2e}")


IN_WAVE = [ppx.TRI_CR_PCR, ppx.TRI_CR_SHFL, ppx.TRI_PCR_SHFL, ppx.TRI_PCR_REG, ppx.TRI_WM, ppx.TRI_LF]
ALL_ALGOS = [ppx.TRI_CR, ppx.TRI_PCR] + IN_WAVE + [a | ppx.TRI_PIPE for a in IN_WAVE]


@pytest.mark.parametrize("algo", ALL_ALGOS)
def test_boundary_coefficients_are_ignored(cuda, algo):
    n, batch = 256, 8
    a, b, c, d, _ = inputs.tridiag_input(n, batch, np.float32, seed=2)
    cfg = ppx.make_config(2, 128, 4, algo)  # P = 8: n / P = 32 lanes per system
    x_clean = _solve([to_dev(v, cuda) for v in (a, b, c, d)], n, batch, np.float32, cfg)
    a2, c2 = a.copy(), c.copy()
    a2[:, 0] = np.nan
    c2[:, -1] = np.inf
    banner(f"tridiag NaN boundary algo={algo}")
    x_pois = _solve([to_dev(v, cuda) for v in (a2, b, c2, d)], n, batch, np.float32, cfg)
    assert np.array_equal(x_clean, x_pois)
    assert np.all(np.isfinite(x_pois))


def test_x_may_alias_d(cuda):
    n, batch = 512, 10
    a, b, c, d, _ = inputs.tridiag_input(n, batch, np.float64, seed=4)
    dev = [to_dev(v, cuda) for v in (a, b, c, d)]
    banner("tridiag x aliases d")
    x = _solve(dev, n, batch, np.float64, x=dev[3])
    assert oracle.tridiag_residual(a, b, c, d, x).max() <= 1e-12


def _full_size_cases():
    """(n, dtype, algo) of the full-size test: every variant at the sweep's
    smallest and largest size where a configuration of it exists (the in-wave
    variants need n / P <= 64)."""
    cases = []
    for n in (32, 1024):
        for dtype in (np.float32, np.float64):
            algos = {c.algo for c in ppx.enumerate_configs(ppx.OP_TRIDIAG, CODE[dtype], n)}
            cases += [(n, dtype, a) for a in ALL_ALGOS if a in algos]
    return cases


@pytest.mark.parametrize("n,dtype,algo", _full_size_cases())
def test_full_size(cuda, n, dtype, algo):
    """Benchmark sweep size: 2^22 unknowns per call; every system checked
    against the residual bar and the forward-error bound."""
    batch = (1 << 22) // n
    a, b, c, d, xt = inputs.tridiag_input(n, batch, dtype, seed=31)
    dev = [to_dev(v, cuda) for v in (a, b, c, d)]
    cfg = ppx.resolve_config(ppx.OP_TRIDIAG, CODE[dtype], n, batch)
    cfg.algo = algo
    cfg.lds_elems = 0
    if not ppx.config_valid(ppx.OP_TRIDIAG, CODE[dtype], n, cfg):
        cfg = [c for c in ppx.enumerate_configs(ppx.OP_TRIDIAG, CODE[dtype], n) if c.algo == algo][0]
    banner(f"tridiag full n={n} {np.dtype(dtype).name} {cfg}")
    x = _solve(dev, n, batch, dtype, cfg)
    r = oracle.tridiag_residual(a, b, c, d, x)
    assert r.max() <= TOL[dtype]
    fe, fb = tridiag_forward_check(a, b, c, d, x, oracle.thomas(a, b, c, d))
    assert np.all(fe <= fb), f"forward error {fe.max():.3e} over its bound"


# (n, dtype, L, G_b, algo): persistent variants with batches that make every
# workgroup loop several times and leave a ragged last round
PERSISTENT = [(64, np.float32, 64, 4, ppx.TRI_CR_SHFL | ppx.TRI_PIPE),
              (256, np.float32, 128, 4, ppx.TRI_PCR_REG | ppx.TRI_PIPE),
              (128, np.float64, 64, 2, ppx.TRI_PCR_REG | ppx.TRI_PIPE),
              (32, np.float64, 128, 16, ppx.TRI_PCR_SHFL | ppx.TRI_PIPE),
              (128, np.float32, 256, 16, ppx.TRI_CR_SHFL | ppx.TRI_PIPE),
              (128, np.float32, 128, 4, ppx.TRI_WM | ppx.TRI_PIPE),
              (64, np.float64, 64, 2, ppx.TRI_WM | ppx.TRI_PIPE),
              (32, np.float32, 256, 64, ppx.TRI_WM | ppx.TRI_PIPE),
              (256, np.float32, 256, 8, ppx.TRI_LF | ppx.TRI_PIPE),
              (128, np.float64, 128, 2, ppx.TRI_LF | ppx.TRI_PIPE)]


@pytest.mark.parametrize("n,dtype,L,G,algo", PERSISTENT)
def test_persistent_variants_loop_and_tail(cuda, n, dtype, L, G, algo):
    batch = (1 << 22) // n + 5
    cfg = ppx.make_config(2, L, G, algo)
    assert ppx.config_valid(ppx.OP_TRIDIAG, CODE[dtype], n, cfg)
    a, b, c, d, _ = inputs.tridiag_input(n, batch, dtype, seed=n + 3)
    banner(f"tridiag persistent n={n} batch={batch} {np.dtype(dtype).name} {cfg}")
    x = _solve([to_dev(v, cuda) for v in (a, b, c, d)], n, batch, dtype, cfg)
    r = oracle.tridiag_residual(a, b, c, d, x)
    assert r.max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_wm_lf_forward_error_matches_cr(cuda, dtype):
    """Wang & Mou and Ladner-Fischer against CR on the same systems: all
    within the residual bar, and forward errors against the oracle of the
    same order."""
    n, batch = 1024, 64
    a, b, c, d, _ = inputs.tridiag_input(n, batch, dtype, seed=41)
    dev = [to_dev(v, cuda) for v in (a, b, c, d)]
    ref = oracle.thomas(a, b, c, d)
    err = {}
    for algo in (ppx.TRI_CR_SHFL, ppx.TRI_WM, ppx.TRI_LF, ppx.TRI_CR_PCR):
        cfg = ppx.make_config(2, 64, 1, algo)  # P = 16, one system per wave
        banner(f"tridiag wm vs cr {np.dtype(dtype).name} algo={algo}")
        x = _solve(dev, n, batch, dtype, cfg)
        assert oracle.tridiag_residual(a, b, c, d, x).max() <= TOL[dtype]
        err[algo] = np.max(np.abs(x - ref)) / np.max(np.abs(ref))
    for algo in (ppx.TRI_WM, ppx.TRI_LF, ppx.TRI_CR_PCR):
        assert err[algo] <= 10 * max(err[ppx.TRI_CR_SHFL], np.finfo(dtype).eps), err
