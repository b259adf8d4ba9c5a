"""GPU tests of the tuning entry points through the C ABI: tune() with each
method records a valid configuration that NULL-config calls then use, the
exhaustive result is the minimum of its own trace, and the learned and
analytical choices are valid members of the space."""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, fft_tol, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_tune_each_method_records_a_valid_config(cuda):
    import torch
    ppx.clear_tune_cache()
    n, batch = 256, 4096
    for method in (ppx.TUNE_ANALYTICAL, ppx.TUNE_LEARNED, ppx.TUNE_EXHAUSTIVE):
        banner(f"tune fft n={n} method={method}")
        cfg, us, evals = ppx.tune(ppx.OP_FFT, ppx.C64, n, batch, method, max_evals=0)
        assert ppx.config_valid(ppx.OP_FFT, ppx.C64, n, cfg) and us > 0
        if method == ppx.TUNE_ANALYTICAL:
            assert evals == 0
        else:
            assert evals >= 1
        assert ppx.resolve_config(ppx.OP_FFT, ppx.C64, n, batch).as_tuple() == cfg.as_tuple()
    # the NULL config now runs the tuned kernel, and it is correct
    x = inputs.fft_input(n, 64, seed=8)
    xd = to_dev(x, cuda)
    y = torch.empty_like(xd)
    ppx.fft_batched(xd, y, n, 64)
    assert oracle.rel_l2(to_host(y), oracle.dft(x)).max() <= fft_tol(n)
    ppx.clear_tune_cache()


def test_exhaustive_is_the_minimum_of_its_trace(cuda):
    banner("tune_ex exhaustive scan")
    rep, trace = ppx.tune_ex(ppx.OP_SCAN, ppx.I32, 1024, 1 << 14, ppx.TUNE_EXHAUSTIVE, reps=10)
    assert len(trace) == rep.ncands == len(ppx.enumerate_configs(ppx.OP_SCAN, ppx.I32, 1024))
    best = min(us for _, us in trace)
    assert rep.best_us == pytest.approx(best)
    banner("tune_ex learned scan")
    rep2, trace2 = ppx.tune_ex(ppx.OP_SCAN, ppx.I32, 1024, 1 << 14, ppx.TUNE_LEARNED, reps=10,
                               max_evals=6)
    assert 1 <= rep2.evals_used <= 6
    ppx.clear_tune_cache()


def test_tridiag_family_filter(cuda):
    banner("tune_ex tridiag CR family")
    rep, trace = ppx.tune_ex(ppx.OP_TRIDIAG, ppx.F32, 64, 1 << 12, ppx.TUNE_EXHAUSTIVE,
                             algo=ppx.TRI_CR, reps=5)
    algos = {c.algo for c, _ in trace}
    assert {ppx.TRI_CR, ppx.TRI_CR_SHFL} <= algos
    assert all(ppx.tri_family(a) == ppx.TRI_CR for a in algos)
    assert ppx.tri_family(ppx.tuned_config(ppx.OP_TRIDIAG, ppx.F32, 64, ppx.TRI_CR).algo) == ppx.TRI_CR
    ppx.clear_tune_cache()


@pytest.mark.parametrize("family", [ppx.TRI_WM, ppx.TRI_LF])
def test_tridiag_wm_lf_families(cuda, family):
    """Each tuner restricted to the Wang & Mou or Ladner-Fischer family
    returns a configuration of that family, recorded under it."""
    for method in (ppx.TUNE_EXHAUSTIVE, ppx.TUNE_ANALYTICAL, ppx.TUNE_LEARNED):
        banner(f"tune_ex tridiag family={family} method={method}")
        rep, trace = ppx.tune_ex(ppx.OP_TRIDIAG, ppx.F64, 256, 1 << 12, method, algo=family, reps=5)
        assert ppx.tri_family(rep.best.algo) == family and rep.best_us > 0
        assert all(ppx.tri_family(c.algo) == family for c, _ in trace)
        assert ppx.tri_family(ppx.tuned_config(ppx.OP_TRIDIAG, ppx.F64, 256, family).algo) == family
    ppx.clear_tune_cache()


def test_scan_float64_tuning(cuda):
    for method in (ppx.TUNE_EXHAUSTIVE, ppx.TUNE_ANALYTICAL, ppx.TUNE_LEARNED):
        banner(f"tune_ex scan f64 method={method}")
        rep, _ = ppx.tune_ex(ppx.OP_SCAN, ppx.F64, 2048, 1 << 10, method, reps=5)
        assert ppx.config_valid(ppx.OP_SCAN, ppx.F64, 2048, rep.best) and rep.best.elems_per_thread <= 16
    ppx.clear_tune_cache()


def test_time_config_and_resources(cuda):
    cfg = ppx.default_config(ppx.OP_FFT, ppx.C64, 1024)
    us = ppx.time_config(ppx.OP_FFT, ppx.C64, 1024, 1 << 12, cfg, reps=5)
    assert us > 0
    r = ppx.kernel_resources(ppx.OP_FFT, ppx.C64, 1024, cfg)
    assert r.threads == 512 and r.regs_per_thread > 0 and r.lds_bytes >= 1024 * 8
    with pytest.raises(ppx.PpxError):
        ppx.time_config(ppx.OP_FFT, ppx.C64, 1024, 16, ppx.make_config(3, 64, 1))


def test_stream_reference_sums_its_inputs(cuda):
    import torch
    banner("stream reference")
    ins = [torch.full((4096,), float(i + 1), dtype=torch.float32, device=cuda) for i in range(4)]
    out = torch.empty(4096, dtype=torch.float32, device=cuda)
    for k in (1, 2, 4):
        ppx.stream_reference(ins[:k], out, 4096 * 4)
        torch.cuda.synchronize()
        assert torch.all(out == float(k * (k + 1) // 2))
