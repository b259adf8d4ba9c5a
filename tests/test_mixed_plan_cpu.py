"""CPU tests of the mixed launch's tile planning (no GPU: configurations come
from the shipped tune cache, or the analytical model's static resource table).

Each job's tiles must follow the configuration its single call uses with a
NULL config (the tuned shape, persistent flag cleared), with the problems per
tile scaled from the tuned block size to the family's, and a valid
single-call configuration reported for it."""
import os

import pytest

from paper_2310_16214_amd import ppx

CACHE = os.path.join(os.path.dirname(ppx.__file__), "tuned", "mi355x.txt")
PIPE = {ppx.OP_FFT: 2, ppx.OP_SCAN: 2, ppx.OP_TRIDIAG: 8}


@pytest.fixture(scope="module")
def tuned():
    ppx.clear_tune_cache()
    ppx.load_tune_cache(CACHE)
    yield
    ppx.clear_tune_cache()


def _job(op, dtype, n, batch, algo=0, direction=-1):
    p = 1 << 12  # 16-byte aligned placeholders: planning never touches memory
    return ppx.make_job(op, dtype, n, batch, p, p, direction=direction, algo=algo, b=p, c=p, d=p)


def _cases():
    out = []
    for k in range(4, 15):
        out.append((ppx.OP_FFT, ppx.C64, 1 << k, 0))
        out.append((ppx.OP_SCAN, ppx.F32, 1 << k, ppx.JOB_SCAN_INCLUSIVE))
        out.append((ppx.OP_SCAN, ppx.I32, 1 << k, ppx.JOB_SCAN_EXCLUSIVE))
        out.append((ppx.OP_SCAN, ppx.F64, 1 << k, ppx.JOB_SCAN_INCLUSIVE))
    for k in range(5, 11):
        for fam in (ppx.TRI_CR, ppx.TRI_PCR, ppx.TRI_CR_PCR, ppx.TRI_WM, ppx.TRI_LF):
            out.append((ppx.OP_TRIDIAG, ppx.F32, 1 << k, fam))
            out.append((ppx.OP_TRIDIAG, ppx.F64, 1 << k, fam))
    return out


@pytest.mark.parametrize("op,dtype,n,algo", _cases())
def test_tiles_follow_the_tuned_configuration(tuned, op, dtype, n, algo):
    batch = max(1, (1 << 22) // n)
    per, cfg = ppx.mixed_tile_config(_job(op, dtype, n, batch, algo))
    if op == ppx.OP_TRIDIAG:
        ref = ppx.tuned_config(op, dtype, n, algo)
    else:
        ref = ppx.resolve_config(op, ppx.C64 if op == ppx.OP_FFT else dtype, n, batch)
    if ref is None:  # no tuned entry: the family's analytical choice
        assert op == ppx.OP_TRIDIAG and ppx.tri_family(cfg.algo) == algo
    elif ppx.mixed_job_is_direct(op, n, batch, ref):  # its own single call
        assert cfg.as_tuple() == ref.as_tuple() and per == ref.problems_per_block
        return
    else:
        want = ref.as_tuple()[:5] + (ref.algo & ~PIPE[op],)
        assert cfg.as_tuple() == want, (cfg, ref)
    assert ppx.config_valid(op, ppx.C64 if op == ppx.OP_FFT else dtype, n, cfg)
    # problems per tile: the tuned workgroup size within the family's limit
    # (256 or 1024 threads; 512 for the float64 hybrid with P = 16) and at
    # least a wave, over the problem's threads -- the tuned G_b where the
    # tuned workgroup is within those bounds
    T = n // cfg.elems_per_thread
    if op == ppx.OP_TRIDIAG and cfg.algo & 7 in (ppx.TRI_CR, ppx.TRI_PCR):
        return  # LDS-exchange tiles: sized by LDS
    if op == ppx.OP_TRIDIAG:  # in-wave (T <= 64) or the hybrid across waves
        limit = 256 if T <= 64 else 512 if (dtype == ppx.F64 and cfg.elems_per_thread == 16) else 1024
    else:
        limit = 256 if T <= 256 else 1024
    block = min(limit, max(cfg.threads_per_block, T, 64))
    assert per == block // T
    if 64 <= cfg.threads_per_block <= limit:
        assert per == cfg.problems_per_block


def test_untuned_fft_shape_gets_a_radix_equal_p_substitute(tmp_path):
    # a radix-2 plain configuration recorded as the tuned one: not a shape
    # the FFT families hold
    plain = ppx.default_config(ppx.OP_FFT, ppx.C64, 1024)
    path = tmp_path / "cache.txt"
    path.write_text("# arch op dtype n algo_filter radix P L G_b S algo us method\n"
                    "gfx950 %d %d 1024 -1 %d %d %d %d %d %d 100.0 0\n"
                    % ((ppx.OP_FFT, ppx.C64) + plain.as_tuple()))
    ppx.clear_tune_cache()
    try:
        ppx.load_tune_cache(str(path))
        assert ppx.resolve_config(ppx.OP_FFT, ppx.C64, 1024, 100).as_tuple() == plain.as_tuple()
        per, cfg = ppx.mixed_tile_config(_job(ppx.OP_FFT, ppx.C64, 1024, 100))
        assert cfg.radix == cfg.elems_per_thread and cfg.radix in (8, 16)
        assert ppx.config_valid(ppx.OP_FFT, ppx.C64, 1024, cfg)
        assert per == cfg.problems_per_block == max(1, 64 // (1024 // cfg.elems_per_thread))
    finally:
        ppx.clear_tune_cache()


def test_job_errors():
    p = 1 << 12
    bad = [ppx.make_job(ppx.OP_FFT, ppx.F32, 64, 1, p, p),  # FFT needs c64
           ppx.make_job(ppx.OP_SCAN, ppx.F32, 64, 1, p, p, algo=3),
           ppx.make_job(ppx.OP_TRIDIAG, ppx.F32, 64, 1, p, p, algo=ppx.TRI_CR_SHFL, b=p, c=p, d=p),
           ppx.make_job(ppx.OP_TRIDIAG, ppx.F64, 8192, 1, p, p, algo=ppx.TRI_CR, b=p, c=p, d=p),
           ppx.make_job(ppx.OP_SCAN, ppx.F32, 100, 1, p, p),
           ppx.make_job(ppx.OP_SCAN, ppx.F32, 64, 1, p + 8, p)]
    for j in bad:
        with pytest.raises(ppx.PpxError):
            ppx.mixed_tile_config(j)


def test_noalloc_refuses_oversize_calls_before_any_gpu_work():
    # planning runs on the host before the device is touched, so these are
    # refused here without a GPU (pointers are never dereferenced)
    p = 1 << 12
    many = [ppx.make_job(ppx.OP_SCAN, ppx.F32, 64, 1, p, p)] * (ppx.NOALLOC_MAX_JOBS + 1)
    with pytest.raises(ppx.PpxError) as e:
        ppx.launch_mixed_noalloc(many, stream=0)
    assert e.value.code == ppx.EINVAL and "PPX_NOALLOC_MAX_JOBS" in str(e.value)
    # tiled (not a persistent configuration, which would run as its own call)
    job = ppx.make_job(ppx.OP_TRIDIAG, ppx.F32, 16384, 1, p, p, algo=ppx.TRI_CR_PCR, b=p, c=p, d=p)
    per, cfg = ppx.mixed_tile_config(job)
    assert not cfg.algo & ppx.TRI_PIPE
    big = ppx.make_job(ppx.OP_TRIDIAG, ppx.F32, 16384, (ppx.NOALLOC_MAX_TILES + 1) * per, p, p,
                       algo=ppx.TRI_CR_PCR, b=p, c=p, d=p)
    with pytest.raises(ppx.PpxError) as e:
        ppx.launch_mixed_noalloc([big], stream=0)
    assert e.value.code == ppx.EINVAL and "PPX_NOALLOC_MAX_TILES" in str(e.value)


def test_argument_launch_rule(tuned):
    # at most PPX_MIXED_ARG_JOBS jobs in every family: records in the kernel
    # arguments; one more job in a family: the device tables
    small = [_job(ppx.OP_SCAN, ppx.I32, 32, 1 + k) for k in range(ppx.MIXED_ARG_JOBS)]
    assert ppx.mixed_argument_launch(small)
    assert not ppx.mixed_argument_launch(small + [_job(ppx.OP_SCAN, ppx.F32, 64, 5)])
    # other families do not count against it, nor do jobs that run as their own call
    others = [_job(ppx.OP_FFT, ppx.C64, 1 << (4 + k % 11), 3) for k in range(8)]
    assert ppx.mixed_argument_launch(small + others)
    big = _job(ppx.OP_FFT, ppx.C64, 1 << 14, 300)
    _, cfg = ppx.mixed_tile_config(big)
    if ppx.mixed_job_is_direct(ppx.OP_FFT, 1 << 14, 300, cfg):
        assert ppx.mixed_argument_launch([big])
        assert ppx.mixed_argument_launch(small + [big])
    with pytest.raises(ppx.PpxError):
        ppx.mixed_argument_launch([ppx.make_job(ppx.OP_SCAN, ppx.F32, 100, 1, 1 << 12, 1 << 12)])
