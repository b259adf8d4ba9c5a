"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and rejects bad arguments before touching the HIP runtime."""
import ctypes

import pytest

from paper_2310_16214_amd import ppx

L = ppx.lib()


def test_exports_every_declared_function():
    names = ppx.header_functions()
    assert {"fft_batched", "scan_batched", "tridiag_batched", "tune"} <= set(names)
    for name in names:
        assert hasattr(L, name), f"libppx.so does not export {name}"


def _rc(fn):
    rc = fn()
    return rc, ppx.last_error()


BUF = 4096  # a fake, 16-byte aligned "device" address: never dereferenced


@pytest.mark.parametrize("args,msg", [
    ((0, BUF, 1024, 1, -1), "null"),
    ((BUF + 4, BUF, 1024, 1, -1), "aligned"),
    ((BUF, BUF, 1000, 1, -1), "power of two"),
    ((BUF, BUF, 8, 1, -1), "power of two"),
    ((BUF, BUF, 1 << 24, 1, -1), "power of two"),
    ((BUF, BUF, 1024, 0, -1), "batch"),
    ((BUF, BUF, 1024, 1, 0), "direction"),
    ((BUF, BUF + 16, 1024, 4, -1), "overlap"),
])
def test_fft_argument_errors(args, msg):
    rc, err = _rc(lambda: L.fft_batched(*args, None, None))
    assert rc == ppx.EINVAL and msg in err


# ------------------------------------------------------------ large-N FFT

@pytest.mark.parametrize("args,msg", [
    ((0, BUF, 1 << 16, 1, -1), "null"),
    ((BUF + 8, 1 << 30, 1 << 16, 1, -1), "aligned"),
    ((BUF, 1 << 30, 1 << 14, 1, -1), "power of two"),
    ((BUF, 1 << 40, 1 << 24, 1, -1), "power of two"),
    ((BUF, 1 << 30, 3 << 15, 1, -1), "power of two"),
    ((BUF, 1 << 30, 1 << 16, 0, -1), "batch"),
    ((BUF, 1 << 30, 1 << 16, 1, 2), "direction"),
    ((BUF, BUF, 1 << 16, 1, -1), "overlap"),
    ((BUF, BUF + (1 << 19), 1 << 16, 2, -1), "overlap"),
])
def test_fft_large_argument_errors(args, msg):
    rc, err = _rc(lambda: ppx._tl("fft_batched_large")(*args, None, None))
    assert rc == ppx.EINVAL and msg in err, err


def test_fft_batched_forwards_large_n_and_rejects_a_config():
    # the large path checks its own arguments: in == out is refused
    rc, err = _rc(lambda: L.fft_batched(BUF, BUF, 1 << 16, 1, -1, None, None))
    assert rc == ppx.EINVAL and "overlap" in err
    cfg = ppx.make_config(16, 1024, 1)
    rc, err = _rc(lambda: L.fft_batched(BUF, 1 << 30, 1 << 16, 1, -1, ctypes.byref(cfg), None))
    assert rc == ppx.EINVAL and "plan" in err


def test_fft_plans():
    for ln in range(15, 24):
        n = 1 << ln
        plans = ppx.enumerate_fft_plans(n)
        assert plans, n
        for p in plans:
            assert ppx.fft_plan_valid(n, p)
            l2 = ln - p.log2_n1
            for radix, length, tile, ncols, extra in ((p.radix_a, l2, p.tile_a, 1 << p.log2_n1, 2056),
                                                      (p.radix_b, p.log2_n1, p.tile_b, 1 << l2, 0)):
                threads = tile * (1 << length) // radix
                lds = (-(-tile * ((1 << length) + 1) // 256) * 256 + extra) * 8
                assert radix in (8, 16) and ncols % tile == 0
                assert tile in ((2, 4, 8, 16, 32, 64) if length <= 10 else (2, 4, 8))
                assert 64 <= threads <= 1024 and lds <= 160 * 1024
        keys = [p.as_tuple() for p in plans]
        assert keys == sorted(keys) and len(set(keys)) == len(keys)
        d = ppx.default_fft_plan(n)
        assert d.as_tuple() in keys
        # the most even split (n1 <= n2 on a tie)
        uneven = lambda l1: (abs(2 * l1 - ln), 2 * l1 > ln)  # noqa: E731
        assert all(uneven(d.log2_n1) <= uneven(q[0]) for q in keys)
    assert ppx.default_fft_plan(1 << 20).as_tuple() == (10, 16, 16, 16, 16)
    assert ppx.default_fft_plan(1 << 23).as_tuple() == (11, 16, 16, 4, 8)  # 2^12 x 2^11
    assert (13, 16, 16, 16, 2) in [p.as_tuple() for p in ppx.enumerate_fft_plans(1 << 23)]
    assert not ppx.fft_plan_valid(1 << 16, ppx.make_plan(8, 4, 16))      # radix 4
    assert not ppx.fft_plan_valid(1 << 16, ppx.make_plan(11, 16, 16))    # n1 = 2048 too long
    assert not ppx.fft_plan_valid(1 << 16, ppx.make_plan(6, 8, 16))      # n2 = 1024 with radix 8
    assert not ppx.fft_plan_valid(1 << 14, ppx.make_plan(7, 16, 16))     # not a large size
    assert not ppx.fft_plan_valid(1 << 16, ppx.make_plan(8, 16, 16, 32, 128))  # tile 128
    assert not ppx.fft_plan_valid(1 << 20, ppx.make_plan(10, 16, 16, 32, 16))  # 32 x 1025 values of LDS
    assert not ppx.fft_plan_valid(1 << 21, ppx.make_plan(10, 16, 16, 16, 16))  # pass A column of 2048
    assert not ppx.fft_plan_valid(1 << 21, ppx.make_plan(11, 16, 16, 16, 16))  # 16 x 2049 values of LDS
    assert ppx.fft_plan_valid(1 << 21, ppx.make_plan(11, 16, 16, 16, 8))
    assert ppx.fft_plan_valid(1 << 16, ppx.make_plan(8, 16, 16, 16, 8))       # narrow tiles at any length
    assert not ppx.fft_plan_valid(1 << 16, ppx.make_plan(8, 16, 16, 16, 1))   # tile 1
    assert ppx.fft_plan_valid(1 << 16, ppx.make_plan(8, 16, 16, 64, 64))
    with pytest.raises(ppx.PpxError):
        ppx.enumerate_fft_plans(1 << 14)


def test_scan_and_tridiag_argument_errors():
    for fn in (L.scan_batched, L.scan_exclusive_batched):
        assert fn(BUF, BUF, 64, 1, ppx.C64, None, None) == ppx.EINVAL
        assert fn(BUF, 0, 64, 1, ppx.I32, None, None) == ppx.EINVAL
        assert fn(BUF + 8, BUF, 64, 1, ppx.F64, None, None) == ppx.EINVAL
        assert fn(BUF, BUF, 48, 1, ppx.F64, None, None) == ppx.EINVAL
        # float64: 8 bytes per element when checking overlap
        rc = fn(BUF, BUF + 256, 64, 1, ppx.F64, None, None)
        assert rc == ppx.EINVAL and "overlap" in ppx.last_error()
    assert L.tridiag_batched(BUF, BUF * 2, BUF * 3, BUF * 4, BUF * 5, 64, 1, ppx.I32,
                             None, None) == ppx.EINVAL
    # x may alias d but nothing else
    rc = L.tridiag_batched(BUF, BUF * 2, BUF * 3, BUF * 4, BUF, 64, 1, ppx.F32, None, None)
    assert rc == ppx.EINVAL and "alias" in ppx.last_error()


def test_explicit_config_errors():
    bad = ppx.make_config(16, 64, 1)  # n=64: P = 1 < radix
    rc = L.fft_batched(BUF, BUF, 64, 1, -1, ctypes.byref(bad), None)
    assert rc == ppx.ECONFIG
    assert not ppx.config_valid(ppx.OP_FFT, ppx.C64, 1024, ppx.make_config(3, 256, 1))
    assert not ppx.config_valid(ppx.OP_FFT, ppx.C64, 1024, ppx.make_config(4, 96, 1))
    assert not ppx.config_valid(ppx.OP_SCAN, ppx.I32, 1024, ppx.make_config(4, 256, 1))
    assert not ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 1024, ppx.make_config(2, 256, 1, 5))
    # P = n*G_b/L must lie in [2, 32]
    assert not ppx.config_valid(ppx.OP_SCAN, ppx.I32, 4096, ppx.make_config(2, 64, 1))
    assert ppx.config_valid(ppx.OP_SCAN, ppx.I32, 4096, ppx.make_config(2, 128, 1))
    # an inconsistent explicit P or S is rejected, 0 derives them
    c = ppx.make_config(2, 128, 1, elems_per_thread=16)
    assert not ppx.config_valid(ppx.OP_SCAN, ppx.I32, 4096, c)
    c = ppx.make_config(16, 256, 1, lds_elems=7)
    assert not ppx.config_valid(ppx.OP_FFT, ppx.C64, 4096, c)


def test_scan_float64_space():
    # float64 scan keeps at most 16 elements per thread
    assert ppx.config_valid(ppx.OP_SCAN, ppx.F64, 4096, ppx.make_config(2, 256, 1))
    assert not ppx.config_valid(ppx.OP_SCAN, ppx.F64, 4096, ppx.make_config(2, 128, 1))
    assert ppx.config_valid(ppx.OP_SCAN, ppx.F32, 4096, ppx.make_config(2, 128, 1))
    for n in (16, 1024, 16384):
        cs = ppx.enumerate_configs(ppx.OP_SCAN, ppx.F64, n)
        assert cs and all(c.elems_per_thread <= 16 for c in cs)
        c = ppx.resolve_config(ppx.OP_SCAN, ppx.F64, n, 1 << 16)
        assert ppx.config_valid(ppx.OP_SCAN, ppx.F64, n, c)


def test_tridiag_wm_space():
    wm = ppx.TRI_WM
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 1024, ppx.make_config(2, 64, 1, wm))       # P 16
    assert not ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 2048, ppx.make_config(2, 128, 1, wm))  # 128 lanes
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F64, 64, ppx.make_config(2, 64, 2, wm | ppx.TRI_PIPE))
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F64, 64, ppx.make_config(2, 64, 8, wm | ppx.TRI_PIPE))  # P 8
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F64, 1024, ppx.make_config(2, 64, 1, wm | ppx.TRI_PIPE))  # P 16
    assert not ppx.config_valid(ppx.OP_TRIDIAG, ppx.F64, 2048, ppx.make_config(2, 64, 1, wm | ppx.TRI_PIPE))
    assert not ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 64, ppx.make_config(2, 64, 4, 16))
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 64, ppx.make_config(2, 64, 4, ppx.TRI_CR_PCR))
    assert ppx.tri_family(ppx.TRI_CR_PCR | ppx.TRI_PIPE) == ppx.TRI_CR_PCR
    assert ppx.config_valid(ppx.OP_TRIDIAG, ppx.F32, 64, ppx.make_config(2, 64, 4, ppx.TRI_LF))
    assert ppx.tri_family(wm | ppx.TRI_PIPE) == wm
    assert ppx.tri_family(ppx.TRI_LF | ppx.TRI_PIPE) == ppx.TRI_LF
    cs = ppx.enumerate_configs(ppx.OP_TRIDIAG, ppx.F64, 256)
    assert any(c.algo == wm for c in cs) and any(c.algo == wm | ppx.TRI_PIPE for c in cs)
    assert not any(ppx.tri_family(c.algo) == wm for c in ppx.enumerate_configs(ppx.OP_TRIDIAG, ppx.F32, 4096))


def test_fft_p32_thread_cap():
    assert ppx.config_valid(ppx.OP_FFT, ppx.C64, 16384, ppx.make_config(16, 512, 1))
    assert not ppx.config_valid(ppx.OP_FFT, ppx.C64, 16384, ppx.make_config(16, 1024, 2, 1))


def test_enumeration_respects_the_space():
    for op, dt in ((ppx.OP_FFT, ppx.C64), (ppx.OP_SCAN, ppx.I32), (ppx.OP_TRIDIAG, ppx.F32)):
        for n in (16, 256, 4096, 16384):
            for c in ppx.enumerate_configs(op, dt, n):
                assert ppx.config_valid(op, dt, n, c)
                assert c.elems_per_thread * c.threads_per_block == n * c.problems_per_block
                assert 64 <= c.threads_per_block <= 1024
                assert 1 <= c.problems_per_block <= 64
                if op == ppx.OP_FFT:
                    assert c.radix in (2, 4, 8, 16) and c.radix <= c.elems_per_thread
    # FFT space per size: radix x L x G_b x exchange variant, before validity
    assert 0 < len(ppx.enumerate_configs(ppx.OP_FFT, ppx.C64, 1024)) <= 4 * 5 * 5 * 2


def test_default_is_plain_per_problem_kernel():
    for n in (16, 1024, 16384):
        c = ppx.default_config(ppx.OP_FFT, ppx.C64, n)
        assert c.radix == 2 and c.problems_per_block == 1
        assert c.threads_per_block == min(n // 2, 1024)
        assert c.elems_per_thread == n // c.threads_per_block


def test_resolve_without_gpu_is_valid():
    for op, dt in ((ppx.OP_FFT, ppx.C64), (ppx.OP_SCAN, ppx.F32), (ppx.OP_TRIDIAG, ppx.F64)):
        for n in (16, 1024):
            c = ppx.resolve_config(op, dt, n, 1 << 16)
            assert ppx.config_valid(op, dt, n, c), (op, n, c)


def test_stream_reference_rejects_bad_arguments():
    # validation runs before any HIP call
    for k, nbytes in ((0, 64), (5, 64), (1, 0), (1, 20)):
        ins = [16] * max(k, 1)
        with pytest.raises(ppx.PpxError) as e:
            ppx.stream_reference(ins[:k] if k else [], 16, nbytes)
        assert e.value.code == ppx.EINVAL
