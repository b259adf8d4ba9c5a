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
    ((BUF, BUF, 32768, 1, -1), "power of two"),
    ((BUF, BUF, 1024, 0, -1), "batch"),
    ((BUF, BUF, 1024, 1, 0), "direction"),
    ((BUF, BUF + 16, 1024, 4, -1), "overlap"),
])
def test_fft_argument_errors(args, msg):
    rc, err = _rc(lambda: L.fft_batched(*args, None, None))
    assert rc == ppx.EINVAL and msg in err


def test_scan_and_tridiag_argument_errors():
    assert L.scan_batched(BUF, BUF, 64, 1, ppx.F64, None, None) == ppx.EINVAL
    assert L.scan_batched(BUF, 0, 64, 1, ppx.I32, None, None) == ppx.EINVAL
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
