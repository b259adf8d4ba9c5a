"""CPU oracle for the batched parallel-prefix operations -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library: the two share no code.  The only module
both sides use is the seeded input generator, which holds none of the
operations' arithmetic.

Each function follows the paper's definition of the operation (Sec. III of
arXiv:2310.16214) in double precision, by the plain route:

* :func:`dft` -- the complex DFT by its O(N^2) definition (Sec. III, FFT;
  forward sign -1, unnormalised inverse sign +1).
* :func:`scan` -- inclusive sum scan (Sec. III, "Scan Operator": every element
  becomes the sum from the first element up to itself), int32 modulo 2^32,
  floating point in float64; ``exclusive=True`` gives the exclusive form (the
  sum of the elements strictly before, 0 for the first).
* :func:`thomas` -- the solution of the tridiagonal system of Sec. III by
  tridiagonal Gaussian elimination (Thomas algorithm), float64.
* :func:`tridiag_residual`, :func:`rel_l2` -- the error measures used to assess
  a GPU result.
* :func:`phi` -- the harmonic-mean performance-portability metric of Sec. VI.

The C part (``oracle.c``) is compiled with gcc on first use (or by the
package-level build step) into ``liboracle.so`` beside this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (-O2, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            i64 = ctypes.c_int64
            ci = ctypes.c_int
            lib.oracle_dft.argtypes = [dp, dp, i64, i64, ci, ci]
            lib.oracle_dft_bins.argtypes = [dp, dp, i64, i64, ctypes.POINTER(ctypes.c_int64), i64, ci, ci]
            lib.oracle_scan_u32.argtypes = [u32p, u32p, i64, i64, ci]
            lib.oracle_scan_f64.argtypes = [dp, dp, i64, i64, ci]
            lib.oracle_scan_excl_u32.argtypes = [u32p, u32p, i64, i64, ci]
            lib.oracle_scan_excl_f64.argtypes = [dp, dp, i64, i64, ci]
            lib.oracle_thomas.argtypes = [dp, dp, dp, dp, dp, i64, i64, ci]
            lib.oracle_tridiag_residual.argtypes = [dp, dp, dp, dp, dp, dp,
                                                    i64, i64, ci]
            for f in (lib.oracle_dft, lib.oracle_dft_bins, lib.oracle_scan_u32, lib.oracle_scan_f64,
                      lib.oracle_scan_excl_u32, lib.oracle_scan_excl_f64,
                      lib.oracle_thomas, lib.oracle_tridiag_residual):
                f.restype = ci
            _lib = lib
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_2d(x, n=None):
    x = np.asarray(x)
    if x.ndim == 1:
        x = x[None, :]
    if x.ndim != 2:
        raise ValueError("expected [batch][n] or [n]")
    return x


def _check(rc, what):
    if rc == -3:
        raise FloatingPointError(f"{what}: zero pivot")
    if rc != 0:
        raise RuntimeError(f"{what}: oracle returned {rc}")


def dft(x, inverse: bool = False, nthreads: int = 0) -> np.ndarray:
    """O(N^2) DFT of every row of ``x`` (complex), returned as complex128.

    X[k] = sum_j x[j] exp(-2 pi i j k / N) (forward) or with +2 pi i
    (inverse, unnormalised).  Inputs are promoted exactly to float64.
    """
    x = _as_2d(x)
    batch, n = x.shape
    xr = np.empty((batch, n, 2), dtype=np.float64)
    xr[..., 0] = np.real(x)
    xr[..., 1] = np.imag(x)
    out = np.empty_like(xr)
    rc = _load().oracle_dft(_ptr(xr, ctypes.c_double), _ptr(out, ctypes.c_double),
                            n, batch, 1 if inverse else -1, nthreads)
    _check(rc, "oracle_dft")
    return out[..., 0] + 1j * out[..., 1]


def dft_bins(x, ks, inverse: bool = False, nthreads: int = 0) -> np.ndarray:
    """Bins ``ks`` of the DFT of every row of ``x``, each by its O(N)
    definition: [batch][len(ks)] complex128 (same convention as :func:`dft`)."""
    x = _as_2d(x)
    batch, n = x.shape
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    xr = np.empty((batch, n, 2), dtype=np.float64)
    xr[..., 0] = np.real(x)
    xr[..., 1] = np.imag(x)
    out = np.empty((batch, len(ks), 2), dtype=np.float64)
    rc = _load().oracle_dft_bins(_ptr(xr, ctypes.c_double), _ptr(out, ctypes.c_double), n, batch,
                                 ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(ks),
                                 1 if inverse else -1, nthreads)
    _check(rc, "oracle_dft_bins")
    return out[..., 0] + 1j * out[..., 1]


def scan(x, nthreads: int = 0, exclusive: bool = False) -> np.ndarray:
    """Inclusive (or, with ``exclusive``, exclusive) sum scan of every row.

    int32 input -> int32 output computed modulo 2^32 (bit pattern of the
    wrapped sum); any floating input -> float64 output, summed left to right.
    """
    x = _as_2d(x)
    batch, n = x.shape
    lib = _load()
    if x.dtype == np.int32 or x.dtype == np.uint32:
        xi = np.ascontiguousarray(x).view(np.uint32)
        y = np.empty((batch, n), dtype=np.uint32)
        f = lib.oracle_scan_excl_u32 if exclusive else lib.oracle_scan_u32
        rc = f(_ptr(xi, ctypes.c_uint32), _ptr(y, ctypes.c_uint32), n, batch, nthreads)
        _check(rc, "oracle scan (u32)")
        return y.view(x.dtype)
    if not np.issubdtype(x.dtype, np.floating):
        raise TypeError("scan oracle takes int32 or floating input")
    xf = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty((batch, n), dtype=np.float64)
    f = lib.oracle_scan_excl_f64 if exclusive else lib.oracle_scan_f64
    rc = f(_ptr(xf, ctypes.c_double), _ptr(y, ctypes.c_double), n, batch, nthreads)
    _check(rc, "oracle scan (f64)")
    return y


def thomas(a, b, c, d, nthreads: int = 0) -> np.ndarray:
    """float64 solution of a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i per row.

    a[:, 0] and c[:, -1] are ignored (the unknowns they multiply are absent).
    """
    arrs = [np.ascontiguousarray(_as_2d(v), dtype=np.float64) for v in (a, b, c, d)]
    batch, n = arrs[1].shape
    for v in arrs:
        if v.shape != (batch, n):
            raise ValueError("a, b, c, d must share one [batch][n] shape")
    x = np.empty((batch, n), dtype=np.float64)
    rc = _load().oracle_thomas(*[_ptr(v, ctypes.c_double) for v in arrs],
                               _ptr(x, ctypes.c_double), n, batch, nthreads)
    _check(rc, "oracle_thomas")
    return x


def tridiag_residual(a, b, c, d, x, nthreads: int = 0) -> np.ndarray:
    """Per-system ||A x - d||_2 / ||d||_2 in float64 on the stored coefficients."""
    arrs = [np.ascontiguousarray(_as_2d(v), dtype=np.float64) for v in (a, b, c, d, x)]
    batch, n = arrs[1].shape
    rel = np.empty(batch, dtype=np.float64)
    rc = _load().oracle_tridiag_residual(*[_ptr(v, ctypes.c_double) for v in arrs],
                                         _ptr(rel, ctypes.c_double), n, batch, nthreads)
    _check(rc, "oracle_tridiag_residual")
    return rel


def rel_l2(y, ref) -> np.ndarray:
    """Per-problem relative L2 error ||y_b - ref_b||_2 / ||ref_b||_2 (float64)."""
    y = _as_2d(y).astype(np.complex128 if np.iscomplexobj(y) else np.float64)
    ref = _as_2d(ref)
    num = np.sqrt(np.sum(np.abs(y - ref) ** 2, axis=1))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=1))
    return num / np.where(den > 0, den, 1.0)


def phi(efficiencies) -> float:
    """Harmonic mean of per-size efficiencies (Sec. VI): |C| / sum_i 1/e_i.

    Each e_i is a method's performance on size i as a fraction of the best
    observed performance on that size (0 < e_i <= 1).
    """
    e = [float(v) for v in efficiencies]
    if not e or any(v <= 0 for v in e):
        raise ValueError("efficiencies must be positive and non-empty")
    return len(e) / sum(1.0 / v for v in e)
