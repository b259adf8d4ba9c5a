"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the CPU oracle's
callers.  It draws random numbers and lays them out; it holds none of the
operations' arithmetic.  Every generator uses ``numpy.random.default_rng(seed)``
and draws its arrays in the fixed order documented on each function, so a
(config, seed) pair always produces the same bytes.

Workload shapes follow the paper's batched setup (Sec. VI: many independent
problems of a power-of-two size N resident on the GPU) with the value
distributions of the benchmark configurations:

* FFT: real and imaginary parts i.i.d. uniform[-1, 1].
* scan: int32 uniform on the integers [-100, 100]; float32 uniform [0, 1).
* tridiagonal: a, c uniform[-1, 1], b = |a| + |c| + uniform[1, 2] (strictly
  diagonally dominant), a known solution x uniform[-1, 1] and d = A x formed
  in float64 from the rounded coefficients, then rounded to the dtype.
"""
from __future__ import annotations

import numpy as np


def fft_input(n: int, batch: int, seed: int = 0) -> np.ndarray:
    """complex64 [batch][n]; draws the real array, then the imaginary array."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=(batch, n)).astype(np.float32)
    im = rng.uniform(-1.0, 1.0, size=(batch, n)).astype(np.float32)
    out = np.empty((batch, n), dtype=np.complex64)
    out.real = re
    out.imag = im
    return out


def scan_input(n: int, batch: int, dtype, seed: int = 0) -> np.ndarray:
    """int32 uniform on [-100, 100] or float32 uniform [0, 1), shape [batch][n]."""
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    if dtype == np.int32:
        return rng.integers(-100, 101, size=(batch, n), dtype=np.int32)
    if dtype == np.float32:
        return rng.random(size=(batch, n), dtype=np.float32)
    if dtype == np.float64:
        return rng.random(size=(batch, n), dtype=np.float64)
    raise TypeError(f"unsupported scan dtype {dtype}")


def scan_input_spiked(n: int, batch: int, dtype, seed: int = 0, spike: float = 1.0e6) -> np.ndarray:
    """float32 or float64 uniform [0, 1), shape [batch][n], with one value per
    row replaced by ``spike`` at a position p with (p + 1) % 32 == 0, i.e. at
    the end of a 32-element block (hence of every aligned chunk of 2..32
    elements that contains it).  Draw order: the uniform array, then the
    block index of each row (integers on [0, n/32), or 0 when n < 32, where
    the spike goes at n - 1)."""
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    x = rng.random(size=(batch, n), dtype=dtype)
    blocks = max(1, n // 32)
    pos = rng.integers(0, blocks, size=batch) * 32 + min(32, n) - 1
    x[np.arange(batch), pos] = spike
    return x


def scan_input_normal(n: int, batch: int, dtype, seed: int = 0) -> np.ndarray:
    """Standard-normal values (mixed signs) drawn in float64 and rounded to
    float32 or float64, shape [batch][n]."""
    return np.random.default_rng(seed).standard_normal(size=(batch, n)).astype(np.dtype(dtype))


def scan_input_dyadic(n: int, batch: int, seed: int = 0):
    """float64 values k * 2^-20, integer k uniform on [0, 2^20), shape
    [batch][n]; returns (k as int64, values).  Every partial sum of up to 2^33
    such values is exact in float64, so any summation order gives the same
    bits."""
    k = np.random.default_rng(seed).integers(0, 1 << 20, size=(batch, n))
    return k, k.astype(np.float64) * 2.0 ** -20


def tridiag_input(n: int, batch: int, dtype, seed: int = 0):
    """Diagonally dominant tridiagonal systems with a known solution.

    Returns (a, b, c, d, x_true), each [batch][n] of ``dtype``.  Draw order:
    a, c, the diagonal margin u ~ U[1, 2], then x_true.  d is A x_true in
    float64 on the rounded a, b, c, x_true (a[:, 0] and c[:, -1] multiply
    absent unknowns and do not enter d), then rounded to ``dtype``.
    """
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    a = rng.uniform(-1.0, 1.0, size=(batch, n)).astype(dtype)
    c = rng.uniform(-1.0, 1.0, size=(batch, n)).astype(dtype)
    u = rng.uniform(1.0, 2.0, size=(batch, n))
    b = (np.abs(a.astype(np.float64)) + np.abs(c.astype(np.float64)) + u).astype(dtype)
    x = rng.uniform(-1.0, 1.0, size=(batch, n)).astype(dtype)
    a64, b64, c64, x64 = (v.astype(np.float64) for v in (a, b, c, x))
    d64 = b64 * x64
    d64[:, 1:] += a64[:, 1:] * x64[:, :-1]
    d64[:, :-1] += c64[:, :-1] * x64[:, 1:]
    return a, b, c, d64.astype(dtype), x


def batch_for_total(n: int, total: int) -> int:
    """Number of problems of size n that make up `total` elements."""
    return max(1, total // n)
