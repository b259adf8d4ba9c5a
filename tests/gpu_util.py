"""Helpers shared by the GPU parity tests (no arithmetic of the operations)."""
import sys

import numpy as np


def banner(msg):
    """Print and flush the case name before a GPU step, so a failing run names it."""
    sys.stdout.write(f"\n[gpu-case] {msg}\n")
    sys.stdout.flush()


def to_dev(arr, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def fft_tol(n):
    """Per-problem relative-L2 bound for the FP32 FFT: 1e-5 * log2 N."""
    return 1e-5 * np.log2(n)


def scan_f32_bound(x):
    """Elementwise bound for an FP32 blocked-tree inclusive sum: (log2 N + 32)
    ulp-units (2^-23) times the running sum of |x|."""
    n = x.shape[1]
    return (np.ceil(np.log2(n)) + 32) * 2.0 ** -23 * np.cumsum(np.abs(x.astype(np.float64)), axis=1)


def scan_bound(x, unit, exclusive=False, oracle_unit=0.0):
    """Elementwise bound for a blocked-tree sum scan in a precision with unit
    roundoff `unit`: (ceil(log2 N) + 32) units times the sum of |x_j| over the
    elements the output is defined by (j <= i inclusive, j < i exclusive), so
    the first exclusive output must be exactly 0.

    oracle_unit: the oracle itself rounds (float64 inputs summed left to right
    in float64): add its i * oracle_unit at element i."""
    n = x.shape[1]
    s = np.cumsum(np.abs(x.astype(np.float64)), axis=1)
    if exclusive:
        s = np.concatenate([np.zeros_like(s[:, :1]), s[:, :-1]], axis=1)
    k = (np.ceil(np.log2(n)) + 32) * unit + np.arange(n) * oracle_unit
    return k * s


def tridiag_forward_check(a, b, c, d, x, ref):
    """Forward error of a tridiagonal solve x against the float64 oracle
    solution ref, per system, with the bound it must meet.

    For a strictly row diagonally dominant A, ||A^-1||_inf <= 1 / min_i
    (|b_i| - |a_i| - |c_i|) (Varah), with a_0 and c_{n-1} left out, so
    ||x - x*||_inf <= ||A^-1||_inf * ||A x - d||_inf for the exact solution
    x*.  The residual is formed in float64 on the stored coefficients; the
    oracle's own error (float64 Thomas on a system with kappa_inf <= 6) is
    covered by a 1e-12 relative allowance.  Returns (err, bound), each
    [batch], in the infinity norm."""
    a, b, c, d, x = (np.asarray(v, dtype=np.float64) for v in (a, b, c, d, x))
    a = a.copy()
    c = c.copy()
    a[:, 0] = 0.0
    c[:, -1] = 0.0
    r = b * x - d
    r[:, 1:] += a[:, 1:] * x[:, :-1]
    r[:, :-1] += c[:, :-1] * x[:, 1:]
    margin = np.min(np.abs(b) - np.abs(a) - np.abs(c), axis=1)
    assert np.all(margin > 0), "system not strictly diagonally dominant"
    err = np.max(np.abs(x - ref), axis=1)
    bound = np.max(np.abs(r), axis=1) / margin + 1e-12 * np.maximum(1.0, np.max(np.abs(ref), axis=1))
    return err, bound
