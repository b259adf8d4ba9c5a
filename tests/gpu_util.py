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


def scan_bound(x, unit, exclusive=False, oracle_rounds=False):
    """Elementwise bound for a blocked-tree sum scan in a precision with unit
    roundoff `unit`: (log2 N + 32) units times the running sum of |x|.

    exclusive: the lane network adds thread totals, so an exclusive output
    carries the rounding of a sum running to the end of its thread's chunk
    (at most 31 elements on): the running sum is taken there.
    oracle_rounds: the oracle itself rounds (float64 inputs summed left to
    right in float64): add its i * unit at element i."""
    n = x.shape[1]
    s = np.cumsum(np.abs(x.astype(np.float64)), axis=1)
    if exclusive:
        s = s[:, np.minimum(np.arange(n) + 31, n - 1)]
    k = np.ceil(np.log2(n)) + 32
    if oracle_rounds:
        k = k + np.arange(n)
    return k * unit * s
