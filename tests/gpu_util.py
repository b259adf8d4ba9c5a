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
