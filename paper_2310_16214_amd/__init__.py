"""Batched parallel-prefix kernels (FFT, scan, tridiagonal) for AMD MI355X.

The compute path is the C-ABI library ``libppx.so`` (hand-written HIP for
gfx950); :mod:`paper_2310_16214_amd.ppx` is its thin ctypes binding and
:mod:`paper_2310_16214_amd.inputs` the seeded workload generators.  Loading the
binding does not touch the GPU; the first call that needs the library raises if
it has not been built.
"""
__all__ = ["inputs", "ppx"]
