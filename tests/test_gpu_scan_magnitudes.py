"""GPU parity of the float scans on inputs of mixed magnitude and sign (Sec.
III, "Scan Operator", inclusive and exclusive forms).

Each output must be within (ceil(log2 N) + 32) unit roundoffs times the sum
of |x_j| over exactly the elements it is defined by (j <= i inclusive, j < i
exclusive), plus the float64 oracle's own left-to-right rounding.  Two input
classes reach what uniform positive inputs cannot:

* uniform[0, 1) with one 1e6 at the end of a 32-element block per row: an
  output just before the spike, inside the same thread's chunk, has a small
  defining sum while the thread's chunk total is huge;
* standard-normal values: partial sums cancel, so the running sum of |x|
  and not the sum itself sets the scale.

For float32 the spiked recipe has an exact float64 oracle (multiples of
2^-24 below 1 plus an integer, at most 44 significant bits).
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, scan_bound, to_dev, to_host

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
DT = {"f32": (np.float32, ppx.F32, U32), "f64": (np.float64, ppx.F64, U64)}


def _inputs(kind, n, batch, dtype, seed):
    if kind == "spiked":
        return inputs.scan_input_spiked(n, batch, dtype, seed=seed)
    return inputs.scan_input_normal(n, batch, dtype, seed=seed)


@pytest.mark.parametrize("n", [64, 1024, 16384])
@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["spiked", "normal"])
def test_every_config_definition_bound(cuda, n, dt, kind):
    import torch
    dtype, code, unit = DT[dt]
    batch = 9
    x = _inputs(kind, n, batch, dtype, seed=n + (7 if kind == "spiked" else 8) + (100 if dt == "f64" else 0))
    xd = to_dev(x, cuda)
    y = torch.empty_like(xd)
    worst = 0.0
    for excl in (False, True):
        ref = oracle.scan(x, exclusive=excl)
        bound = scan_bound(x, unit, exclusive=excl, oracle_unit=U64)
        f = ppx.scan_exclusive_batched if excl else ppx.scan_batched
        for cfg in ppx.enumerate_configs(ppx.OP_SCAN, code, n):
            banner(f"scan {kind} {dt} n={n} excl={excl} {cfg}")
            f(xd, y, n, batch, code, cfg)
            out = to_host(y).astype(np.float64)
            err = np.abs(out - ref)
            if excl:
                assert np.all(out[:, 0] == 0.0), f"{cfg}: first exclusive output not 0"
            bad = err > bound
            assert not bad.any(), (f"{cfg} excl={excl}: {np.count_nonzero(bad)} outputs over the bound, "
                                   f"worst ratio {np.max(err / np.maximum(bound, 1e-300)):.3e}")
            worst = max(worst, float(np.max(err / np.maximum(bound, 1e-300))))
    print(f"scan {kind} {dt} n={n}: worst error / bound {worst:.3e}")


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_full_size_spiked_null_config(cuda, dt):
    """Benchmark sweep size (2^24 elements), the configuration a NULL config
    resolves to, every element against the definition-shaped bound."""
    dtype, code, unit = DT[dt]
    n = 1024
    batch = (1 << 24) // n
    x = inputs.scan_input_spiked(n, batch, dtype, seed=41)
    xd = to_dev(x, cuda)
    import torch
    y = torch.empty_like(xd)
    for excl in (False, True):
        banner(f"scan full spiked {dt} n={n} excl={excl}")
        (ppx.scan_exclusive_batched if excl else ppx.scan_batched)(xd, y, n, batch, code)
        out = to_host(y).astype(np.float64)
        err = np.abs(out - oracle.scan(x, exclusive=excl))
        assert np.all(err <= scan_bound(x, unit, exclusive=excl, oracle_unit=U64))
