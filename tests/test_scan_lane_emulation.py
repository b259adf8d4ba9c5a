"""CPU regression test for the rounding behaviour of the scan kernels' lane
arithmetic (no GPU, no library call).

The kernels' float arithmetic is emulated step by step in numpy float32,
with the kernels' order of operations: thread-serial scan of P values, a
wave64 lane network over the thread totals (Kogge-Stone: row shifts 1, 2, 4,
8 inside 16-lane rows, then the two row broadcasts; or Ladner-Fischer:
broadcast of the lower half's last lane at each level), one LDS total per
wave for problems spanning several waves, then the add-back of the thread's
prefix.  The thread's exclusive prefix is the previous lane's inclusive value
(a one-lane shift).  The test checks that this keeps every output within the
definition-shaped bound of Sec. III's scan (a multiple of the unit roundoff
times the sum of |x_j| over j <= i, or j < i for the exclusive form), on the
input that defeats the other way of forming the prefix (the lane's inclusive
value minus its own total), and that the test notices that other way.
"""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs
from tests.gpu_util import scan_bound

F = np.float32


def lanes_ks(tot):
    """Kogge-Stone lane network over one wave (64 values), segment = wave."""
    x = tot.copy()
    lane = np.arange(64)
    for d in (1, 2, 4, 8):
        y = np.where(lane % 16 >= d, np.roll(x, d), F(0))
        x = np.where(lane >= d, x + y, x).astype(F)
    row = lane // 16
    x = np.where((row == 1) | (row == 3), x + np.where(row == 1, x[15], x[47]), x).astype(F)
    x = np.where(row >= 2, x + x[31], x).astype(F)
    return x


def lanes_lf(tot):
    """Ladner-Fischer lane network over one wave: at level d the lanes with
    bit d set add the last lane of the lower half of their 2d-block."""
    x = tot.copy()
    lane = np.arange(64)
    for d in (1, 2, 4, 8, 16, 32):
        src = (lane & ~(2 * d - 1)) | (d - 1)
        x = np.where(lane & d, x + x[src], x).astype(F)
    return x


def emulate(x, P, network, exclusive, subtract):
    """One problem of n float32 values, n / P threads of P values each."""
    n = x.size
    T = n // P
    assert T % 64 == 0, "whole waves only"
    v = x.reshape(T, P).astype(F).copy()
    tot = np.empty(T, F)
    for t in range(T):  # 1. thread-serial scan
        if exclusive:
            run = F(0)
            for j in range(P):
                e = v[t, j]
                v[t, j] = run
                run = F(run + e)
            tot[t] = run
        else:
            for j in range(1, P):
                v[t, j] = F(v[t, j] + v[t, j - 1])
            tot[t] = v[t, P - 1]
    prefix = np.empty(T, F)
    wave_tot = []
    for w in range(T // 64):  # 2. lane network, per wave
        inc = network(tot[64 * w:64 * w + 64])
        if subtract:
            pre = (inc - tot[64 * w:64 * w + 64]).astype(F)
        else:
            pre = np.concatenate([[F(0)], inc[:-1]]).astype(F)
        prefix[64 * w:64 * w + 64] = pre
        wave_tot.append(inc[63])
    for w in range(T // 64):  # 3. totals of the earlier waves, in order
        for u in range(w):
            prefix[64 * w:64 * w + 64] = (prefix[64 * w:64 * w + 64] + wave_tot[u]).astype(F)
    return (v + prefix[:, None]).astype(F).reshape(n)  # 4. add-back


def worst_ratio(n, P, network, exclusive, subtract, trials=40, seed=0):
    x = inputs.scan_input_spiked(n, trials, np.float32, seed=seed)
    ref = oracle.scan(x, exclusive=exclusive)
    bound = scan_bound(x, 2.0 ** -24, exclusive=exclusive)
    out = np.stack([emulate(x[b], P, network, exclusive, subtract) for b in range(trials)]).astype(np.float64)
    err = np.abs(out - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    return float(r.max())


@pytest.mark.parametrize("network", [lanes_ks, lanes_lf], ids=["ks", "lf"])
@pytest.mark.parametrize("P,n", [(4, 256), (8, 512), (2, 256), (4, 1024)])
@pytest.mark.parametrize("exclusive", [False, True])
def test_shifted_prefix_within_definition_bound(network, P, n, exclusive):
    assert worst_ratio(n, P, network, exclusive, subtract=False) <= 1.0


@pytest.mark.parametrize("network", [lanes_ks, lanes_lf], ids=["ks", "lf"])
@pytest.mark.parametrize("exclusive", [False, True])
def test_subtracted_prefix_is_caught(network, exclusive):
    # the cancelling form: the spiked input drives it far over the bound
    assert worst_ratio(256, 4, network, exclusive, subtract=True) > 10.0


def test_networks_are_scans():
    # both emulated networks compute the inclusive scan exactly on integers
    t = np.arange(1, 65, dtype=F)
    assert np.array_equal(lanes_ks(t), np.cumsum(t))
    assert np.array_equal(lanes_lf(t), np.cumsum(t))
