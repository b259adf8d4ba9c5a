"""GPU parity of the two-pass large-N FFT (16384 < N <= 2^23) against the
oracle: every plan at N = 2^15 and 2^16 on whole problems (every bin by its
definition), the tuned and the default plan on one whole problem at 2^17 and
2^18, every plan at 2^20 .. 2^23 (narrow pass-B tiles for columns of
more than 1024 values), the default plan at full size up to 2^23 and the
shipped tuned plans at 2^22 and 2^23 on one and three problems, on sampled
bins (each bin by its definition) plus Parseval, forward and inverse.  Bar:
per-problem relative L2 <= 1e-5 * log2 N."""
import os

import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import inputs, ppx
from tests.gpu_util import banner, fft_tol, to_dev, to_host

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(ppx.__file__), "tuned", "mi355x.txt")


def _run(x, n, batch, plan=None, direction=-1):
    import torch
    xd = to_dev(x, "cuda")
    y = torch.empty_like(xd)
    ppx.fft_batched_large(xd, y, n, batch, direction, plan)
    return to_host(y)


@pytest.mark.parametrize("n", [1 << 15, 1 << 16])
def test_every_plan_matches_oracle(cuda, n):
    batch = 2
    x = inputs.fft_input(n, batch, seed=n + 3)
    every = np.arange(n)  # all bins, computed in parallel over (problem, bin)
    ref = oracle.dft_bins(x, every)
    refi = oracle.dft_bins(x, every, inverse=True)
    plans = ppx.enumerate_fft_plans(n)
    assert plans
    worst = 0.0
    for p in plans:
        banner(f"fft large n={n} {p}")
        err = oracle.rel_l2(_run(x, n, batch, p), ref).max()
        erri = oracle.rel_l2(_run(x, n, batch, p, +1), refi).max()
        worst = max(worst, err, erri)
        assert err <= fft_tol(n) and erri <= fft_tol(n), (p, err, erri)
    print(f"n={n}: {len(plans)} plans, worst rel-L2 {worst:.3e}")


@pytest.mark.parametrize("ln", [17, 18])
def test_tuned_plan_every_bin(cuda, ln):
    """One problem at 2^17 and 2^18, the tuned (NULL) and the default plan,
    forward: every bin against its O(N) definition."""
    n = 1 << ln
    x = inputs.fft_input(n, 1, seed=ln + 60)
    ref = oracle.dft_bins(x, np.arange(n))
    for plan in (None, ppx.default_fft_plan(n)):
        banner(f"fft large n={n} every bin, plan {plan}")
        err = oracle.rel_l2(_run(x, n, 1, plan), ref).max()
        print(f"n={n} plan {plan}: rel-L2 {err:.3e} (bound {fft_tol(n):.1e})")
        assert err <= fft_tol(n), (plan, err)


def _sampled_bins(x, y, n, rng, problems, inverse=False):
    ks = np.unique(np.concatenate([[0, 1, n // 2, n - 1], rng.integers(0, n, 44)]))
    for b in problems:
        ref = oracle.dft_bins(x[b:b + 1], ks, inverse=inverse)[0]
        err = np.linalg.norm(y[b, ks] - ref) / np.linalg.norm(ref)
        assert err <= fft_tol(n), (b, err)


def _parseval(x, y, n):
    px = np.sum(np.abs(x.astype(np.complex128)) ** 2, axis=1) * n
    py = np.sum(np.abs(y.astype(np.complex128)) ** 2, axis=1)
    assert np.max(np.abs(py - px) / px) <= 2 * fft_tol(n)


@pytest.mark.parametrize("ln", [20, 21, 22, 23])
def test_every_plan_sampled_bins(cuda, ln):
    """Every plan, forward and inverse, two problems: 48 bins each by
    definition, every bin through Parseval."""
    n = 1 << ln
    batch = 2
    x = inputs.fft_input(n, batch, seed=ln + 40)
    ks = np.unique(np.concatenate([[0, 1, n // 2, n - 1], np.random.default_rng(ln).integers(0, n, 44)]))
    refs = {d: oracle.dft_bins(x, ks, inverse=d > 0) for d in (-1, +1)}  # [problem][bin]
    import torch
    xd = to_dev(x, cuda)
    yd = torch.empty_like(xd)
    kd = torch.from_numpy(ks).to(cuda)
    energy = np.sum(np.abs(x.astype(np.complex128)) ** 2, axis=1) * n  # Parseval: sum |X|^2
    plans = ppx.enumerate_fft_plans(n)
    assert plans
    for p in plans:
        for direction in (-1, +1):
            banner(f"fft large n={n} {p} dir={direction}")
            ppx.fft_batched_large(xd, yd, n, batch, direction, p)
            y_ks = to_host(yd[:, kd])
            err = np.linalg.norm(y_ks - refs[direction], axis=1) / np.linalg.norm(refs[direction], axis=1)
            assert err.max() <= fft_tol(n), (p, direction, err)
            e_gpu = (yd.to(torch.complex128).abs() ** 2).sum(dim=1).cpu().numpy()
            assert np.max(np.abs(e_gpu - energy) / energy) <= 2 * fft_tol(n), (p, direction)
    print(f"n={n}: {len(plans)} plans")


@pytest.mark.parametrize("ln", [17, 18, 19, 20, 21, 22, 23])
def test_default_plan_sampled_bins(cuda, ln):
    """Full 256 MiB call (2^25 / N problems); 3 problems checked on 48 bins
    each (their DFT by definition), the rest of the output through Parseval."""
    n = 1 << ln
    batch = (1 << 25) // n
    banner(f"fft large n={n} batch={batch} default plan")
    x = inputs.fft_input(n, batch, seed=ln)
    y = _run(x, n, batch)
    _sampled_bins(x, y, n, np.random.default_rng(ln), (0, batch // 2, batch - 1))
    _parseval(x, y, n)  # every problem: sum |X|^2 = N sum |x|^2


@pytest.fixture
def shipped_plans():
    ppx.clear_tune_cache()
    ppx.load_tune_cache(CACHE)
    yield
    ppx.clear_tune_cache()


@pytest.mark.parametrize("ln,batch", [(22, 1), (22, 3), (23, 1), (23, 3)])
def test_shipped_plan_few_problems(cuda, shipped_plans, ln, batch):
    """The shipped tuned plans at 2^22 and 2^23 on one and three problems,
    forward and inverse.  Their persistent passes run one workgroup per CU;
    where a row holds two grid-steps of tiles or more (both passes at 2^23),
    the steps take the row's line groups in turn, and with one or three rows
    the walk wraps from row to row at every problem boundary.  48 bins per
    problem by definition, every bin through Parseval."""
    n = 1 << ln
    plan = ppx.tuned_fft_plan(n)
    assert plan is not None
    x = inputs.fft_input(n, batch, seed=10 * ln + batch)
    rng = np.random.default_rng(10 * ln + batch)
    for direction in (-1, +1):
        banner(f"fft large n={n} batch={batch} shipped plan {plan} dir={direction}")
        y = _run(x, n, batch, plan, direction)
        _sampled_bins(x, y, n, rng, range(batch), inverse=direction > 0)
        _parseval(x, y, n)


def test_inverse_roundtrip_and_forwarding(cuda):
    import torch
    n, batch = 1 << 17, 3
    x = inputs.fft_input(n, batch, seed=17)
    xd = to_dev(x, cuda)
    f = torch.empty_like(xd)
    ppx.fft_batched(xd, f, n, batch, -1)  # forwards to the large path
    back = torch.empty_like(xd)
    ppx.fft_batched_large(f, back, n, batch, +1)
    err = oracle.rel_l2(to_host(back) / n, x).max()
    assert err <= 2 * fft_tol(n)
    with pytest.raises(ppx.PpxError) as e:
        ppx.fft_batched_large(xd, xd, n, batch, -1)
    assert e.value.code == ppx.EINVAL


def test_tuned_plan_is_used(cuda):
    n = 1 << 15
    best, us, evals, trace = ppx.tune_fft_large(n, 64, 0, reps=5)
    assert evals == len(ppx.enumerate_fft_plans(n)) and us > 0
    assert best.as_tuple() in [p.as_tuple() for p, _ in trace]
    x = inputs.fft_input(n, 2, seed=9)
    err = oracle.rel_l2(_run(x, n, 2), oracle.dft_bins(x, np.arange(n))).max()  # NULL plan: the tuned one
    assert err <= fft_tol(n)
