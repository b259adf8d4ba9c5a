"""CPU tests of the tuning engine (include/ppx_tune.h): the occupancy model and
the analytical guideline against the paper's GM20B figures, the Bayesian
search on fake evaluators, the GP posterior against scikit-learn, Expected
Improvement against its closed form, Phi, and the tune cache."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import ppx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gm20b():
    """GM20B limits from Sec. II: 64 warps, 32 blocks, 64K registers in four
    partitions allocated per warp in 256-register granules, 64 KB shared per
    SM, 48 KB per block, 2 SMs."""
    return ppx.DeviceModel(wave_size=32, partitions=4, regs_per_partition=16384, reg_granule=256,
                           max_waves_per_cu=64, max_blocks_per_cu=32, lds_per_cu=65536,
                           lds_per_block=49152, lds_granule=256, num_cus=2)


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def test_gm20b_occupancy_table():
    m = gm20b()
    for warps, regs, shared, occ, blocks in (map(int, r) for r in _rows("gm20b_occupancy.txt")):
        b, w = ppx.occupancy(m, ppx.Resource(warps * 32, regs, shared))
        assert b == blocks, (warps, regs, shared)
        assert round(100 * w / 64) == occ


def test_gfx950_model_matches_compiler_occupancy():
    # the compiler reports 4 waves/SIMD for 128 VGPRs and 2 for 196
    m = ppx.device_model_gfx950()
    assert ppx.occupancy(m, ppx.Resource(1024, 128, 0)) == (1, 16)
    assert ppx.occupancy(m, ppx.Resource(512, 196, 0)) == (1, 8)
    assert ppx.occupancy(m, ppx.Resource(64, 16, 0)) == (32, 32)
    assert ppx.occupancy(m, ppx.Resource(256, 32, 81920)) == (2, 8)


# Register use per thread that the paper states for the GM20B kernels:
# P = 2 fits in 32 registers (Sec. V-A); P = 4 needs 40 for the FFT and the
# tridiagonal solvers (Sec. V-A, V-C) but stays within 32 for the scan (Sec. V-B).
def _candidates(op, n):
    cands, res = [], []
    for P in (2, 4):
        for L in (32, 64, 128, 256, 512, 1024):
            if (P * L) % n:
                continue
            G = P * L // n
            if op == "fft":
                regs, variants = (32 if P == 2 else 40), [(P * L, P * L * 8)]
            elif op == "scan":
                regs, variants = 32, [(32 * G, 32 * G * 4)]  # 32 slots per problem
            else:
                regs = 32 if P == 2 else 40
                variants = [(G * n, G * n * 16)]  # 4 coefficients of 4 bytes
                if n // P <= 32:
                    variants.append((0, 0))  # the problem fits in a warp: shuffles
            for S, shared in variants:
                cands.append(ppx.Config(P if op == "fft" else 2, P, L, G, S, 0))
                res.append(ppx.Resource(L, regs, shared))
    return cands, res


def test_guideline_reproduces_paper_choices():
    m = gm20b()
    for op, n, S, P, L in _rows("gm20b_analytical_configs.txt"):
        n, S, P, L = int(n), int(S), int(P), int(L)
        cands, res = _candidates(op, n)
        k = ppx.analytical_pick(m, cands, res, batch=(1 << 26) // n, flags=0)
        c = cands[k]
        assert (c.lds_elems, c.elems_per_thread, c.threads_per_block) == (S, P, L), (op, n, c)


def test_guideline_prefers_radix_over_blocks():
    # step 4: a radix-4 candidate at 75% occupancy beats a radix-2 one at 100%
    m = gm20b()
    cands = [ppx.Config(2, 2, 64, 2, 128, 0), ppx.Config(4, 4, 64, 4, 256, 0)]
    res = [ppx.Resource(64, 32, 1024), ppx.Resource(64, 40, 2048)]
    assert ppx.analytical_pick(m, cands, res, batch=1 << 20) == 1
    # but not when the larger radix drops occupancy below 60% (step 3 is then moot)
    res[1] = ppx.Resource(64, 64, 2048)
    assert ppx.analytical_pick(m, cands, res, batch=1 << 20) == 0


def test_guideline_step3_maximises_occupancy_then_P():
    m = gm20b()
    cands = [ppx.Config(2, 2, 32, 1, 64, 0), ppx.Config(2, 4, 32, 2, 128, 0),
             ppx.Config(2, 8, 1024, 128, 0, 0)]
    res = [ppx.Resource(32, 64, 512), ppx.Resource(32, 64, 1024), ppx.Resource(1024, 64, 0)]
    # all at 50%: the tie goes to the larger P
    assert ppx.analytical_pick(m, cands, res, batch=1 << 20) == 2


def test_grid_fill_term():
    m = ppx.device_model_gfx950()
    big = ppx.Config(2, 32, 64, 16, 0, 0)
    small = ppx.Config(2, 2, 64, 1, 0, 0)
    res = [ppx.Resource(64, 40, 0), ppx.Resource(64, 10, 0)]
    # 2^16 problems in blocks of 16 give 4096 blocks, fewer than the 256 CUs x
    # 32 resident blocks; blocks of 1 fill the chip
    assert ppx.analytical_pick(m, [big, small], res, 1 << 16, flags=0) == 0
    assert ppx.analytical_pick(m, [big, small], res, 1 << 16, flags=ppx.ANALYTICAL_GRID_FILL) == 1


# ------------------------------------------------------------ Bayesian search

def _fft_space():
    return ppx.enumerate_configs(ppx.OP_FFT, ppx.C64, 1024)


def _planted_cost(c, opt=(16, 256, 4, 0)):
    lr, ll, lg = math.log2(c.radix), math.log2(c.threads_per_block), math.log2(c.problems_per_block)
    o = (math.log2(opt[0]), math.log2(opt[1]), math.log2(opt[2]))
    return 100.0 * (1 + 0.3 * (lr - o[0]) ** 2 + 0.2 * (ll - o[1]) ** 2 + 0.1 * (lg - o[2]) ** 2
                    + 0.5 * abs(c.algo - opt[3]))


def test_bo_finds_planted_optimum_with_few_evaluations():
    # The stop rule (5 evaluations without progress) can end a search early,
    # so the property is statistical over seeds.
    cands = _fft_space()
    costs = [_planted_cost(c) for c in cands]
    opt = int(np.argmin(costs))
    found, evals, ratios = 0, [], []
    for seed in range(20):
        best, order, vals = ppx.bo_search(cands, _planted_cost, seed=seed)
        found += best == opt
        evals.append(len(order))
        ratios.append(costs[best] / costs[opt])
        assert len(set(order)) == len(order)  # never re-evaluates a candidate
        assert vals == pytest.approx([costs[i] for i in order])
    assert found >= 16
    assert np.mean(ratios) <= 1.2
    assert np.mean(evals) < len(cands) / 4


def test_bo_stop_rule_five_without_progress():
    cands = _fft_space()
    calls = []

    def flat(c):
        calls.append(1)
        return 7.0  # nothing ever improves on the first sample
    best, order, _ = ppx.bo_search(cands, flat, n_init=3, patience=5, seed=0)
    assert len(order) == 3 + 5 and len(calls) == 8


def test_bo_failed_runs_get_a_high_time():
    cands = _fft_space()

    def sometimes_fails(c):
        return -1.0 if c.radix == 2 else _planted_cost(c)
    best, order, vals = ppx.bo_search(cands, sometimes_fails, seed=3)
    worst_ok = max(v for i, v in zip(order, vals) if cands[i].radix != 2)
    for i, v in zip(order, vals):
        if cands[i].radix == 2:
            assert v == pytest.approx(10 * worst_ok)
    assert cands[best].radix != 2


def test_bo_respects_max_evals_and_seed():
    cands = _fft_space()
    a = ppx.bo_search(cands, _planted_cost, max_evals=6, seed=11)
    b = ppx.bo_search(cands, _planted_cost, max_evals=6, seed=11)
    assert len(a[1]) == 6 and a == b


def test_exhaustive_is_the_phi_reference():
    # Phi of the exhaustive choice is 1 by construction
    cands = _fft_space()
    costs = np.array([_planted_cost(c) for c in cands])
    e = [costs.min() / costs[int(np.argmin(costs))]] * 11
    assert ppx.phi(e) == 1.0


# ------------------------------------------------------------ GP and EI

def test_gp_posterior_matches_sklearn():
    from sklearn.gaussian_process import GaussianProcessRegressor
    from sklearn.gaussian_process.kernels import ConstantKernel, Matern, WhiteKernel
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (12, 4))
    y = np.sin(3 * X[:, 0]) + X[:, 1] ** 2 - X[:, 2] * X[:, 3]
    Xq = rng.uniform(0, 1, (7, 4))
    ls = np.array([0.4, 0.7, 1.3, 0.9])
    sf2, noise = 1.7, 1e-3
    k = (ConstantKernel(sf2, "fixed") * Matern(length_scale=ls, length_scale_bounds="fixed", nu=2.5)
         + WhiteKernel(noise, "fixed"))
    g = GaussianProcessRegressor(kernel=k, optimizer=None, alpha=0.0, normalize_y=False).fit(X, y)
    mu_ref, sd_ref = g.predict(Xq, return_std=True)
    mu, var = ppx.gp_posterior(X, y, ls, sf2, noise, Xq)
    assert np.allclose(mu, mu_ref, atol=1e-9)
    assert np.allclose(var + noise, sd_ref ** 2, atol=1e-9)  # sklearn's std includes the noise


def test_expected_improvement_closed_form():
    from scipy.stats import norm
    for mu, sd, best in ((0.3, 0.2, 0.5), (1.0, 0.5, 0.2), (-1.0, 2.0, 0.0)):
        z = (best - mu) / sd
        ref = (best - mu) * norm.cdf(z) + sd * norm.pdf(z)
        assert ppx.expected_improvement(mu, sd, best) == pytest.approx(ref, rel=1e-12)
    assert ppx.expected_improvement(1.0, 0.0, 2.0) == pytest.approx(1.0)
    assert ppx.expected_improvement(3.0, 0.0, 2.0) == 0.0


def test_phi_matches_oracle_definition():
    for e in ([1.0], [1.0, 0.5], [0.9, 0.7, 1.0, 0.95]):
        assert ppx.phi(e) == pytest.approx(oracle.phi(e), rel=1e-15)


# ------------------------------------------------------------ tune cache

def test_tune_cache_round_trip(tmp_path):
    ppx.clear_tune_cache()
    p = tmp_path / "cache.txt"
    p.write_text("# comment\n"
                 "gfx950 0 3 1024 -1 8 8 128 1 1024 0 123.5 0\n"
                 "gfx950 2 1 256 1 2 4 64 1 512 1 40.0 2\n"
                 "gfx950 0 3 1024 0 3 8 128 1 0 0 1.0 0\n"   # invalid radix: skipped
                 "gfx942 0 3 64 -1 4 4 64 4 256 0 1.0 0\n")  # another architecture
    assert ppx.load_tune_cache(str(p)) == 2
    c = ppx.tuned_config(ppx.OP_FFT, ppx.C64, 1024)
    assert c.as_tuple() == (8, 8, 128, 1, 1024, 0)
    assert ppx.resolve_config(ppx.OP_FFT, ppx.C64, 1024, 1 << 15).as_tuple() == c.as_tuple()
    assert ppx.tuned_config(ppx.OP_TRIDIAG, ppx.F32, 256, algo=1).algo == 1
    assert ppx.tuned_config(ppx.OP_TRIDIAG, ppx.F32, 256) is None
    q = tmp_path / "saved.txt"
    ppx.save_tune_cache(str(q))
    ppx.clear_tune_cache()
    assert ppx.load_tune_cache(str(q)) == 2
    assert ppx.tuned_config(ppx.OP_FFT, ppx.C64, 1024).as_tuple() == c.as_tuple()
    ppx.clear_tune_cache()


def test_tune_cache_keeps_large_fft_plans(tmp_path):
    ppx.clear_tune_cache()
    p = tmp_path / "plans.txt"
    p.write_text("gfx950 plan 1048576 8 16 8 4 16 304.3 0\n"
                 "gfx950 plan 8388608 11 16 16 4 8 373.5 0\n"
                 "gfx950 plan 65536 8 4 16 16 16 1.0 0\n"       # radix 4: not a valid plan, skipped
                 "gfx950 plan 16384 7 16 16 16 16 1.0 0\n")     # not a large size: skipped
    assert ppx.load_tune_cache(str(p)) == 2
    assert ppx.tuned_fft_plan(1 << 20).as_tuple() == (8, 16, 8, 4, 16)
    assert ppx.tuned_fft_plan(1 << 16) is None
    q = tmp_path / "saved.txt"
    ppx.save_tune_cache(str(q))
    ppx.clear_tune_cache()
    assert ppx.tuned_fft_plan(1 << 20) is None
    assert ppx.load_tune_cache(str(q)) == 2
    assert ppx.tuned_fft_plan(1 << 23).as_tuple() == (11, 16, 16, 4, 8)
    ppx.clear_tune_cache()


# ---------------------------------------------------------------- online BO

def _cost(c):
    """A deterministic synthetic cost with structure in every feature."""
    import math
    return (1.0 + 0.3 * abs(math.log2(c.threads_per_block) - 8) + 0.2 * abs(math.log2(c.problems_per_block) - 2)
            + 0.05 * c.algo + 0.01 * c.radix)


def _drive(t):
    order = []
    c, cand = t.next()
    while cand:
        order.append(c.as_tuple())
        t.report(_cost(c))
        c, cand = t.next()
    return order, c


def test_online_session_replays_the_offline_search():
    """One evaluation at a time, the online session proposes exactly the
    candidates the offline learned search evaluates (same BO state, seed and
    stopping rule) and ends on its best."""
    for op, dt, n, algo in ((ppx.OP_SCAN, ppx.I32, 1024, -1), (ppx.OP_FFT, ppx.C64, 4096, -1),
                            (ppx.OP_TRIDIAG, ppx.F32, 256, ppx.TRI_CR)):
        cands = [c for c in ppx.enumerate_configs(op, dt, n)
                 if algo < 0 or ppx.tri_family(c.algo) == ppx.tri_family(algo)]
        best, order, _ = ppx.bo_search(cands, _cost, patience=5, min_rel=0.01, seed=0x231016214)
        t = ppx.OnlineTuner(op, dt, n, 1 << 16, algo=algo)
        got, final = _drive(t)
        assert got == [cands[i].as_tuple() for i in order]
        assert final.as_tuple() == cands[best].as_tuple()
        st = t.status()
        assert st["converged"] and st["evals"] == len(order) and st["best_cost"] == _cost(cands[best])
        t.close()


def test_online_session_protocol():
    t = ppx.OnlineTuner(ppx.OP_SCAN, ppx.F32, 2048, 4096, max_evals=4)
    c0, cand = t.next(explore=False)  # before any evaluation: the analytical choice
    assert not cand and ppx.config_valid(ppx.OP_SCAN, ppx.F32, 2048, c0)
    with pytest.raises(ppx.PpxError):
        t.report(1.0)                  # nothing pending
    c1, cand = t.next()
    assert cand
    c2, cand2 = t.next()               # a cost is awaited: the current choice
    assert not cand2 and c2.as_tuple() == c0.as_tuple()
    t.report(-1.0)                     # a failed run
    for _ in range(3):
        c, cand = t.next()
        assert cand
        t.report(2.0)
    c, cand = t.next()                 # max_evals reached
    assert not cand and t.status()["converged"] and t.status()["evals"] == 4
    assert t.status()["best_cost"] == 2.0
    t.close()


def test_server_online_flag():
    with pytest.raises(ppx.PpxError):
        ppx.Server(1 << 20, flags=ppx.SERVE_ONLINE_TUNE)  # needs the per-request mode
    s = ppx.Server(1 << 24, flags=ppx.SERVE_PER_REQUEST | ppx.SERVE_ONLINE_TUNE | ppx.SERVE_NULL_DEVICE)
    ids = [s.submit(ppx.make_job(ppx.OP_SCAN, ppx.I32, 1024, 64, 1 << 20, None)) for _ in range(3)]
    for _ in range(4):
        s.progress()
    assert sorted(c.id for c in s.poll()) == ids
    assert s.online_stats() == dict(sessions=0, evaluations=0, converged=0)  # nothing is timed without a GPU
    s.close()
