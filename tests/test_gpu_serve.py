"""GPU tests of the request loop: every job served in the mix equals the same
job launched alone (bitwise), sampled jobs match the oracle, and the
per-request baseline serves the same trace within tolerance."""
import numpy as np
import pytest

import oracle
from paper_2310_16214_amd import ppx
from paper_2310_16214_amd.serve_bench import Pools, make_trace
from tests.gpu_util import banner, fft_tol, scan_f32_bound, to_dev

pytestmark = pytest.mark.gpu


def _small_trace(pools, njobs, seed):
    trace = make_trace(njobs, 200000.0, seed, pools)
    # keep it quick: cap the batch counts
    out = []
    for job, t, m in trace:
        job.batch = min(job.batch, 64)
        m["batch"] = job.batch
        m["elems"] = job.n * job.batch
        m["bytes"] = {"fft": 16, "scan": 8, "tridiag": 20}[m["op"]] * m["elems"]
        out.append((job, t, m))
    return out


def _host_out(meta):
    return np.empty((meta["batch"], meta["n"]),
                    dtype=np.complex64 if meta["op"] == "fft" else np.float32)


def _oracle_check(pools, meta, y):
    n, batch, off = meta["n"], meta["batch"], meta["offset"]
    if meta["op"] == "fft":
        x = pools.fft[off:off + n * batch].cpu().numpy().reshape(batch, n)
        assert oracle.rel_l2(y, oracle.dft(x)).max() <= fft_tol(n)
    elif meta["op"] == "scan":
        x = pools.scan[off:off + n * batch].cpu().numpy().reshape(batch, n)
        assert np.all(np.abs(y.astype(np.float64) - oracle.scan(x)) <= scan_f32_bound(x))
    else:
        coeffs = [v[off:off + n * batch].cpu().numpy().reshape(batch, n) for v in pools.tri]
        assert oracle.tridiag_residual(*coeffs, y).max() <= 1e-4


@pytest.mark.parametrize("mode", [ppx.SERVE_FUSED, ppx.SERVE_PER_REQUEST])
def test_served_jobs_match_alone_and_oracle(cuda, mode):
    import torch
    pools = Pools(cuda, seed=4)
    trace = _small_trace(pools, 40, seed=9)
    banner(f"serve mode={mode} jobs={len(trace)}")
    srv = ppx.Server(1 << 30, max_inflight=2, flags=mode)
    comps = srv.replay([(j, t) for j, t, _ in trace], auto_release=False)
    outs = []
    for c, (_, _, m) in zip(comps, trace):
        outs.append(srv.read(c.id, _host_out(m)))
    srv.close()
    for k, ((job, _, m), y) in enumerate(zip(trace, outs)):
        if mode == ppx.SERVE_FUSED:
            # the same job alone in its own mixed launch: identical bits
            alone = torch.empty(m["batch"] * m["n"] * (2 if m["op"] == "fft" else 1),
                                dtype=torch.float32, device=cuda)
            j2 = ppx.Job.from_buffer_copy(job)
            j2.out = alone.data_ptr()
            ppx.launch_mixed([j2])
            torch.cuda.synchronize()
            a = alone.cpu().numpy().view(y.dtype).reshape(y.shape)
            assert np.array_equal(a, y), (k, m)
        if k % 4 == 0:
            _oracle_check(pools, m, y)


def test_backpressure_with_a_tight_budget(cuda):
    pools = Pools(cuda, seed=5)
    trace = _small_trace(pools, 30, seed=2)
    biggest = max(m["bytes"] for _, _, m in trace) + 4096
    banner("serve tight budget")
    srv = ppx.Server(biggest, max_inflight=2, flags=ppx.SERVE_FUSED)
    comps = srv.replay([(j, t) for j, t, _ in trace], auto_release=True)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(trace) and st["peak_used_bytes"] <= biggest
    assert all(c.complete_us >= c.admit_us >= c.arrival_us for c in comps)


def test_online_tuning_serves_correct_results(cuda):
    """Per-request serving with online learned tuning: three repeated job
    classes large enough to be timed; every served output agrees with the
    same job solved alone (and sampled problems with the oracle), whatever
    candidate served it, and each class's search makes progress."""
    import torch
    pools = Pools(cuda, seed=6)
    rng = np.random.default_rng(12)
    trace = []
    for k in range(90):
        op = ("fft", "scan", "tridiag")[k % 3]
        n, batch = {"fft": (1024, 1024), "scan": (1024, 1024), "tridiag": (256, 4096)}[op]
        elems = n * batch
        if op == "fft":
            off = int(rng.integers(0, pools.fft.numel() - elems + 1)) & ~1
            job = ppx.make_job(ppx.OP_FFT, ppx.C64, n, batch, pools.fft.data_ptr() + 8 * off, None)
        elif op == "scan":
            off = int(rng.integers(0, pools.scan.numel() - elems + 1)) & ~3
            job = ppx.make_job(ppx.OP_SCAN, ppx.F32, n, batch, pools.scan.data_ptr() + 4 * off, None)
        else:
            off = int(rng.integers(0, pools.tri[0].numel() - elems + 1)) & ~3
            p = [v.data_ptr() + 4 * off for v in pools.tri]
            job = ppx.make_job(ppx.OP_TRIDIAG, ppx.F32, n, batch, p[0], None, algo=ppx.TRI_CR,
                               b=p[1], c=p[2], d=p[3])
        trace.append((job, 0.0, dict(op=op, n=n, batch=batch, offset=off)))
    banner(f"serve online tuning jobs={len(trace)}")
    srv = ppx.Server(1 << 32, max_inflight=2, flags=ppx.SERVE_PER_REQUEST | ppx.SERVE_ONLINE_TUNE)
    comps = srv.replay([(j, t) for j, t, _ in trace], auto_release=False)
    outs = [srv.read(c.id, _host_out(m)) for c, (_, _, m) in zip(comps, trace)]
    st = srv.online_stats()
    srv.close()
    assert st["sessions"] == 3 and 9 <= st["evaluations"] <= len(trace)
    for k, ((job, _, m), y) in enumerate(zip(trace, outs)):
        n, batch, off = m["n"], m["batch"], m["offset"]
        if m["op"] == "fft":
            x = pools.fft[off:off + n * batch]
            ref = torch.empty_like(x)
            ppx.fft_batched(x, ref, n, batch, -1)
            assert oracle.rel_l2(y, ref.cpu().numpy().reshape(batch, n)).max() <= 2 * fft_tol(n)
            if k < 3:
                xs = x.cpu().numpy().reshape(batch, n)[:2]
                assert oracle.rel_l2(y[:2], oracle.dft(xs)).max() <= fft_tol(n)
        elif m["op"] == "scan":
            x = pools.scan[off:off + n * batch].cpu().numpy().reshape(batch, n)
            assert np.all(np.abs(y.astype(np.float64) - oracle.scan(x)) <= scan_f32_bound(x))
        else:
            coeffs = [v[off:off + n * batch].cpu().numpy().reshape(batch, n) for v in pools.tri]
            assert oracle.tridiag_residual(*coeffs, y).max() <= 1e-4


@pytest.mark.parametrize("mode", [ppx.SERVE_FUSED, ppx.SERVE_PER_REQUEST])
def test_served_exclusive_and_float64_scans(cuda, mode):
    """Scan jobs of both forms in int32 and float64 (dyadic values, exact)
    through either mode of the request loop, against the oracle exactly."""
    from paper_2310_16214_amd import inputs
    jobs, hosts = [], []
    for k, (dt, form, n, batch) in enumerate([(ppx.I32, 1, 512, 40), (ppx.F64, 1, 4096, 9),
                                               (ppx.F64, 0, 64, 500), (ppx.I32, 0, 16384, 2)]):
        if dt == ppx.F64:
            _, x = inputs.scan_input_dyadic(n, batch, seed=70 + k)
        else:
            x = inputs.scan_input(n, batch, np.int32, seed=70 + k)
        xd = to_dev(x, cuda)
        jobs.append((ppx.make_job(ppx.OP_SCAN, dt, n, batch, xd, None, algo=form), xd))
        hosts.append((x, form))
    banner(f"serve scans mode={mode}")
    srv = ppx.Server(1 << 28, max_inflight=2, flags=mode)
    comps = srv.replay([(j, 0.0) for j, _ in jobs], auto_release=False)
    for c, (x, form) in zip(comps, hosts):
        y = srv.read(c.id, np.empty_like(x))
        assert np.array_equal(y, oracle.scan(x, exclusive=form == 1)), (x.dtype, form)
    srv.close()
