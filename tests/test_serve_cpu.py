"""CPU tests of the request loop's bookkeeping (null-device server): FIFO
admission by HBM budget, back-pressure, release, continuous batching and
latency records."""
import pytest

from paper_2310_16214_amd import ppx

ADDR = 1 << 20  # fake, aligned device addresses: never dereferenced


def _job(n, batch, op=ppx.OP_SCAN, dtype=ppx.I32, out=None):
    return ppx.make_job(op, dtype, n, batch, ADDR, out, b=ADDR, c=ADDR, d=ADDR)


def test_admission_respects_budget_and_fifo():
    # each job: 1024 * 64 int32 in + out = 512 KiB; budget holds three
    s = ppx.Server(3 * 512 * 1024, max_inflight=4, flags=ppx.SERVE_NULL_DEVICE)
    ids = [s.submit(_job(1024, 64)) for _ in range(5)]
    assert s.progress() == 3                      # three fit (one per launch: each launch
    st = s.stats()                                # takes at most budget / max_inflight)
    assert st["admitted"] == 3 and st["pending"] == 2 and st["launches"] == 3
    assert st["used_bytes"] == 3 * 512 * 1024
    assert s.progress() == 0                      # the launch completes; no room yet
    done = s.poll()
    assert [c.id for c in done] == ids[:3]
    s.release(ids[0])
    assert s.progress() == 1                      # one slot freed: the 4th job
    s.release(ids[1])
    s.release(ids[2])
    assert s.progress() == 1
    assert s.stats()["peak_used_bytes"] <= 3 * 512 * 1024


def test_launch_takes_its_share_of_the_budget():
    # budget for four jobs, two launches in flight: two launches of two jobs
    # each, so one is queued behind the other instead of one taking it all
    s = ppx.Server(4 * 512 * 1024, max_inflight=2, flags=ppx.SERVE_NULL_DEVICE)
    for _ in range(6):
        s.submit(_job(1024, 64))
    assert s.progress() == 4
    st = s.stats()
    assert st["launches"] == 2 and st["admitted"] == 4 and st["max_inflight_seen"] == 2
    # a job larger than the share still goes, alone
    s2 = ppx.Server(2 * 512 * 1024, max_inflight=4, flags=ppx.SERVE_NULL_DEVICE)
    big = s2.submit(_job(1024, 96))               # 768 KiB > 256 KiB share
    assert s2.progress() == 1 and s2.stats()["launches"] == 1
    s2.progress()
    assert [c.id for c in s2.poll()] == [big]


def test_large_job_is_delayed_not_overtaken():
    s = ppx.Server(1 << 20, max_inflight=4, flags=ppx.SERVE_NULL_DEVICE)
    a = s.submit(_job(1024, 64))          # 512 KiB
    big = s.submit(_job(1024, 96))        # 768 KiB: waits for a
    c = s.submit(_job(16, 1))             # tiny, but must not overtake big
    assert s.progress() == 1
    s.progress()
    assert [x.id for x in s.poll()] == [a]
    assert s.stats()["pending"] == 2
    s.release(a)
    assert s.progress() == 2              # big and then c, in order
    s.progress()
    assert [x.id for x in s.poll()] == [big, c]


def test_oversized_job_is_refused():
    s = ppx.Server(1 << 16, max_inflight=1, flags=ppx.SERVE_NULL_DEVICE)
    with pytest.raises(ppx.PpxError) as e:
        s.submit(_job(1024, 64))
    assert e.value.code == ppx.ENOMEM


def test_invalid_jobs_are_refused():
    s = ppx.Server(1 << 30, max_inflight=1, flags=ppx.SERVE_NULL_DEVICE)
    with pytest.raises(ppx.PpxError):
        s.submit(_job(1000, 4))
    with pytest.raises(ppx.PpxError):
        s.submit(_job(64, 4, op=ppx.OP_FFT, dtype=ppx.I32))
    with pytest.raises(ppx.PpxError):
        s.release(12345)


def test_continuous_batching_and_inflight_cap():
    s = ppx.Server(1 << 30, max_inflight=2, flags=ppx.SERVE_NULL_DEVICE)
    for _ in range(4):
        s.submit(_job(64, 8))
    assert s.progress() == 4                      # spread over the two free slots
    assert s.stats()["launches"] == 2
    for _ in range(5):
        s.submit(_job(64, 8))
    assert s.progress() == 5                      # the next step's arrivals: 3 + 2
    assert s.stats()["launches"] == 4
    one = ppx.Server(1 << 30, max_inflight=1, flags=ppx.SERVE_NULL_DEVICE)
    for _ in range(7):
        one.submit(_job(64, 8))
    assert one.progress() == 7                    # one slot: every pending job in one launch
    assert one.stats()["launches"] == 1
    per = ppx.Server(1 << 30, max_inflight=2, flags=ppx.SERVE_NULL_DEVICE | ppx.SERVE_PER_REQUEST)
    for _ in range(4):
        per.submit(_job(64, 8))
    assert per.progress() == 2                    # one job per launch, two launches in flight


def test_arena_reuses_released_memory():
    s = ppx.Server(4 << 20, max_inflight=1, flags=ppx.SERVE_NULL_DEVICE)
    outs = set()
    for _ in range(6):
        i = s.submit(_job(1024, 256))             # 1 MiB out + 1 MiB in
        s.progress()
        s.progress()
        (c,) = s.poll()
        outs.add(c.out)
        s.release(i)
    assert len(outs) == 1                         # first fit returns the same block


def test_replay_records_latencies_in_request_order():
    s = ppx.Server(1 << 30, max_inflight=2, flags=ppx.SERVE_NULL_DEVICE)
    reqs = [(_job(64, 4), 100.0 * k) for k in range(20)]
    comps = s.replay(reqs)
    assert len(comps) == 20
    for (job, t), c in zip(reqs, comps):
        assert c.complete_us >= c.admit_us >= c.arrival_us
    arr = [c.arrival_us for c in comps]
    assert arr == sorted(arr)
    assert s.stats()["released"] == 20 and s.stats()["used_bytes"] == 0


def test_scan_job_forms_are_validated():
    s = ppx.Server(1 << 24, flags=ppx.SERVE_NULL_DEVICE)
    for dt in (ppx.I32, ppx.F32, ppx.F64):
        for form in (ppx.JOB_SCAN_INCLUSIVE, ppx.JOB_SCAN_EXCLUSIVE):
            s.submit(ppx.make_job(ppx.OP_SCAN, dt, 256, 4, ADDR, None, algo=form))
    with pytest.raises(ppx.PpxError):
        s.submit(ppx.make_job(ppx.OP_SCAN, ppx.F32, 256, 4, ADDR, None, algo=2))
    with pytest.raises(ppx.PpxError):
        s.submit(ppx.make_job(ppx.OP_SCAN, ppx.C64, 256, 4, ADDR, None))
    s.close()
