"""Serving policy on the CPU with a fake device and a fake clock: HBM budget
never exceeded, FIFO admission, grouping, every request completes."""
import pytest

from paper_2304_14492_amd import serve


def _reqs(n, gap, sizes=((48, 64, 10), (96, 128, 20), (192, 256, 30))):
    out = []
    for i in range(n):
        H, W, nm = sizes[i % len(sizes)]
        out.append(serve.Request(rid=i, t_arrival=i * gap, H=H, W=W, nmax=nm))
    return out


def _run(reqs, budget, max_inflight=4, max_batch=8):
    clock = serve.FakeClock()
    dev = serve.FakeDevice(clock)
    sch = serve.Scheduler(dev, budget, max_inflight=max_inflight, max_batch=max_batch)
    done = serve.run_stream(reqs, sch, clock=clock, sleep=lambda: clock.advance(1e-5))
    return sch, dev, done


def test_all_complete_within_budget_fifo():
    reqs = _reqs(200, 2e-5)
    budget = 12 * 192 * 256 * 3  # about three large requests
    sch, dev, done = _run(reqs, budget)
    assert len(done) == 200
    assert sch.peak_used <= budget
    assert sch.used == 0
    admits = sorted(done, key=lambda r: r.rid)
    for a, b in zip(admits, admits[1:]):
        assert a.t_admit <= b.t_admit  # FIFO
    for r in done:
        assert r.t_arrival <= r.t_admit <= r.t_done
        assert r.result == ("done", r.rid)


def test_tiny_budget_serialises():
    reqs = _reqs(30, 1e-6, sizes=((100, 100, 10),))
    budget = 12 * 100 * 100  # exactly one request
    sch, dev, done = _run(reqs, budget)
    assert len(done) == 30
    assert all(len(ln.reqs) == 1 for ln in dev.launched)
    # service intervals never overlap
    spans = sorted((ln.handle, ln.t_launch) for ln in dev.launched)
    for (end_a, _), (_, start_b) in zip(spans, spans[1:]):
        assert start_b >= end_a - 1e-12


def test_grouping_same_plan():
    reqs = [serve.Request(rid=i, t_arrival=0.0, H=64, W=64, nmax=8) for i in range(20)]
    sch, dev, done = _run(reqs, 10**9, max_inflight=4, max_batch=8)
    assert len(done) == 20
    assert max(len(ln.reqs) for ln in dev.launched) == 8


def test_oversized_request_rejected():
    clock = serve.FakeClock()
    sch = serve.Scheduler(serve.FakeDevice(clock), budget_bytes=1000)
    with pytest.raises(ValueError):
        sch.submit(serve.Request(rid=0, t_arrival=0.0, H=100, W=100, nmax=4))


def test_latency_stats():
    reqs = _reqs(100, 1e-4)
    sch, dev, done = _run(reqs, 10**9)
    st = serve.latency_stats(done)
    assert st["count"] == 100
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["p999_ms"]


def test_zero_budget_requests_time_out():
    # the budget drops to 0 (memory held elsewhere): nothing is admitted, and
    # every request expires once it has waited timeout_s; restoring the
    # budget serves later requests normally
    clock = serve.FakeClock()
    dev = serve.FakeDevice(clock)
    sch = serve.Scheduler(dev, budget_bytes=10**9, timeout_s=1e-3)
    sch.set_budget(0)
    first = _reqs(10, 1e-5)
    done = serve.run_stream(first, sch, clock=clock, sleep=lambda: clock.advance(1e-5))
    assert done == [] and dev.launched == []
    assert sorted(r.rid for r in sch.expired) == list(range(10))
    for r in sch.expired:
        assert r.status == "timeout" and r.result is None
        assert 1e-3 < r.t_done - r.t_arrival <= 1e-3 + 2e-5
    sch.set_budget(10**9)
    later = [serve.Request(rid=100 + i, t_arrival=i * 1e-5, H=48, W=64, nmax=10) for i in range(5)]
    done = serve.run_stream(later, sch, clock=clock, sleep=lambda: clock.advance(1e-5))
    assert sorted(r.rid for r in done) == [100 + i for i in range(5)]
    assert all(r.status == "done" for r in done)
    assert sch.used == 0


def test_full_queue_refuses_with_busy():
    clock = serve.FakeClock()
    dev = serve.FakeDevice(clock)
    sch = serve.Scheduler(dev, budget_bytes=10**9, max_waiting=3)
    sch.set_budget(0)
    for i in range(3):
        sch.submit(serve.Request(rid=i, t_arrival=0.0, H=48, W=64, nmax=10))
    r = serve.Request(rid=3, t_arrival=0.0, H=48, W=64, nmax=10)
    with pytest.raises(serve.SchedulerBusy):
        sch.submit(r)
    assert r.status == "busy" and len(sch.waiting) == 3
    # through run_stream the refused requests are collected, the rest served
    sch.set_budget(10**9)
    rejected = []
    burst = [serve.Request(rid=10 + i, t_arrival=0.0, H=48, W=64, nmax=10) for i in range(6)]
    done = serve.run_stream(burst, sch, clock=clock, sleep=lambda: clock.advance(1e-5), rejected=rejected)
    assert len(done) + len(rejected) == 9
    assert all(r.status == "busy" for r in rejected) and len(rejected) >= 1
    assert sch.used == 0


def test_idle_sleep_until_next_arrival():
    clock = serve.FakeClock()
    dev = serve.FakeDevice(clock)
    sch = serve.Scheduler(dev, budget_bytes=10**9)
    slept = []

    def idle(dt):
        slept.append(dt)
        clock.advance(dt)

    reqs = [serve.Request(rid=i, t_arrival=i * 0.01, H=48, W=64, nmax=10) for i in range(5)]
    done = serve.run_stream(reqs, sch, clock=clock, sleep=lambda: clock.advance(1e-5), idle_sleep=idle)
    assert len(done) == 5
    # idle gaps of ~10 ms are slept through (waking 0.2 ms early), never past an arrival
    assert len(slept) >= 4 and all(0 < dt < 0.01 for dt in slept)
    for r in done:
        assert r.t_admit - r.t_arrival <= 2e-5
