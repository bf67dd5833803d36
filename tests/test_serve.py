"""Serving loop logic on the CPU with a fake executor (oracle flows, scripted delays)."""
import numpy as np
import pytest

import oracle
import synth
from paper_1306_2461_amd.serve import BudgetExceeded, Server, poisson_arrivals
from serve_fake import FakeClock, FakeExecutor


def _frames(stream, n, size):
    return [f for f, _, _ in synth.stream_frames(stream, n, size=size)]


def test_stream_order_and_results_match_oracle():
    clock = FakeClock()
    ex = FakeExecutor(2, 3, 2, clock=clock)
    srv = Server(ex, clock=clock)
    fr = {s: _frames(s, 4, (40, 48)) for s in (0, 1)}
    reqs = {s: [srv.submit(s, f) for f in fr[s]] for s in (0, 1)}
    srv.drain()
    for s in (0, 1):
        assert [r.has_flow for r in reqs[s]] == [False, True, True, True]
        for t in range(1, 4):
            u, v = oracle.flow(fr[s][t - 1], fr[s][t], 2, 3, 2)
            assert np.array_equal(reqs[s][t].u, u) and np.array_equal(reqs[s][t].v, v)
    # one frame per stream per push: 4 pushes of 2
    assert ex.pushes == [2, 2, 2, 2]


def test_late_arrivals_join_next_push():
    clock = FakeClock()
    ex = FakeExecutor(1, 2, 1, delay=1.0, clock=clock)
    srv = Server(ex, clock=clock)
    frames = [_frames(s, 2, (24, 24)) for s in range(3)]
    srv.submit(0, frames[0][0])
    assert srv.step() == 1                      # push 1 in flight
    clock.advance(0.5)
    srv.submit(1, frames[1][0])
    srv.submit(2, frames[2][0])
    srv.submit(0, frames[0][1])
    assert srv.step() == 3                      # arrivals during push 1 batch together
    assert len(srv.inflight) == 2 and srv.poll() == 0
    clock.advance(0.5)
    assert srv.poll() == 1
    clock.advance(0.5)
    assert srv.poll() == 3


def test_admission_by_budget_waits_then_admits():
    clock = FakeClock()
    per = FakeExecutor(1, 2, 1).session_bytes(32, 32)
    ex = FakeExecutor(1, 2, 1, budget_bytes=2 * per + 10, delay=0.5, clock=clock)
    srv = Server(ex, clock=clock)
    f = {s: _frames(s, 2, (32, 32)) for s in range(3)}
    for s in range(3):
        srv.submit(s, f[s][0])
    assert srv.step() == 2                      # third stream waits for budget
    assert len(srv.pending) == 1 and ex.resident == 2 * per
    srv.drain(0)
    srv.close_stream(0)
    assert ex.resident == per
    assert srv.step() == 1                      # now admitted
    assert [a[1] for a in srv.admission_log].count("open") == 3


def test_rejections_do_not_poison_other_streams():
    clock = FakeClock()
    per = FakeExecutor(1, 2, 1).session_bytes(32, 32)
    ex = FakeExecutor(1, 2, 1, budget_bytes=per + 1, clock=clock)
    srv = Server(ex, clock=clock)
    good = _frames(0, 3, (32, 32))
    big = np.zeros((64, 64), np.uint8)           # needs more than the whole budget
    rq = [srv.submit(0, good[0]), srv.submit(1, big), srv.submit(0, good[1])]
    bad_size = srv.submit(0, np.zeros((16, 16), np.uint8))
    rq.append(srv.submit(0, good[2]))
    srv.drain()
    assert bad_size.error and "differs" in bad_size.error
    assert rq[1].error and "budget" in rq[1].error
    assert [r.has_flow for r in (rq[0], rq[2], rq[3])] == [False, True, True]
    assert len(srv.rejected) == 2


def test_slow_executor_grows_queue_and_p99():
    clock = FakeClock()
    ex = FakeExecutor(1, 2, 1, delay=0.05, clock=clock)
    srv = Server(ex, clock=clock)
    streams = [_frames(s, 6, (24, 24)) for s in range(2)]
    arr = poisson_arrivals(streams, rate_per_stream=100.0, seed=1)
    for t, s, f in arr:                          # everything arrives before any completion
        srv.submit(s, f, t)
    clock.t = max(a[0] for a in arr)
    while srv.pending or srv.inflight:
        srv.step()
        if not srv.poll():
            srv.ex.wait(srv.inflight[0][0])
    st = srv.stats()
    assert st["flows"] == 10 and st["p99_ms"] >= st["p50_ms"] > 0


def test_poisson_arrivals_keep_stream_order():
    streams = [[np.full((2, 2), i, np.uint8) for i in range(5)] for _ in range(3)]
    arr = poisson_arrivals(streams, 250.0)
    assert len(arr) == 15 and all(a[0] <= b[0] for a, b in zip(arr, arr[1:]))
    for s in range(3):
        vals = [int(f[0, 0]) for t, sid, f in arr if sid == s]
        assert vals == sorted(vals)


def test_busy_executor_keeps_order_and_keep_predicate():
    """A full staging ring makes the executor refuse a push (Busy): the requests stay pending in
    order and go out after an earlier push completes; flows of requests not kept are dropped."""
    clock = FakeClock()
    ex = FakeExecutor(1, 2, 1, delay=1.0, clock=clock, ring=1)
    srv = Server(ex, clock=clock, keep=lambda r: r.stream_id == 0)
    fr = {s: _frames(s, 3, (24, 24)) for s in (0, 1)}
    reqs = {s: [srv.submit(s, f) for f in fr[s]] for s in (0, 1)}
    assert srv.step() == 2                       # push 1: first frames of both streams
    assert srv.step() == 0 and srv.busy          # ring of one is full
    assert len(srv.pending) == 4 and ex.busy_count == 1
    srv.drain()
    assert ex.pushes == [2, 2, 2]
    for t in (1, 2):
        u, v = oracle.flow(fr[0][t - 1], fr[0][t], 1, 2, 1)
        assert np.array_equal(reqs[0][t].u, u) and reqs[0][t].has_flow
        assert reqs[1][t].u is None and reqs[1][t].has_flow


def test_inflight_bound_merges_arrivals_into_one_push():
    """With the in-flight bound reached, frames that arrive wait on the host and go out together
    in one push once an earlier push completes; without the bound each goes out on its own."""
    for bound, expect in ((1, [1, 3]), (None, [1, 1, 1, 1])):
        clock = FakeClock()
        ex = FakeExecutor(1, 2, 1, delay=1.0, clock=clock)
        srv = Server(ex, clock=clock, max_inflight=bound)
        fr = {s: _frames(s, 1, (24, 24)) for s in range(4)}
        srv.submit(0, fr[0][0])
        srv.step()
        for s in (1, 2, 3):
            clock.advance(0.1)
            srv.submit(s, fr[s][0])
            srv.step()
            assert srv.busy == (bound is not None)
        srv.drain()
        assert ex.pushes == expect, (bound, ex.pushes)
        assert len(srv.done) == 4 and all(not r.has_flow for r in srv.done)


def test_open_stream_admits_ahead_and_checks_size():
    clock = FakeClock()
    ex = FakeExecutor(1, 2, 1, delay=0.5, clock=clock, budget_bytes=3 * (2 * 24 * 24 * 2 + 16 * 24 * 24))
    srv = Server(ex, clock=clock)
    assert srv.open_stream(0, (24, 24)) and srv.open_stream(1, (24, 24))
    assert ex.resident == 2 * ex.session_bytes(24, 24) and len(srv.admission_log) == 2
    with pytest.raises(ValueError):
        srv.open_stream(0, (32, 32))
    with pytest.raises(BudgetExceeded):
        srv.open_stream(2, (480, 640))           # never fits
    assert srv.open_stream(3, (24, 24)) and not srv.open_stream(4, (24, 24))   # full for now
    fr = _frames(0, 2, (24, 24))
    reqs = [srv.submit(0, f) for f in fr]
    srv.drain()
    assert ex.pushes == [1, 1] and reqs[1].has_flow and len(srv.admission_log) == 3
