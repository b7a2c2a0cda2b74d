"""Scheduling logic of the continuous-batching server, on the CPU.

A stand-in executor replaces the GPU: each batch costs 100 bytes per query
word, finishes a fixed delay after launch on a manual clock, and returns the
sum of its query's word ids.  No device work happens here.
"""
import numpy as np
import pytest

from paper_2107_06433_amd.serve import RejectedError, Request, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    def __init__(self, clock, delay=1.0):
        self.clock, self.delay = clock, delay
        self.launched = []
        self.live = 0
        self.max_live = 0

    def cost(self, reqs):
        return 100 * sum(len(r.ids) for r in reqs)

    def launch(self, reqs):
        self.launched.append([r.rid for r in reqs])
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"t": self.clock() + self.delay, "reqs": reqs}

    def done(self, h):
        return self.clock() >= h["t"]

    def results(self, h):
        return [int(r.ids.sum()) for r in h["reqs"]]

    def release(self, h):
        self.live -= 1


def req(n, base=0):
    return Request(ids=np.arange(base, base + n, dtype=np.int32), weights=np.ones(n, np.float32), arrival=0.0)


def test_fifo_budget_and_slots():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, mem_budget=1000, max_batch=3, max_inflight=2)
    futs = [sch.submit(req(n, 10 * i)) for i, n in enumerate([2, 3, 4, 1, 5, 2, 2])]
    used = []
    for step in range(20):
        clock.t = step * 0.5
        sch.poll(clock.t)
        sch.admit(clock.t)
        used.append(sch.used)
        assert sch.used <= 1000
        assert len(sch.inflight) <= 2
    assert all(f.done() for f in futs)
    # FIFO: batches take consecutive request ids in order
    flat = [rid for b in ex.launched for rid in b]
    assert flat == sorted(flat) == list(range(7))
    assert all(len(b) <= 3 for b in ex.launched)
    assert ex.max_live <= 2
    assert [f.result() for f in futs] == [int(np.arange(10 * i, 10 * i + n).sum())
                                          for i, n in enumerate([2, 3, 4, 1, 5, 2, 2])]


def test_memory_frees_on_completion_and_later_requests_get_admitted():
    clock = Clock()
    ex = FakeExecutor(clock, delay=1.0)
    sch = Scheduler(ex, mem_budget=500, max_batch=8, max_inflight=4)
    a = sch.submit(req(4))      # 400 bytes
    sch.admit(0.0)
    b = sch.submit(req(3))      # 300 bytes: does not fit beside a
    sch.admit(0.1)
    assert len(sch.inflight) == 1 and len(sch.pending) == 1
    clock.t = 1.0
    sch.poll(1.0)
    assert a.done() and sch.used == 0
    sch.admit(1.0)
    assert len(sch.inflight) == 1 and not sch.pending
    clock.t = 2.0
    sch.poll(2.0)
    assert b.result() == 3


def test_request_larger_than_budget_is_rejected_and_queue_moves_on():
    clock = Clock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, mem_budget=250, max_batch=4, max_inflight=2)
    big = sch.submit(req(5))
    small = sch.submit(req(2))
    sch.admit(0.0)
    with pytest.raises(RejectedError):
        big.result(timeout=0)
    clock.t = 1.0
    sch.poll(1.0)
    assert small.result(timeout=0) == 1
    assert len(sch.rejected) == 1


def test_drain_finishes_in_flight_work():
    clock = Clock()
    ex = FakeExecutor(clock, delay=0.3)
    sch = Scheduler(ex, mem_budget=10_000, max_batch=2, max_inflight=1)
    futs = [sch.submit(req(2, i)) for i in range(5)]

    def tick():
        clock.t += 0.1
        return clock.t

    sch.drain(tick)
    assert all(f.done() for f in futs) and not sch.inflight and sch.used == 0
    assert sch.batches == 3


class FailingExecutor(FakeExecutor):
    """Fails in cost() for queries holding word id 666, in launch() for id 777
    and while polling a batch that holds id 888."""

    def cost(self, reqs):
        if any(666 in r.ids for r in reqs):
            raise ValueError("bad query")
        return super().cost(reqs)

    def launch(self, reqs):
        if any(777 in r.ids for r in reqs):
            raise RuntimeError("launch failed")
        h = super().launch(reqs)
        h["boom"] = any(888 in r.ids for r in reqs)
        return h

    def done(self, h):
        if h["boom"]:
            raise RuntimeError("device error")
        return super().done(h)


def test_executor_errors_resolve_futures_and_keep_the_budget():
    clock = Clock()
    ex = FailingExecutor(clock, delay=0.5)
    sch = Scheduler(ex, mem_budget=10_000, max_batch=1, max_inflight=2)
    ok1 = sch.submit(req(2))
    bad_cost = sch.submit(Request(ids=np.array([1, 666], np.int32), weights=np.ones(2, np.float32), arrival=0.0))
    bad_launch = sch.submit(Request(ids=np.array([777], np.int32), weights=np.ones(1, np.float32), arrival=0.0))
    bad_poll = sch.submit(Request(ids=np.array([888], np.int32), weights=np.ones(1, np.float32), arrival=0.0))
    ok2 = sch.submit(req(3, 10))
    for step in range(10):
        clock.t = 0.5 * step
        sch.poll(clock.t)
        sch.admit(clock.t)
    assert ok1.result(timeout=0) == 1 and ok2.result(timeout=0) == 33
    with pytest.raises(ValueError):
        bad_cost.result(timeout=0)
    with pytest.raises(RuntimeError, match="launch failed"):
        bad_launch.result(timeout=0)
    with pytest.raises(RuntimeError, match="device error"):
        bad_poll.result(timeout=0)
    assert sch.used == 0 and not sch.inflight and not sch.pending


def test_invalid_newcomer_does_not_block_a_forming_batch():
    clock = Clock()
    ex = FailingExecutor(clock, delay=0.1)
    sch = Scheduler(ex, mem_budget=10_000, max_batch=4, max_inflight=1)
    a = sch.submit(req(2))
    bad = sch.submit(Request(ids=np.array([666], np.int32), weights=np.ones(1, np.float32), arrival=0.0))
    b = sch.submit(req(2, 5))
    sch.admit(0.0)
    assert ex.launched == [[0, 2]]
    with pytest.raises(ValueError):
        bad.result(timeout=0)
    clock.t = 1.0
    sch.poll(1.0)
    assert a.result(timeout=0) == 1 and b.result(timeout=0) == 11


def test_server_thread_survives_failures_and_rejects_oversized_queries():
    import time as _time

    from paper_2107_06433_amd.serve import Server

    class WallExecutor(FailingExecutor):
        def __init__(self):
            super().__init__(_time.perf_counter, delay=0.01)

    srv = Server(None, 10.0, 15, executor=WallExecutor(), mem_budget=10_000, max_batch=1, max_inflight=2,
                 max_query_len=8)
    too_long = srv.submit(np.arange(9), np.ones(9))
    empty = srv.submit([], [])
    bad = srv.submit([666], [1.0])
    boom = srv.submit([777], [1.0])
    good = [srv.submit(np.arange(i, i + 3), np.ones(3)) for i in range(5)]
    srv.close()
    with pytest.raises(ValueError, match="at most 8"):
        too_long.result(timeout=5)
    with pytest.raises(ValueError):
        empty.result(timeout=5)
    with pytest.raises(ValueError):
        bad.result(timeout=5)
    with pytest.raises(RuntimeError):
        boom.result(timeout=5)
    assert [f.result(timeout=5) for f in good] == [3 * i + 3 for i in range(5)]
