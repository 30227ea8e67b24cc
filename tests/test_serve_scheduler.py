"""Serving scheduler logic on the CPU, against a test-only fake executor whose
steps finish at scripted times on a fake clock and whose results come from
the oracle. (The product has no CPU path: this executor lives in tests/.)"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_00332_amd import synth
from paper_2305_00332_amd.serve import Request, Scheduler, latency_summary, poisson_requests


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Step duration = base + per_point * points; optional failing step ids."""

    def __init__(self, clock, pool, ws_per_req=1000, base=0.001, per_point=1e-9, fail_steps=()):
        self.clock = clock
        self.pool = pool
        self.ws_per_req = ws_per_req
        self.base = base
        self.per_point = per_point
        self.fail_steps = set(fail_steps)
        self.launched = []
        self.n_steps = 0

    def series_len(self, s):
        return len(self.pool[s])

    def request_ws(self, r):
        return self.ws_per_req * (1 + r.n_out // 1000)

    def reserve(self, reqs):
        return {"bytes": sum(self.request_ws(r) for r in reqs)}

    @staticmethod
    def token_bytes(token):
        return token["bytes"]

    def release(self, token):
        pass

    def launch(self, reqs, slot, token):
        sid = self.n_steps
        self.n_steps += 1
        self.launched.append((sid, slot, [r.rid for r in reqs], self.clock.t))
        dur = self.base + self.per_point * sum(r.n for r in reqs)
        return {"sid": sid, "end": self.clock.t + dur, "reqs": list(reqs)}

    def poll(self, h):
        return self.clock.t >= h["end"]

    def collect(self, h):
        if h["sid"] in self.fail_steps:
            raise RuntimeError("injected device failure")
        return [oracle.minmaxlttb(self.pool[r.series][r.lo: r.hi], r.n_out, r.r_ps) for r in h["reqs"]]


def _pool():
    return [synth.to_numpy(synth.random_walk(n, 100 + i)) for i, n in enumerate([5000, 20000, 777, 50000])]


def _drive(sched, reqs, dt=0.0002, limit=100.0):
    """Advance the fake clock, submitting at arrival times, until all complete."""
    clock = sched.clock
    reqs = sorted(reqs, key=lambda r: r.arrival)
    sched.start()
    i = 0
    while i < len(reqs) or not sched.idle():
        while i < len(reqs) and reqs[i].arrival <= sched.now():
            sched.submit(reqs[i])
            i += 1
        sched.tick()
        clock.t += dt
        assert clock.t < limit
    return sched.completed


def _reqs(pool, count, rate, seed):
    return poisson_requests(rate, count, [len(p) for p in pool], seed, n_out_range=(3, 400), min_len=10)


def test_every_result_is_the_request_alone():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool)
    sched = Scheduler(ex, n_slots=2, ws_budget=10 ** 9, clock=clock)
    done = _drive(sched, _reqs(pool, 200, 3000, 1))
    assert len(done) == 200
    for r in done:
        assert r.error is None
        want = oracle.minmaxlttb(pool[r.series][r.lo: r.hi], r.n_out, r.r_ps)
        assert np.array_equal(r.result, want)
    assert max(ex_b for ex_b in sched.batch_sizes) > 1  # requests were batched
    assert sched.max_in_flight == 2  # steps overlapped


def test_admission_by_workspace_queues_instead_of_failing():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, ws_per_req=1000, base=0.01)
    budget = 3000  # room for at most three requests (n_out < 1000) at a time
    sched = Scheduler(ex, n_slots=4, ws_budget=budget, clock=clock)
    seen_max = [0]
    orig_tick = sched.tick

    def tick():
        orig_tick()
        assert sched.ws_in_use <= budget
        seen_max[0] = max(seen_max[0], sched.ws_in_use)

    sched.tick = tick
    reqs = [Request(i, 0, 0, 1000, 100, 2, arrival=0.0) for i in range(12)]
    done = _drive(sched, reqs)
    assert all(r.error is None for r in done) and len(done) == 12
    assert seen_max[0] == budget


def test_slots_bound_in_flight_steps_and_are_reused():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=0.005)
    sched = Scheduler(ex, n_slots=2, ws_budget=10 ** 9, max_batch=1, clock=clock)
    done = _drive(sched, [Request(i, 1, 0, 5000, 50, 4, arrival=0.0) for i in range(9)])
    assert len(done) == 9 and all(r.error is None for r in done)
    assert sched.max_in_flight == 2
    assert {s for _, s, _, _ in ex.launched} == {0, 1}


def test_late_arrivals_join_while_other_steps_run():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=0.05)
    sched = Scheduler(ex, n_slots=2, ws_budget=10 ** 9, clock=clock)
    reqs = [Request(0, 0, 0, 5000, 10, 2, arrival=0.0)] + \
           [Request(i, 1, 0, 20000, 10, 2, arrival=0.01 + 0.001 * i) for i in range(1, 6)]
    _drive(sched, reqs)
    first_step_end = 0.0 + 0.05
    # the later arrivals were admitted on the second slot before the first step ended
    second = [t for sid, slot, rids, t in ex.launched if 1 in rids][0]
    assert second < first_step_end


def test_invalid_and_oversized_requests_fail_alone():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, ws_per_req=1000)
    sched = Scheduler(ex, n_slots=2, ws_budget=5000, clock=clock)
    reqs = [
        Request(0, 0, 0, 1000, 100, 4, arrival=0.0),
        Request(1, 0, 0, 1000, 2, 4, arrival=0.0),        # n_out < 3
        Request(2, 0, 0, 1000, 100, 1, arrival=0.0),      # r_ps < 2
        Request(3, 0, 4000, 6000, 100, 4, arrival=0.0),   # outside the series
        Request(4, 0, 0, 1000, 100_000, 4, arrival=0.0),  # workspace above the whole budget
        Request(5, 2, 0, 777, 100, 4, arrival=0.0),
    ]
    done = {r.rid: r for r in _drive(sched, reqs)}
    assert done[0].error is None and done[5].error is None
    for rid in (1, 2, 3, 4):
        assert done[rid].error is not None and done[rid].result is None


def test_injected_step_failure_fails_only_that_step():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=0.01, fail_steps={1})
    sched = Scheduler(ex, n_slots=1, ws_budget=10 ** 9, max_batch=2, clock=clock)
    reqs = [Request(i, 1, 0, 20000, 100, 4, arrival=0.0) for i in range(6)]
    done = {r.rid: r for r in _drive(sched, reqs)}
    failed = {rid for rid, r in done.items() if r.error}
    assert failed == set(ex.launched[1][2])
    assert all(done[rid].result is not None for rid in done if rid not in failed)


def test_cancel_queued_request():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=1.0)
    sched = Scheduler(ex, n_slots=1, ws_budget=10 ** 9, max_batch=1, clock=clock)
    sched.start()
    for i in range(3):
        sched.submit(Request(i, 0, 0, 1000, 10, 2, arrival=0.0))
    sched.tick()  # request 0 admitted, 1 and 2 queued
    assert sched.cancel(2) and not sched.cancel(0)
    while not sched.idle():
        clock.t += 0.1
        sched.tick()
    by = {r.rid: r for r in sched.completed}
    assert by[2].error == "cancelled" and by[0].error is None and by[1].error is None


def test_fifo_admission_order():
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=0.01)
    sched = Scheduler(ex, n_slots=1, ws_budget=10 ** 9, max_batch=3, clock=clock)
    reqs = [Request(i, i % 4, 0, 700, 10, 2, arrival=0.0001 * i) for i in range(10)]
    _drive(sched, reqs)
    order = [rid for _, _, rids, _ in ex.launched for rid in rids]
    assert order == sorted(order)


def test_latency_summary_fields():
    pool = _pool()
    clock = FakeClock()
    sched = Scheduler(FakeExecutor(clock, pool), n_slots=2, ws_budget=10 ** 9, clock=clock)
    s = latency_summary(_drive(sched, _reqs(pool, 50, 1000, 3)))
    assert s["requests"] == 50 and s["p99_ms"] >= s["p50_ms"] > 0 and s["errors"] == 0


def test_free_slots_share_the_queue():
    """Queued requests are spread over the free slots: two requests and four
    free slots give two steps of one; twelve give four steps of three."""
    pool = _pool()
    clock = FakeClock()
    ex = FakeExecutor(clock, pool, base=0.05)
    sched = Scheduler(ex, n_slots=4, ws_budget=10 ** 9, clock=clock)
    sched.start()
    for i in range(2):
        sched.submit(Request(i, 0, 0, 1000, 10, 2, arrival=0.0))
    sched.tick()
    assert sorted(len(r) for _, _, r, _ in ex.launched) == [1, 1]
    while not sched.idle():
        clock.t += 0.01
        sched.tick()
    ex.launched.clear()
    for i in range(12):
        sched.submit(Request(10 + i, 0, 0, 1000, 10, 2, arrival=clock.t))
    sched.tick()
    assert [len(r) for _, _, r, _ in ex.launched] == [3, 3, 3, 3]


class ShortArenaExecutor(FakeExecutor):
    """reserve() refuses steps of more than `fit` requests (a fragmented arena)."""

    def __init__(self, *a, fit=2, **k):
        super().__init__(*a, **k)
        self.fit = fit
        self.refused = 0

    def reserve(self, reqs):
        if len(reqs) > self.fit:
            self.refused += 1
            return None
        return super().reserve(reqs)


def test_step_shrinks_when_its_exact_memory_does_not_fit():
    pool = _pool()
    clock = FakeClock()
    ex = ShortArenaExecutor(clock, pool, base=0.01, fit=2)
    sched = Scheduler(ex, n_slots=1, ws_budget=10 ** 9, clock=clock)
    reqs = [Request(i, 1, 0, 20000, 100, 4, arrival=0.0) for i in range(7)]
    done = _drive(sched, reqs)
    assert len(done) == 7 and all(r.error is None for r in done)
    assert ex.refused > 0 and max(sched.batch_sizes) == 2
    order = [rid for _, _, rids, _ in ex.launched for rid in rids]
    assert order == sorted(order)  # requests put back keep their place


def test_arena_first_fit_alignment_and_merging():
    from paper_2305_00332_amd.serve import Arena

    a = Arena(4096)
    b1 = a.alloc(1)
    b2 = a.alloc(300)
    b3 = a.alloc(256)
    assert b1 == (0, 256) and b2 == (256, 512) and b3 == (768, 256)
    assert a.used == 1024
    assert a.alloc(4096) is None
    a.release(b2)
    assert a.alloc(600) == (1024, 768)  # the 512-byte hole is too small
    assert a.alloc(512) == (256, 512)  # ... but fits this one exactly
    for blk in ((0, 256), (256, 512), (768, 256), (1024, 768)):
        a.release(blk)
    assert a.free == [(0, 4096)] and a.used == 0
    assert a.alloc(4096) == (0, 4096)
