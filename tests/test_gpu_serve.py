"""Serving on the GPU: every request's result in the mix equals the same
request computed alone (single-series call; tolerance 0) and, on a sample, the
oracle; steps really overlap and batch; a tight workspace budget queues."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth
from paper_2305_00332_amd.serve import GpuExecutor, PlainGpuExecutor, Request, Scheduler, latency_summary, \
    poisson_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    lengths = synth.batch_lengths(32, 1e4, 2e6, 12)
    x, y, offsets = synth.batch_series(lengths, 12, device="cuda")
    torch.cuda.synchronize()
    return x, y, offsets, lengths


def _alone(pool, r):
    x, y, offsets, _ = pool
    o = int(offsets[r.series]) + r.lo
    return ops.minmaxlttb(y[o: o + r.n], r.n_out, r.r_ps, x=x[o: o + r.n]).cpu().numpy()


@pytest.mark.parametrize("executor", [GpuExecutor, PlainGpuExecutor])
def test_results_in_the_mix_equal_alone(pool, executor):
    x, y, offsets, lengths = pool
    ex = executor(y, offsets, lengths, x=x, n_slots=3)
    sched = Scheduler(ex, n_slots=3, ws_budget=64 << 20, max_batch=None if executor is GpuExecutor else 1)
    reqs = poisson_requests(20_000, 400, lengths, seed=5)
    done = sched.run_open_loop(reqs, timeout=120)
    assert len(done) == 400
    assert all(r.error is None for r in done), [r.error for r in done if r.error][:3]
    for r in done:
        assert np.array_equal(r.result, _alone(pool, r)), f"request {r.rid}"
    rng = np.random.default_rng(1)
    for i in rng.choice(400, size=20, replace=False):
        r = done[i]
        o = int(offsets[r.series]) + r.lo
        want = oracle.minmaxlttb(y[o: o + r.n].cpu().numpy(), r.n_out, r.r_ps, x[o: o + r.n].cpu().numpy())
        assert np.array_equal(r.result, want)
    if executor is GpuExecutor:
        assert sched.max_in_flight > 1
        assert max(sched.batch_sizes) > 1
    s = latency_summary(done)
    print(executor.__name__, s, flush=True)


def test_tight_budget_queues_and_bad_requests_fail_alone(pool):
    x, y, offsets, lengths = pool
    probe = GpuExecutor(y, offsets, lengths, x=x, n_slots=1, arena_bytes=1 << 20)
    one = probe.request_ws(Request(0, 0, 0, 10, 4000, 4))
    del probe
    ex = GpuExecutor(y, offsets, lengths, x=x, n_slots=2, arena_bytes=2 * one)
    sched = Scheduler(ex, n_slots=2)
    reqs = poisson_requests(50_000, 60, lengths, seed=9, n_out_range=(3000, 4000), r_ps_choices=(4,))
    reqs.append(Request(1000, 0, 0, 100, 2, 4, arrival=0.0))           # invalid n_out
    reqs.append(Request(1001, 0, 0, int(lengths[0]) + 5, 100, 4, arrival=0.0))  # outside the series
    done = {r.rid: r for r in sched.run_open_loop(reqs, timeout=120)}
    assert done[1000].error and done[1001].error
    for rid, r in done.items():
        if rid < 1000:
            assert r.error is None
            assert np.array_equal(r.result, _alone(pool, r))
    assert sched.ws_in_use == 0


@pytest.mark.parametrize("executor", [GpuExecutor, PlainGpuExecutor])
def test_device_memory_held_stays_within_the_budget(pool, executor):
    """The arena is the whole budget: serving a burst allocates no other
    device memory, whatever the batch sizes, and every step's memory returns."""
    x, y, offsets, lengths = pool
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    budget = 48 << 20
    ex = executor(y, offsets, lengths, x=x, n_slots=3, arena_bytes=budget)
    sched = Scheduler(ex, n_slots=3, max_batch=None if executor is GpuExecutor else 1)
    reqs = poisson_requests(1e9, 300, lengths, seed=21)
    done = sched.run_open_loop(reqs, timeout=120)
    torch.cuda.synchronize()
    assert len(done) == 300 and all(r.error is None for r in done)
    assert torch.cuda.max_memory_allocated() - base <= budget
    assert 0 < sched.max_ws_in_use <= budget
    assert ex.blocks.used == 0 and ex.blocks.free == [(0, budget)]
    for r in done[::15]:
        assert np.array_equal(r.result, _alone(pool, r)), f"request {r.rid}"
    if executor is GpuExecutor:
        assert max(sched.batch_sizes) > 1
