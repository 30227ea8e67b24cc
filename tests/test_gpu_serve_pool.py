"""Serving against the full serving pool (512 series, lengths log-uniform in
[1e4, 1e8], ~5.4e9 points: float32 random walk + sinusoids + noise, int64
irregular x, ~65 GB resident): a burst of 400 requests served by continuous
batching, every result compared with the oracle on that sub-range alone
(tolerance 0), including sub-ranges of more than 1e7 points served inside
batched steps."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import synth
from paper_2305_00332_amd.serve import GpuExecutor, Scheduler, poisson_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serving_pool():
    lengths = synth.batch_lengths(512, 1e4, 1e8, 5)
    print(f"generating the serving pool: {int(lengths.sum())} points", flush=True)
    x, y, offsets = synth.batch_series(lengths, 5, device="cuda", sinusoids=True)
    torch.cuda.synchronize()
    yield x, y, offsets, lengths
    del x, y
    torch.cuda.empty_cache()


def test_burst_on_the_serving_pool_equals_the_oracle(serving_pool):
    x, y, offsets, lengths = serving_pool
    ex = GpuExecutor(y, offsets, lengths, x=x, n_slots=3, arena_bytes=1 << 30)
    sched = Scheduler(ex, n_slots=3, max_batch=128)
    reqs = poisson_requests(1e12, 400, lengths, seed=77)
    done = sched.run_open_loop(reqs, timeout=300)
    assert len(done) == 400 and all(r.error is None for r in done), [r.error for r in done if r.error][:3]
    long_batched = [r for r in done if r.n > 10 ** 7 and r.batch > 1]
    print(f"{len(sched.batch_sizes)} steps, batch sizes {sched.batch_sizes}; "
          f"{len(long_batched)} sub-ranges above 1e7 points in batched steps", flush=True)
    assert len(long_batched) >= 10
    assert max(sched.batch_sizes) > 1
    segs = [(int(offsets[r.series]) + r.lo, r.n, r.n_out, r.r_ps) for r in done]

    def fetch(lo, hi):
        return y[lo:hi].cpu().numpy(), x[lo:hi].cpu().numpy()

    print("comparing every request with the oracle", flush=True)
    want = oracle.minmaxlttb_segments(fetch, segs, workers=16)
    bad = [r.rid for r, w in zip(done, want) if not np.array_equal(r.result, w)]
    assert not bad, f"{len(bad)} requests differ from the oracle, first {bad[:5]}"
