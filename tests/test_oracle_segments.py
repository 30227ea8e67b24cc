"""oracle.minmaxlttb_segments (many segments of one series pair, in slabs and
on a thread pool) returns exactly minmaxlttb of each segment alone."""
from __future__ import annotations

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("workers,slab", [(1, 1 << 40), (4, 5000), (8, 0), (3, 300_000)])
def test_segments_equal_one_call_each(workers, slab):
    rng = np.random.default_rng(workers * 7 + 1)
    N = 400_000
    y = np.cumsum(rng.standard_normal(N)).astype(np.float32)
    x = np.cumsum(1 + rng.integers(0, 2000, N)).astype(np.int64)
    segs = []
    for _ in range(120):
        n = int(rng.integers(1, 60_000))
        o = int(rng.integers(0, N - n + 1))
        segs.append((o, n, int(rng.integers(3, 700)), int(rng.choice([2, 4, 7]))))
    segs.append(segs[5])  # the same segment twice
    fetched = []

    def fetch(lo, hi):
        fetched.append((lo, hi))
        return y[lo:hi], x[lo:hi]

    got = oracle.minmaxlttb_segments(fetch, segs, workers=workers, slab_points=slab)
    for (o, n, no, r), g in zip(segs, got):
        assert np.array_equal(g, oracle.minmaxlttb(y[o:o + n], no, r, x[o:o + n]))
    assert all(0 <= lo < hi <= N for lo, hi in fetched)


def test_implicit_x_segments():
    y = np.cumsum(np.random.default_rng(3).standard_normal(50_000)).astype(np.float32)
    segs = [(0, 50_000, 100, 4), (10, 2, 3, 2), (1000, 20_000, 500, 2)]
    got = oracle.minmaxlttb_segments(lambda lo, hi: (y[lo:hi], None), segs, workers=2)
    for (o, n, no, r), g in zip(segs, got):
        assert np.array_equal(g, oracle.minmaxlttb(y[o:o + n], no, r))
