"""Step (a3), the next-bucket means, on its own: mmlttb_lttb_means against the
oracle's means, bit for bit (section 2.2.1 LTTB: the third vertex of a bucket's
triangle is the average point of the next bucket).

The one-thread-per-bucket kernel sums buckets of up to 16 points in binary64
when that is exact (X below 2^53, Y values within 2^(29 - bits(count)) of each
other in scale) and with the exact accumulators otherwise; the series below
put buckets on both sides of each of those limits, and the wide-bucket kernel
is covered by buckets of 40 and 200 points."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.int64)


def _span_series(m, seed, span):
    """Values 1.x * 2^-e with e uniform in [0, span], random signs: buckets mix
    scales up to 2^span apart."""
    rng = np.random.default_rng(seed)
    e = rng.integers(0, span + 1, m)
    v = (1.0 + rng.random(m)) * np.exp2(-e.astype(np.float64)) * rng.choice([-1.0, 1.0], m)
    return v.astype(np.float32)


def _series(kind, m, seed):
    if kind == "walk":
        return synth.to_numpy(synth.random_walk(m, seed))
    if kind == "ties":
        return synth.to_numpy(synth.ties_series(m, seed))
    if kind == "subnormal":
        return synth.to_numpy(synth.subnormal_series(m, seed))
    if kind == "extreme":
        return synth.to_numpy(synth.extreme_series(m, seed))
    if kind.startswith("span"):
        return _span_series(m, seed, int(kind[4:]))
    return np.full(m, -0.0 if seed % 2 else 3.5, dtype=np.float32)


def _x(kind, m, seed):
    if kind == "implicit":
        return None
    if kind == "irregular":
        return synth.to_numpy(synth.irregular_x(m, seed))
    return synth.to_numpy(synth.epoch_x(m, seed))  # sums of 2^53 or more: the exact path


KINDS = ["walk", "ties", "subnormal", "extreme", "constant", "span20", "span24", "span25", "span26", "span27",
         "span29", "span40"]
PER_BUCKET = [2, 4, 8, 15, 16, 17, 40, 200]


@pytest.mark.parametrize("per_bucket", PER_BUCKET)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("xkind", ["implicit", "irregular", "epoch"])
def test_means_equal_the_oracle_bit_for_bit(kind, per_bucket, xkind):
    seed = 1000 + PER_BUCKET.index(per_bucket) * 37 + KINDS.index(kind)
    n_out = 202
    m = 2 + (n_out - 2) * per_bucket + (seed % 7)  # a ragged last bucket
    y = _series(kind, m, seed)
    x = _x(xkind, m, seed)
    MX, MY = ops.lttb_means(torch.from_numpy(y).to(DEV), n_out,
                            x=None if x is None else torch.from_numpy(x).to(DEV))
    wx, wy = oracle.lttb_means(y, n_out, x)
    np.testing.assert_array_equal(_bits(MX.cpu().numpy()), _bits(wx))
    np.testing.assert_array_equal(_bits(MY.cpu().numpy()), _bits(wy))


def test_means_feed_the_same_picks():
    """MinMaxLTTB over series whose preselected buckets straddle the scale
    limit gives the oracle's picks (the means are the only input it shares)."""
    for seed, span in [(1, 24), (2, 26), (3, 28), (4, 60)]:
        y = _span_series(400_003, seed, span)
        for n_out, r_ps in [(1000, 4), (500, 8), (300, 16)]:
            got = ops.minmaxlttb(torch.from_numpy(y).to(DEV), n_out, r_ps).cpu().numpy()
            np.testing.assert_array_equal(got, oracle.minmaxlttb(y, n_out, r_ps))


def test_means_rejects_what_lttb_keeps_whole():
    y = torch.zeros(100, dtype=torch.float32, device=DEV)
    with pytest.raises(RuntimeError):
        ops.lttb_means(y, 100)
    with pytest.raises(RuntimeError):
        ops.lttb_means(y, 2)
