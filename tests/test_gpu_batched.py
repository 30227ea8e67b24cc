"""Batched MinMaxLTTB: every series' result equals the oracle on that series
alone and the single-series GPU call (tolerance 0), for batches mixing
identity series (n <= n_out), fully preselected series, small-bin and
large-bin series, sequential-chain fallbacks, implicit and int64 x and
misaligned starts; plus the full-size batch of 4096 series."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import _lib, ops, synth

pytestmark = pytest.mark.gpu


def _random_batch(seed, count, nmax):
    rng = np.random.default_rng(seed)
    lengths = np.floor(np.exp(rng.uniform(0, np.log(nmax), size=count))).astype(np.int64) + 1
    n_outs = rng.choice([3, 4, 10, 50, 200, 500, 1000, 2000], size=count)
    r_pss = rng.choice([2, 2, 3, 4, 4, 8, 100], size=count)
    return lengths, n_outs, r_pss


def _check_batch(x, y, offsets, lengths, n_outs, r_pss, sample=None):
    segs = [(int(o), int(n), int(no), int(r)) for o, n, no, r in zip(offsets, lengths, n_outs, r_pss)]
    out, outoff = ops.minmaxlttb_batched(y, segs, x_base=x)
    got = out.cpu().numpy()
    idx = range(len(segs)) if sample is None else sample
    for i in idx:
        o, n, no, r = segs[i]
        k = min(n, no)
        g = got[outoff[i]: outoff[i] + k]
        ys = y[o: o + n].cpu().numpy()
        xs = None if x is None else x[o: o + n].cpu().numpy()
        want = oracle.minmaxlttb(ys, no, r, xs)
        assert np.array_equal(g, want), f"series {i}: n={n} n_out={no} r_ps={r}"
        single = ops.minmaxlttb(y[o: o + n].contiguous() if (o % 4) == 0 else y[o: o + n], no, r,
                                x=None if x is None else x[o: o + n]).cpu().numpy()
        assert np.array_equal(g, single), f"series {i} differs from the single-series call"
    return got, outoff


@pytest.fixture(params=[ops.CHAIN_AUTO, ops.CHAIN_SEQUENTIAL], ids=["autochain", "seqchain"])
def chain_mode(request):
    old = ops.get_tuning()
    ops.set_tuning(0, 0, request.param)
    yield request.param
    ops.set_tuning(*old)


@pytest.mark.parametrize("seed", range(6))
def test_random_batches(seed, chain_mode):
    lengths, n_outs, r_pss = _random_batch(seed, 60, 300_000)
    x, y, offsets = synth.batch_series(lengths, seed, device="cuda", with_x=bool(seed % 2))
    _check_batch(x, y, offsets, lengths, n_outs, r_pss)


def test_misaligned_and_gapped_offsets():
    rng = np.random.default_rng(7)
    lengths = rng.integers(1, 50_000, size=40)
    gaps = rng.integers(0, 7, size=40)
    offsets = np.cumsum(np.concatenate([[3], (lengths + gaps)[:-1]]))
    total = int(offsets[-1] + lengths[-1] + 5)
    y = synth.random_walk(total, 7, device="cuda")
    x = synth.irregular_x(total, 8, device="cuda")
    n_outs = rng.choice([3, 100, 1000], size=40)
    r_pss = rng.choice([2, 4, 6], size=40)
    _check_batch(x, y, offsets, lengths, n_outs, r_pss)
    _check_batch(None, y, offsets, lengths, n_outs, r_pss)


def test_batch_of_one_and_repeat_identical():
    y = synth.random_walk(1_000_003, 9, device="cuda")
    out1, _ = ops.minmaxlttb_batched(y, [(0, 1_000_003, 1000, 4)])
    single = ops.minmaxlttb(y, 1000, 4)
    assert torch.equal(out1[:1000], single)
    ws = torch.empty(ops.batched_workspace_size([(0, 1_000_003, 1000, 4)]), dtype=torch.uint8, device="cuda")
    out2, _ = ops.minmaxlttb_batched(y, [(0, 1_000_003, 1000, 4)], ws=ws)
    out3, _ = ops.minmaxlttb_batched(y, [(0, 1_000_003, 1000, 4)], ws=ws)
    assert torch.equal(out2, out1) and torch.equal(out3, out1)


def test_invalid_segment_rejected_before_any_work():
    y = synth.random_walk(1000, 1, device="cuda")
    out = torch.full((20,), -7, dtype=torch.int64, device="cuda")
    for bad in [(0, 0, 10, 4), (0, 100, 2, 4), (0, 100, 10, 1), (-1, 100, 10, 4)]:
        with pytest.raises(_lib.MmlttbError) as e:
            ops.minmaxlttb_batched(y, [(0, 500, 10, 4), bad], out=out)
        assert e.value.code == _lib.EINVAL
    assert torch.all(out == -7)  # nothing was enqueued


def test_workspace_size_independent_of_lengths():
    a = ops.batched_workspace_size([(0, 10, 100, 4), (10, 10, 200, 2)])
    b = ops.batched_workspace_size([(0, 10 ** 9, 100, 4), (10 ** 9, 10 ** 7, 200, 2)])
    assert a == b > 0


def test_full_batch_4096_series():
    """4096 series, lengths log-uniform in [1e3, 1e7] (~4.6e9 points), int64
    irregular x, n_out in {200, 500, 1000, 2000}, r_ps = 4. Every series is
    compared with the oracle on that series alone and with the single-series
    GPU call."""
    lengths = synth.batch_lengths(4096, 1e3, 1e7, 4)
    n_outs = synth.choice([200, 500, 1000, 2000], 4096, 40)
    print(f"generating {int(lengths.sum())} points", flush=True)
    x, y, offsets = synth.batch_series(lengths, 4, device="cuda")
    torch.cuda.synchronize()
    segs = [(int(o), int(n), int(no), 4) for o, n, no in zip(offsets, lengths, n_outs)]
    out, outoff = ops.minmaxlttb_batched(y, segs, x_base=x)
    got = out.cpu().numpy()
    print("batched call done; comparing every series with the oracle", flush=True)

    def fetch(lo, hi):
        return y[lo:hi].cpu().numpy(), x[lo:hi].cpu().numpy()

    want = oracle.minmaxlttb_segments(fetch, segs, workers=16)
    bad = [i for i, (o, n, no, r) in enumerate(segs)
           if not np.array_equal(got[outoff[i]: outoff[i] + min(n, no)], want[i])]
    assert not bad, f"{len(bad)} series differ from the oracle, first {bad[:5]}"
    print("comparing with single-series calls", flush=True)
    for i, (o, n, no, r) in enumerate(segs):
        single = ops.minmaxlttb(y[o: o + n], no, r, x=x[o: o + n]).cpu().numpy()
        assert np.array_equal(got[outoff[i]: outoff[i] + min(n, no)], single), f"series {i}"
    del x, y
    torch.cuda.empty_cache()
