"""Full-size workloads, GPU == oracle on every output index (tolerance 0).

- one series of 1e6 points (random walk, implicit x), n_out=1000, r_ps=4,
  MinMaxLTTB and whole-series LTTB;
- one series of 1e8 points (random walk + 3 sinusoids + noise + spikes,
  int64 irregular timestamps), n_out=2000, r_ps in {2, 4, 8}, plus
  whole-series LTTB;
- one series of 1e9 points (random walk, implicit x, 4 GB), n_out in
  {1000, 4000}, r_ps=4 -- the launch configuration the benchmark times.
Inputs are generated on the GPU from fixed seeds and copied to the host for
the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(params=[ops.CHAIN_SEQUENTIAL, ops.CHAIN_SEGMENTED], ids=["seqchain", "segchain"])
def chain_mode(request):
    old = ops.get_tuning()
    ops.set_tuning(0, 0, request.param)
    yield request.param
    ops.set_tuning(*old)


def test_one_million_points(chain_mode):
    y = synth.random_walk(1_000_000, 1, device="cuda")
    y_np = y.cpu().numpy()
    got = ops.minmaxlttb(y, 1000, 4).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, 1000, 4))
    P, m = ops.minmax(y, 1000, 4)
    np.testing.assert_array_equal(P.cpu().numpy(), oracle.minmax(y_np, 1000, 4))
    assert m == 4002
    got_l = ops.lttb(y, 1000).cpu().numpy()
    np.testing.assert_array_equal(got_l, oracle.lttb(y_np, 1000))


def test_hundred_million_points_irregular_x(chain_mode):
    _say("generating 1e8 composite series on the GPU")
    x, y = synth.composite_series(100_000_000, 2, device="cuda")
    y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
    for r_ps in (2, 4, 8):
        _say(f"minmaxlttb n=1e8 n_out=2000 r_ps={r_ps}")
        got = ops.minmaxlttb(y, 2000, r_ps, x=x).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, 2000, r_ps, x_np))
    _say("lttb n=1e8 n_out=2000")
    got_l = ops.lttb(y, 2000, x=x).cpu().numpy()
    np.testing.assert_array_equal(got_l, oracle.lttb(y_np, 2000, x_np))


def test_one_billion_points(chain_mode):
    _say("generating 1e9 random walk on the GPU")
    y = synth.random_walk(1_000_000_000, 3, device="cuda")
    torch.cuda.synchronize()
    y_np = y.cpu().numpy()
    for n_out in (1000, 4000):
        _say(f"minmaxlttb n=1e9 n_out={n_out} r_ps=4")
        got = ops.minmaxlttb(y, n_out, 4).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, n_out, 4))
    P, m = ops.minmax(y, 4000, 4)
    np.testing.assert_array_equal(P.cpu().numpy(), oracle.minmax(y_np, 4000, 4))
    del y
    torch.cuda.empty_cache()


def test_large_output_sizes(chain_mode):
    """n_out of 2^20 and 3*10^5 on 5e7 points: 2M and 1.2M bins, a compaction
    of several rounds in its one workgroup, chains of 32768 segments; whole-
    series LTTB with 1e6 buckets of ~50 points."""
    _say("generating 5e7 composite series on the GPU")
    x, y = synth.composite_series(50_000_000, 9, device="cuda")
    y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
    for n_out, r_ps in [(1 << 20, 4), (300_000, 8)]:
        _say(f"minmaxlttb n=5e7 n_out={n_out} r_ps={r_ps}")
        got = ops.minmaxlttb(y, n_out, r_ps, x=x).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, n_out, r_ps, x_np))
    _say("lttb n=5e7 n_out=1e6")
    got_l = ops.lttb(y, 1_000_000, x=x).cpu().numpy()
    np.testing.assert_array_equal(got_l, oracle.lttb(y_np, 1_000_000, x_np))


def test_short_bins_of_a_long_series():
    """A series of 2e8 points with bins of fewer than 4096 points is streamed
    rather than one work item per bin: bins of at most a quarter tile (763
    points) in tiles of whole bins, longer ones (3051) in fixed chunks of
    65536 points across bin ends (wave_stream_bins)."""
    _say("generating 2e8 random walk on the GPU")
    y = synth.random_walk(200_000_000, 17, device="cuda")
    torch.cuda.synchronize()
    y_np = y.cpu().numpy()
    for n_out, r_ps in [(131072, 4), (65536, 2)]:
        _say(f"minmaxlttb n=2e8 n_out={n_out} r_ps={r_ps}")
        got = ops.minmaxlttb(y, n_out, r_ps).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, n_out, r_ps))
        P, m = ops.minmax(y, n_out, r_ps)
        np.testing.assert_array_equal(P[: int(m)].cpu().numpy(), oracle.minmax(y_np, n_out, r_ps))
    del y


@pytest.mark.parametrize("tile", [2048, 4096, 8192])
def test_short_bin_tiles_around_their_limit(tile):
    """Bins of at most tile / 4 points in a 2e8-point series go to tiles of
    whole bins (the batched small-bin body on one series); one point more goes
    to the chunked stream. For each tile size: bins of exactly tile / 4 and
    tile / 4 + 1 points through MinMaxLTTB, and bins of at most 16 points (256
    bins a tile) through MinMax."""
    y = _walk_2e8()
    y_np = _walk_2e8_np()
    old = ops.get_tuning()
    ops.set_tuning(0, 0, 0, tile)
    try:
        interior = 200_000_000 - 2
        for maxbin in (tile // 4, tile // 4 + 1):
            nb = -(-interior // (maxbin - 1)) - 1  # the fewest bins whose longest has maxbin points
            while -(-interior // nb) > maxbin:
                nb += 1
            assert -(-interior // nb) == maxbin
            _say(f"tile={tile} minmaxlttb n=2e8 bins of at most {maxbin} points (nb={nb}, r_ps=2)")
            got = ops.minmaxlttb(y, nb, 2).cpu().numpy()
            np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, nb, 2))
        nb = -(-interior // 16)
        _say(f"tile={tile} minmax n=2e8 bins of at most 16 points (nb={nb})")
        P, m = ops.minmax(y, nb, 2)
        np.testing.assert_array_equal(P[: int(m)].cpu().numpy(), oracle.minmax(y_np, nb, 2))
    finally:
        ops.set_tuning(*old)


_WALK = {}


def _walk_2e8():
    if "y" not in _WALK:
        _say("generating 2e8 random walk on the GPU")
        _WALK["y"] = synth.random_walk(200_000_000, 23, device="cuda")
        torch.cuda.synchronize()
    return _WALK["y"]


def _walk_2e8_np():
    if "np" not in _WALK:
        _WALK["np"] = _walk_2e8().cpu().numpy()
    return _WALK["np"]
