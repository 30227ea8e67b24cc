"""Pins of the oracle's other Table 1 downsamplers (CPU): MinMax with r_ps = 1
(section 3 footnote), M4 and EveryNth (section 2.2.1), against numpy per-part
argmin/argmax and an element-wise partition (not the oracle's formulas)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_00332_amd import synth
from tests import pins


def _series(seed, n):
    return synth.to_numpy([synth.random_walk, synth.ties_series, synth.subnormal_series,
                           synth.extreme_series][seed % 4](n, seed))


@pytest.mark.parametrize("seed", range(40))
def test_m4_matches_numpy(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 3000))
    n_out = int(rng.integers(4, 400))
    y = _series(seed, n)
    assert np.array_equal(oracle.m4(y, n_out), pins.m4_by_numpy(y, n_out))


@pytest.mark.parametrize("seed", range(40))
def test_minmax_r1_matches_numpy(seed):
    rng = np.random.default_rng(600 + seed)
    n = int(rng.integers(1, 3000))
    n_out = int(rng.integers(3, 400))
    y = _series(seed, n)
    assert np.array_equal(oracle.minmax(y, n_out, 1), pins.minmax_by_numpy(y, n_out, 1))


@pytest.mark.parametrize("n,n_out", [(1, 5), (5, 5), (6, 5), (10, 3), (1000, 7), (10 ** 7 + 3, 997),
                                     (2 ** 40 + 11, 4001)])
def test_everynth_is_part_starts(n, n_out):
    got = oracle.everynth(n, n_out)
    assert len(got) == min(n, n_out)
    if n <= 10 ** 6:
        assert np.array_equal(got, pins.everynth_by_parts(n, n_out))
    else:  # balanced: gaps take only floor(n/n_out) and ceil(n/n_out)
        gaps = set(np.diff(got).tolist()) | {n - int(got[-1])}
        assert gaps <= {n // n_out, -(-n // n_out)} and got[0] == 0


def test_m4_keeps_bin_edges_and_errors():
    y = synth.to_numpy(synth.random_walk(1000, 3))
    out = oracle.m4(y, 40)  # 10 bins of 100 points
    for b in range(10):
        assert 100 * b in out and 100 * b + 99 in out
    with pytest.raises(oracle.OracleError):
        oracle.m4(y, 3)
    with pytest.raises(oracle.OracleError):
        oracle.everynth(10, 0)
    with pytest.raises(oracle.OracleError):
        oracle.everynth(0, 10)


# ---------------------------------------------------------------- x-equal-width bins (R14)

def _gappy_x(n, seed):
    """Strictly increasing int64 x with exponential gaps and a few huge jumps."""
    rng = np.random.default_rng(seed)
    gaps = 1 + np.floor(rng.exponential(50.0, size=n)).astype(np.int64)
    jumps = rng.random(n) < 0.002
    gaps[jumps] += rng.integers(10 ** 6, 10 ** 9, size=int(jumps.sum()))
    return np.cumsum(gaps) - 7_000_000 + int(rng.integers(-10 ** 12, 10 ** 12))


@pytest.mark.parametrize("seed", range(30))
def test_xbins_with_unit_steps_is_index_binning(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 4000))
    n_out = int(rng.integers(3, 300))
    r_ps = int(rng.choice([1, 2, 4, 8]))
    y = _series(seed, n)
    x = np.arange(n, dtype=np.int64) + int(rng.integers(-10 ** 15, 10 ** 15))
    assert np.array_equal(oracle.minmax_xbins(y, x, n_out, r_ps), oracle.minmax(y, n_out, r_ps))
    if r_ps >= 2:
        assert np.array_equal(oracle.minmaxlttb_xbins(y, x, n_out, r_ps), oracle.minmaxlttb(y, n_out, r_ps, x))


@pytest.mark.parametrize("seed", range(40))
def test_xbins_matches_numpy_and_lttb_over_p(seed):
    rng = np.random.default_rng(800 + seed)
    n = int(rng.integers(3, 5000))
    n_out = int(rng.integers(3, 400))
    r_ps = int(rng.choice([2, 4, 8]))
    y = _series(seed, n)
    x = _gappy_x(n, seed) if seed % 3 else synth.to_numpy(synth.irregular_x(n, seed))
    want_p = pins.minmax_xbins_by_numpy(y, x, n_out, r_ps)
    assert np.array_equal(oracle.minmax_xbins(y, x, n_out, r_ps), want_p)
    got = oracle.minmaxlttb_xbins(y, x, n_out, r_ps)
    if n <= n_out:
        assert np.array_equal(got, np.arange(n))
    else:  # LTTB over the preselected points (itself pinned), or all of them
        assert np.array_equal(got, want_p[oracle.lttb(y[want_p], n_out, x[want_p])])


def test_xbins_sparse_preselection_keeps_every_point():
    # two clusters far apart: almost every bin is empty, P holds fewer than n_out points
    x = np.concatenate([np.arange(500), 10 ** 12 + np.arange(500)]).astype(np.int64)
    y = synth.to_numpy(synth.random_walk(1000, 5))
    P = oracle.minmax_xbins(y, x, 100, 4)
    assert len(P) < 100
    assert np.array_equal(oracle.minmaxlttb_xbins(y, x, 100, 4), P)


def test_xbins_errors():
    y = synth.to_numpy(synth.random_walk(100, 1))
    x = np.arange(100, dtype=np.int64)
    x[50] = x[49]
    with pytest.raises(oracle.OracleError):
        oracle.minmax_xbins(y, x, 10, 4)
    with pytest.raises(oracle.OracleError):
        oracle.minmaxlttb_xbins(y, np.arange(100), 10, 1)
