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
