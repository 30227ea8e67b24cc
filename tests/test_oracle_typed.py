"""Pins of the oracle's other value types (reading R15; CPU): float64 and
int32 y, float64 x. The exact binary64 sum against math.fsum and closed
forms; MinMax against numpy per bin; MinMaxLTTB reducing to the (pinned)
float32 / int64 paths when the values coincide; general float64 inputs
against exact-rational areas within a rounding bound."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import synth
from tests import pins

DMAX = sys.float_info.max
DMIN_SUB = 5e-324


def _f64_values(seed, n):
    rng = np.random.default_rng(seed)
    kind = seed % 4
    if kind == 0:
        return rng.standard_normal(n) * 10.0 ** rng.integers(-300, 300, size=n)
    if kind == 1:
        return rng.standard_normal(n) * DMIN_SUB * 2 ** rng.integers(0, 60, size=n)  # subnormals
    if kind == 2:  # cancellation around a large value
        big = rng.standard_normal(n // 2 + 1) * 1e200
        return np.concatenate([big, -big, rng.standard_normal(n) * 1e-200])[: n + 2]
    return synth.to_numpy(synth.random_walk(n, seed, dtype=torch.float64))


@pytest.mark.parametrize("seed", range(40))
def test_exact_sum_f64_matches_fsum(seed):
    v = _f64_values(seed, 1 + seed * 37)
    assert oracle.exact_sum_f64(v) == math.fsum(v)


def test_exact_sum_f64_closed_forms():
    assert oracle.exact_sum_f64([DMAX, DMAX]) == math.inf
    assert oracle.exact_sum_f64([-DMAX, -DMAX]) == -math.inf
    assert oracle.exact_sum_f64([DMAX, DMAX, -DMAX]) == DMAX
    assert oracle.exact_sum_f64([DMIN_SUB, DMIN_SUB]) == 2 * DMIN_SUB
    assert oracle.exact_sum_f64([1.0, 2.0 ** -53]) == 1.0            # tie to even (down)
    assert oracle.exact_sum_f64([1.0 + 2.0 ** -52, 2.0 ** -53]) == 1.0 + 2.0 ** -51  # tie to even (up)
    assert oracle.exact_sum_f64([1.0, 2.0 ** -53, 2.0 ** -1074]) == 1.0 + 2.0 ** -52  # sticky
    assert oracle.exact_sum_f64([1e308, -1e308, 1e-308]) == 1e-308
    assert math.copysign(1.0, oracle.exact_sum_f64([-0.0, -0.0])) == 1.0  # an exact zero is +0
    assert oracle.exact_sum_f64([]) == 0.0


@pytest.mark.parametrize("seed", range(30))
def test_minmax_f64_and_i32_match_numpy(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 3000))
    n_out = int(rng.integers(3, 300))
    r_ps = int(rng.choice([1, 2, 4, 8]))
    y64 = _f64_values(seed, n)[:n] if seed % 2 else synth.to_numpy(synth.random_walk(n, seed, dtype=torch.float64))
    y64 = np.where(rng.random(n) < 0.05, -0.0, y64)  # signed zeros among the values
    assert np.array_equal(oracle.minmax_typed(y64, n_out, r_ps), pins.minmax_by_numpy(y64, n_out, r_ps))
    yi = synth.to_numpy(synth.int_series(n, seed, scale=1e3 if seed % 3 else 1e9))
    assert np.array_equal(oracle.minmax_typed(yi, n_out, r_ps), pins.minmax_by_numpy(yi, n_out, r_ps))


@pytest.mark.parametrize("seed", range(30))
def test_typed_reduces_to_float32_path(seed):
    rng = np.random.default_rng(1100 + seed)
    n = int(rng.integers(1, 4000))
    n_out = int(rng.integers(3, 300))
    r_ps = int(rng.choice([2, 4, 8]))
    y32 = synth.to_numpy(synth.random_walk(n, seed) if seed % 2 else synth.ties_series(n, seed))
    xi = synth.to_numpy(synth.irregular_x(n, seed)) if seed % 3 else None
    want = oracle.minmaxlttb(y32, n_out, r_ps, xi)
    assert np.array_equal(oracle.minmaxlttb_typed(y32, n_out, r_ps, xi), want)
    # the same numbers stored as binary64
    assert np.array_equal(oracle.minmaxlttb_typed(y32.astype(np.float64), n_out, r_ps, xi), want)
    # integer timestamps below 2^53 stored as binary64
    if xi is not None:
        assert np.array_equal(oracle.minmaxlttb_typed(y32, n_out, r_ps, xi.astype(np.float64)), want)
    # int32 values exact in float32
    yi = np.round(y32 * 1000).astype(np.int32)
    assert np.array_equal(oracle.minmaxlttb_typed(yi, n_out, r_ps, xi),
                          oracle.minmaxlttb(yi.astype(np.float32), n_out, r_ps, xi))


@pytest.mark.parametrize("seed", range(20))
def test_typed_lttb_near_optimal_general_inputs(seed):
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(10, 600))
    n_out = int(rng.integers(3, max(4, n // 3)))
    r_ps = int(rng.choice([2, 4, 8]))
    y = synth.to_numpy(synth.random_walk(n, seed, dtype=torch.float64)) * (1.0 + 1e-9 * seed)
    x = synth.to_numpy(synth.float_x(n, seed)) if seed % 2 else None
    out = oracle.minmaxlttb_typed(y, n_out, r_ps, x)
    P = oracle.minmax_typed(y, n_out, r_ps)
    pos = np.searchsorted(P, out)
    assert np.array_equal(P[pos], out)  # the output lies in P
    xs = P.astype(np.float64) if x is None else x[P]
    pins.check_lttb_near_optimal(list(xs) if x is not None else [int(v) for v in P], list(y[P]), list(pos), n_out)


def test_typed_errors():
    y = np.arange(10, dtype=np.float64)
    with pytest.raises(TypeError):
        oracle.minmax_typed(np.arange(10, dtype=np.int16), 5, 2)
    y_bad = y.copy()
    y_bad[3] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.minmaxlttb_typed(y_bad, 3, 2)
    x_bad = np.arange(10, dtype=np.float64)
    x_bad[4] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.minmaxlttb_typed(y, 3, 2, x_bad)
    with pytest.raises(oracle.OracleError):
        oracle.minmaxlttb_typed(y, 3, 1)


@pytest.mark.parametrize("seed", range(16))
def test_typed_means_match_fsum(seed):
    rng = np.random.default_rng(1500 + seed)
    m = int(rng.integers(10, 900))
    n_out = int(rng.integers(3, m))
    ph = np.arange(m) % 3  # +1e17, a small value a running binary64 sum would lose, -1e17
    y = _f64_values(seed, m)[:m] if seed % 2 else np.where(ph == 0, 1e17, np.where(ph == 2, -1e17,
                                                                                    rng.standard_normal(m)))
    x = np.cumsum(rng.random(m) + 0.5) + 1e15 if seed % 3 else None
    MX, MY = oracle.lttb_means_typed(y, n_out, x)
    assert np.array_equal(MY, pins.means_by_fsum(y, n_out))
    assert np.array_equal(MX, pins.means_by_fsum(np.arange(m) if x is None else x, n_out))
    yi = synth.to_numpy(synth.int_series(m, seed, scale=1e9))
    _, MYi = oracle.lttb_means_typed(yi, n_out)
    assert np.array_equal(MYi, pins.means_by_fsum(yi.astype(np.float64), n_out))
