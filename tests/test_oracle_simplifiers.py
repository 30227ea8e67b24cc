"""Pins of the oracle's other simplifiers on the preselected points (readings
R16-R18; CPU): Visvalingam-Whyatt and Douglas-Peucker against exact-rational
implementations of their own on small-integer inputs (where every binary64
operation they need is exact or order-preserving), the nesting of their
greedy orders, closed forms, Douglas-Peucker at n_out = 3 equal to LTTB at
n_out = 3, Longest-Line-Bucket against all paths in 60-digit arithmetic, and
the MinMax composition."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2305_00332_amd import synth
from tests import pins


def _small_int_points(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(4, 60))
    X = np.cumsum(rng.integers(1, 9, size=m)).astype(np.float64)
    Y = rng.integers(-40, 41, size=m).astype(np.float64)
    if seed % 3 == 0:
        Y = np.round(Y / 8)  # many ties
    return X, Y


@pytest.mark.parametrize("seed", range(60))
def test_vw_and_dp_equal_exact_rational_versions(seed):
    X, Y = _small_int_points(seed)
    m = len(X)
    rng = np.random.default_rng(10_000 + seed)
    n_out = int(rng.integers(3, m))
    assert list(oracle.simplify_points("vw", X, Y, n_out)) == pins.vw_exact(X.tolist(), Y.tolist(), n_out)
    assert list(oracle.simplify_points("dp", X, Y, n_out)) == pins.dp_exact(X.tolist(), Y.tolist(), n_out)


@pytest.mark.parametrize("alg", ["vw", "dp"])
@pytest.mark.parametrize("seed", range(8))
def test_greedy_orders_nest(alg, seed):
    y = synth.to_numpy(synth.random_walk(600, seed)).astype(np.float64)
    X = np.arange(600, dtype=np.float64)
    prev = None
    for n_out in range(3, 120, 7):
        cur = set(oracle.simplify_points(alg, X, y, n_out).tolist())
        assert len(cur) == n_out and {0, 599} <= cur
        if prev is not None:
            assert prev <= cur
        prev = cur


@pytest.mark.parametrize("seed", range(10))
def test_dp_at_three_is_lttb_at_three(seed):
    y = synth.to_numpy(synth.random_walk(300 + seed, seed))
    x = synth.to_numpy(synth.irregular_x(300 + seed, seed))
    got = oracle.simplify_points("dp", x.astype(np.float64), y.astype(np.float64), 3)
    assert list(got) == list(oracle.lttb(y, 3, x))


def test_collinear_closed_forms():
    m, n_out = 50, 10
    X = np.arange(m, dtype=np.float64)
    Y = 3.0 * X - 7.0  # every area and distance is zero: lowest indices go first / stay last
    assert list(oracle.simplify_points("vw", X, Y, n_out)) == [0] + list(range(m - n_out + 1, m))
    assert list(oracle.simplify_points("dp", X, Y, n_out)) == list(range(n_out - 1)) + [m - 1]


@pytest.mark.parametrize("seed", range(40))
def test_llb_is_the_longest_path(seed):
    rng = np.random.default_rng(20_000 + seed)
    n_out = int(rng.integers(3, 6))
    m = n_out + int(rng.integers(1, 3 * (n_out - 2) + 1))
    X = np.cumsum(rng.random(m) + 0.1) * (10.0 ** rng.integers(-3, 4))
    Y = rng.standard_normal(m) * (10.0 ** rng.integers(-3, 4))
    if seed % 4 == 0:
        Y = np.round(Y)
    got = list(oracle.simplify_points("llb", X, Y, n_out))
    paths = pins.llb_brute(X, Y, n_out)
    best_len = paths[0][0]
    mine = next(t for t, p in paths if p == got)
    scale = sum(abs(float(v)) for v in X) + sum(abs(float(v)) for v in Y)
    assert float(best_len - mine) <= 1e-12 * scale  # optimal up to rounding
    # a clear winner (margin beyond rounding) must be the one chosen
    if len(paths) > 1 and float(paths[0][0] - paths[1][0]) > 1e-9 * scale:
        assert got == paths[0][1]


@pytest.mark.parametrize("alg", ["vw", "dp", "llb"])
@pytest.mark.parametrize("seed", range(6))
def test_minmax_composition(alg, seed):
    n = 2000 + 997 * seed
    y = synth.to_numpy(synth.random_walk(n, seed) if seed % 2 else synth.ties_series(n, seed))
    x = synth.to_numpy(synth.irregular_x(n, seed)) if seed % 3 else None
    n_out, r_ps = 50 + 13 * seed, [2, 4, 8][seed % 3]
    P = pins.minmax_by_numpy(y, n_out, r_ps)
    X = (P if x is None else x[P]).astype(np.float64)
    want = P[oracle.simplify_points(alg, X, y[P].astype(np.float64), n_out)]
    got = oracle.minmax_simplify(alg, y, n_out, r_ps, x)
    assert np.array_equal(got, want)
    pins.check_output_invariants(got, n, n_out)


def test_small_n_and_errors():
    y = synth.to_numpy(synth.random_walk(30, 1))
    for alg in ("vw", "dp", "llb"):
        assert np.array_equal(oracle.minmax_simplify(alg, y, 40, 4), np.arange(30))
        with pytest.raises(oracle.OracleError):
            oracle.minmax_simplify(alg, y, 2, 4)
        with pytest.raises(oracle.OracleError):
            oracle.minmax_simplify(alg, y, 10, 1)
