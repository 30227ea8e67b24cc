"""GPU == oracle for MinMax preselection followed by Visvalingam-Whyatt,
Douglas-Peucker or Longest-Line-Bucket (mmlttb_minmax_simplify), element by
element: random shapes and value families with implicit, int64 and epoch x,
edges around n_out, preselections small enough for LDS and large enough for
the workspace, both x kinds at 1e7 points, argument errors."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
ALGS = ["vw", "dp", "llb"]


def _series(kind, n, seed):
    if kind == "walk":
        return synth.to_numpy(synth.random_walk(n, seed))
    if kind == "ties":
        return synth.to_numpy(synth.ties_series(n, seed))
    if kind == "extreme":
        return synth.to_numpy(synth.extreme_series(n, seed))
    return np.full(n, 2.5, dtype=np.float32)


def _x(seed, n):
    k = seed % 3
    if k == 0:
        return None
    if k == 1:
        return synth.to_numpy(synth.irregular_x(n, seed))
    return synth.to_numpy(synth.epoch_x(n, seed))


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cases(count, seed0, nmax):
    rng = np.random.default_rng(seed0)
    kinds = ["walk", "ties", "extreme", "const"]
    out = []
    for c in range(count):
        n = max(1, int(np.exp(rng.uniform(0, np.log(nmax)))))
        n_out = int(rng.integers(3, max(4, min(n + 3, 1500))))
        r_ps = int(rng.choice([2, 4, 4, 8]))
        out.append((seed0 + c, kinds[c % 4], n, n_out, r_ps))
    return out


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("case", _cases(40, 90_000, 200_000), ids=lambda c: f"s{c[0]}-{c[1]}-n{c[2]}-o{c[3]}-r{c[4]}")
def test_simplifiers_random(alg, case):
    seed, kind, n, n_out, r_ps = case
    y, x = _series(kind, n, seed), _x(seed, n)
    got = ops.minmax_simplify(alg, _dev(y), n_out, r_ps, x=_dev(x)).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmax_simplify(alg, y, n_out, r_ps, x))


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("n,n_out,r_ps", [(1, 3, 2), (3, 3, 2), (4, 3, 2), (5, 3, 2), (66, 3, 100), (130, 64, 2),
                                          (1000, 999, 2), (4099, 1000, 2), (50_000, 1000, 4),
                                          (200_000, 2500, 4), (300_000, 4000, 4)])
def test_simplifiers_edges_and_storage(alg, n, n_out, r_ps):
    # up to ~5000 preselected points the state sits in LDS; 10002 and 16002 use the workspace
    y = _series("walk" if n % 2 else "ties", n, n + n_out)
    got = ops.minmax_simplify(alg, _dev(y), n_out, r_ps).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmax_simplify(alg, y, n_out, r_ps))


def test_ten_million_points():
    print("simplifiers on 1e7 points", file=sys.stderr, flush=True)
    x, y = synth.composite_series(10_000_000, 5, device=DEV)
    y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
    for alg in ALGS:
        got = ops.minmax_simplify(alg, y, 1000, 4, x=x).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmax_simplify(alg, y_np, 1000, 4, x_np))
        got = ops.minmax_simplify(alg, y, 2000, 4).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmax_simplify(alg, y_np, 2000, 4))


def test_simplifier_errors():
    y = _dev(_series("walk", 1000, 1))
    with pytest.raises(RuntimeError, match="alg"):
        ops.minmax_simplify(7, y, 100, 4)
    with pytest.raises(RuntimeError, match="r_ps"):
        ops.minmax_simplify("vw", y, 100, 1)
    with pytest.raises(RuntimeError, match="workspace"):
        ops.minmax_simplify("dp", y, 100, 4, ws=torch.empty(8, dtype=torch.uint8, device=DEV))
    np.testing.assert_array_equal(ops.minmax_simplify("llb", y, 100, 4).cpu().numpy(),
                                  oracle.minmax_simplify("llb", y.cpu().numpy(), 100, 4))


# Douglas-Peucker runs as a split tree built a level at a time, ranked by path
# bottlenecks, with a best-first walk inside the cluster that holds step
# n_out - 2; trees deeper than 512 levels and walks of more than 256 steps or
# over more than 512 nodes go to the greedy loop. Each case below takes one of
# those routes (noted beside it). "noise0" is uniform noise whose first and
# last values are 0: the whole series' chord is then flat and most of the
# tree ranks with its root, in a cluster of ~900 nodes at 3000 points; with
# n <= n_out * r_ps / 2 + 2 every point is preselected.
def _dp_series(kind, n, seed):
    if kind == "noise0":
        y = np.random.default_rng(seed).uniform(-1, 1, n).astype(np.float32)
        y[0] = y[-1] = 0
        return y
    if kind == "zigzag":
        return (np.where(np.arange(n) % 2 == 0, 1.0, -1.0) + np.arange(n) * 1e-5).astype(np.float32)
    if kind == "saw":
        return (np.arange(n) % 1000).astype(np.float32)
    return _series(kind, n, seed)


DP_ROUTES = [
    ("walk", 200_000, 1000, 4),      # one step in a cluster of two nodes
    ("noise0", 1500, 200, 16),       # 198 steps inside the root's cluster of 436 nodes
    ("zigzag", 200_000, 100, 4),     # 10 steps in a cluster of 14
    ("zigzag", 200_000, 1000, 4),    # 4 steps, a 205-level tree
    ("saw", 200_000, 20, 4),         # the boundary cluster taken whole (16 nodes)
    ("const", 200_000, 100, 4),      # a chain n_out - 2 levels deep: every node kept
    ("ties", 200_000, 100, 4),       # 3 steps in a cluster of 14, a 98-level tree
    ("ties", 200_000, 600, 2),       # deeper than 512 levels: the greedy loop
    ("const", 200_000, 1000, 4),     # a chain deeper than 512 levels: the greedy loop
    ("noise0", 3000, 375, 16),       # 373 steps inside the root's cluster: the greedy loop
    ("noise0", 3000, 250, 24),       # 248 steps in a cluster of ~900 nodes: the greedy loop
    ("walk", 200_000, 1015, 4),      # 4062 points: the largest preselection whose tree state fits LDS
    ("walk", 200_000, 1016, 4),      # 4066 points: the smallest whose tree state goes to the workspace
    ("zigzag", 200_000, 1300, 8),    # 10402 points: the tree's arrays in the workspace; 4 steps
    ("noise0", 6000, 1500, 8),       # the workspace, then 1498 steps in the root's cluster: the greedy loop
]


@pytest.mark.parametrize("kind,n,n_out,r_ps", DP_ROUTES, ids=lambda v: str(v))
def test_dp_split_tree_routes(kind, n, n_out, r_ps):
    y = _dp_series(kind, n, n + n_out)
    got = ops.minmax_simplify("dp", _dev(y), n_out, r_ps).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmax_simplify("dp", y, n_out, r_ps))


# Longest-Line-Bucket takes one lane per pair of points of consecutive
# buckets when buckets hold at most 8 points (ceil(2 floor(n_out r_ps / 2) /
# (n_out - 2)) <= 8: r_ps up to 7 for n_out >= 16), else one lane per point.
@pytest.mark.parametrize("r_ps", [2, 3, 6, 7, 8])
@pytest.mark.parametrize("n_out", [3, 4, 50, 1000])
@pytest.mark.parametrize("kind", ["walk", "ties"])
def test_llb_around_the_pair_limit(kind, n_out, r_ps):
    y = _series(kind, 100_000, 7 * n_out + r_ps)
    got = ops.minmax_simplify("llb", _dev(y), n_out, r_ps).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmax_simplify("llb", y, n_out, r_ps))
