"""CPU model of Douglas-Peucker with a point budget as a ranked split tree,
checked against the oracle's greedy loop (reading R17).

The GPU kernel does not run the greedy loop step by step. It builds the tree
of every split the recursion would make, ranks each node by its bottleneck
(the node of lowest priority, priority = (key, lower index first), on its
path from the root), keeps every cluster of nodes sharing a bottleneck that
ranks above the cluster holding step n_out - 2, and walks only that cluster
best-first. This module restates that construction in plain Python, with no
code shared with the oracle or the kernel, and checks it against the oracle
on random, tied, constant, zigzag and noise series, so the ordering argument
the kernel relies on is pinned on the CPU. It also mirrors the kernel's route
choice (tree depth and boundary-walk limits) for the inputs the GPU route
tests use."""
from __future__ import annotations

import functools

import numpy as np
import pytest

import oracle


def _above(key, u, v):
    """pi(u) > pi(v): a larger key, or the same key and a lower index."""
    return key[u] > key[v] or (key[u] == key[v] and u < v)


def split_tree(X, Y, max_depth):
    """Nodes of the split tree down to depth max_depth - 1: key, parent,
    bottleneck; and whether some segment below that depth could still split."""
    m = len(X)
    key, par, bot = {}, {}, {}
    segs = [(0, m - 1, -1)]
    depth = 0
    while segs and depth < max_depth:
        new = []
        for a, b, p in segs:
            if b - a < 2:
                continue
            dx, dy = X[b] - X[a], Y[b] - Y[a]
            best, j = -1.0, -1
            for i in range(a + 1, b):
                c = abs(dx * (Y[i] - Y[a]) - (X[i] - X[a]) * dy)
                if c > best:  # lowest index on ties; a NaN distance never wins
                    best, j = c, i
            if j < 0:
                continue
            with np.errstate(all="ignore"):
                k = float(np.float64(best) * best / (np.float64(dx) * dx + np.float64(dy) * dy))
            key[j] = -1.0 if k != k else k
            par[j] = p
            bot[j] = j if p < 0 or _above(key, bot[p], j) else bot[p]
            new += [(a, j, j), (j, b, j)]
        segs = new
        depth += 1
    deeper = any(b - a >= 2 for a, b, _ in segs)
    return key, par, bot, deeper


def dp_by_clusters(X, Y, n_out):
    """The kept indices (first and last included), and the boundary walk's
    (steps, cluster size)."""
    K = n_out - 2
    key, par, bot, _ = split_tree(X, Y, K)
    nodes = list(key)
    kept = set(nodes)
    steps = size = 0
    if len(nodes) > K:
        rank = functools.cmp_to_key(lambda v, w: 0 if bot[v] == bot[w] else (-1 if _above(key, bot[v], bot[w]) else 1))
        order = sorted(nodes, key=rank)
        head = bot[order[K - 1]]
        kept = {v for v in nodes if bot[v] != head and _above(key, bot[v], head)}
        cluster = [v for v in nodes if bot[v] == head]
        size = len(cluster)
        steps = K - len(kept)
        frontier = [head]
        for _ in range(steps):  # best-first inside the boundary cluster
            v = max(frontier, key=functools.cmp_to_key(lambda u, w: 0 if u == w else (1 if _above(key, u, w) else -1)))
            frontier.remove(v)
            kept.add(v)
            frontier += [c for c in cluster if par[c] == v]
    return np.array(sorted(kept | {0, len(X) - 1})), steps, size


def _series(kind, m, rng):
    X = np.sort(rng.integers(0, 10 * m, m)).astype(np.float64)
    if kind == "walk":
        Y = np.cumsum(rng.standard_normal(m))
    elif kind == "ties":
        Y = rng.integers(0, 3, m).astype(np.float64)
        X = np.arange(m, dtype=np.float64)
    elif kind == "sine":
        Y = np.sin(np.arange(m) * 0.3) + 0.01 * rng.standard_normal(m)
    elif kind == "const":
        Y = np.full(m, 2.0)
    elif kind == "zigzag":
        Y = np.where(np.arange(m) % 2 == 0, 1.0, -1.0) + np.arange(m) * 0.01
    else:  # noise0: uniform noise, first and last 0 (a large root cluster)
        Y = rng.uniform(-1, 1, m)
        Y[0] = Y[-1] = 0.0
    return X, Y.astype(np.float32).astype(np.float64)


KINDS = ["walk", "ties", "sine", "const", "zigzag", "noise0"]


@pytest.mark.parametrize("kind", KINDS)
def test_cluster_ranking_equals_the_greedy_loop(kind):
    rng = np.random.default_rng(2305 + KINDS.index(kind))
    walked = 0
    for _ in range(25):
        m = int(rng.integers(5, 260))
        n_out = int(rng.integers(3, m))
        X, Y = _series(kind, m, rng)
        got, steps, _ = dp_by_clusters(X, Y, n_out)
        np.testing.assert_array_equal(got, oracle.simplify_points("dp", X, Y, n_out))
        walked += steps > 1
    if kind in ("ties", "zigzag", "noise0"):
        assert walked > 0  # some cases end inside a cluster after more than one step


def test_a_planted_wrong_order_inside_the_cluster_is_caught():
    """Walking the boundary cluster by index instead of best-first must differ
    from the greedy loop on some input (the walk is not a formality)."""
    rng = np.random.default_rng(11)
    differs = False
    for _ in range(60):
        m = int(rng.integers(20, 200))
        n_out = int(rng.integers(3, m // 2))
        X, Y = _series("noise0", m, rng)
        K = n_out - 2
        key, par, bot, _ = split_tree(X, Y, K)
        nodes = list(key)
        if len(nodes) <= K:
            continue
        rank = functools.cmp_to_key(lambda v, w: 0 if bot[v] == bot[w] else (-1 if _above(key, bot[v], bot[w]) else 1))
        order = sorted(nodes, key=rank)
        head = bot[order[K - 1]]
        kept = {v for v in nodes if bot[v] != head and _above(key, bot[v], head)}
        cluster = sorted(v for v in nodes if bot[v] == head)
        kept |= set(cluster[: K - len(kept)])  # by index: wrong
        wrong = np.array(sorted(kept | {0, m - 1}))
        if not np.array_equal(wrong, oracle.simplify_points("dp", X, Y, n_out)):
            differs = True
            break
    assert differs


# The kernel's limits: tree levels built before handing over, and the
# boundary walk's steps and nodes.
MAX_LEVELS, MAX_STEPS, MAX_CLUSTER = 512, 256, 512


def kernel_route(X, Y, n_out):
    """The route the split-tree kernel takes: "walk" (best-first inside the
    boundary cluster), "whole" (the boundary cluster kept whole), "all"
    (every node kept), "depth" or "cluster" (handed over to the greedy loop)."""
    K = n_out - 2
    m = len(X)
    key, bot = {}, {}
    segs = [(0, m - 1, -1)]
    levels = min(K, MAX_LEVELS)
    split_last = True
    for _ in range(levels):
        new = []
        for a, b, p in segs:
            if b - a < 2:
                continue
            dx, dy = X[b] - X[a], Y[b] - Y[a]
            c = np.abs(dx * (Y[a + 1:b] - Y[a]) - (X[a + 1:b] - X[a]) * dy)
            c = np.where(np.isnan(c), -1.0, c)
            if c.max() < 0:
                continue
            j = a + 1 + int(np.argmax(c))  # lowest index on ties
            best = c[j - a - 1]
            with np.errstate(all="ignore"):
                k = float(best * best / (dx * dx + dy * dy))
            key[j] = -1.0 if k != k else k
            bot[j] = j if p < 0 or _above(key, bot[p], j) else bot[p]
            new += [(a, j, j), (j, b, j)]
        split_last = bool(new)
        segs = new
        if not split_last:
            break
    if split_last and levels < K:
        return "depth"
    nodes = list(key)
    if len(nodes) <= K:
        return "all"
    ck = sorted(((key[bot[v]], -bot[v]) for v in nodes), reverse=True)
    boundary = ck[K - 1]
    above = sum(1 for c in ck if c > boundary)
    size = sum(1 for c in ck if c == boundary)
    steps = K - above
    if steps == size:
        return "whole"
    return "cluster" if size > MAX_CLUSTER or steps > MAX_STEPS else "walk"


ROUTES = {
    ("walk", 200_000, 1000, 4): "walk",
    ("noise0", 1500, 200, 16): "walk",
    ("zigzag", 200_000, 100, 4): "walk",
    ("zigzag", 200_000, 1000, 4): "walk",
    ("saw", 200_000, 20, 4): "whole",
    ("const", 200_000, 100, 4): "all",
    ("ties", 200_000, 100, 4): "walk",
    ("ties", 200_000, 600, 2): "depth",
    ("const", 200_000, 1000, 4): "depth",
    ("noise0", 3000, 375, 16): "cluster",
    ("noise0", 3000, 250, 24): "cluster",
    ("zigzag", 200_000, 1300, 8): "walk",
    ("noise0", 6000, 1500, 8): "cluster",
}


@pytest.mark.parametrize("case", sorted(ROUTES), ids=str)
def test_gpu_route_cases_take_their_routes(case):
    """Each Douglas-Peucker case of the GPU tests takes the kernel route its
    comment names (the same inputs, preselected by the oracle's MinMax)."""
    import importlib.util
    import os

    spec = importlib.util.spec_from_file_location(
        "gpu_simplifier_cases", os.path.join(os.path.dirname(os.path.abspath(__file__)), "test_gpu_simplifiers.py"))
    gpu_cases = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gpu_cases)
    assert case in gpu_cases.DP_ROUTES
    kind, n, n_out, r_ps = case
    y = gpu_cases._dp_series(kind, n, n + n_out)
    P = oracle.minmax(y, n_out, r_ps)
    X, Y = P.astype(np.float64), y[P].astype(np.float64)
    assert kernel_route(X, Y, n_out) == ROUTES[case]
