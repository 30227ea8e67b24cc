"""Independent checkers used to pin the oracle (no code shared with it).

Everything here is written from the mathematics, not from the oracle's
code: bin and bucket membership by an element-wise inequality, extrema by
numpy's first-occurrence argmin/argmax, sums by math.fsum and Python's
correctly rounded int -> float, triangle areas as exact rationals through
the 3x3 determinant of homogeneous coordinates.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def partition_by_inequality(length: int, parts: int):
    """Partition offsets 0..length-1 into `parts` consecutive groups, where offset t
    belongs to group g exactly when g*length < (t+1)*parts <= (g+1)*length.
    Returns a list of (lo, hi) offset ranges (possibly empty)."""
    groups = [[] for _ in range(parts)]
    g = 0
    for t in range(length):
        while not (g * length < (t + 1) * parts <= (g + 1) * length):
            g += 1
            assert g < parts
        groups[g].append(t)
    out = []
    pos = 0
    for grp in groups:
        if grp:
            assert grp[0] == pos and grp[-1] == pos + len(grp) - 1
            out.append((grp[0], grp[-1] + 1))
            pos = grp[-1] + 1
        else:
            out.append((pos, pos))
    assert pos == length
    return out


def minmax_by_numpy(y: np.ndarray, n_out: int, r_ps: int) -> np.ndarray:
    """MinMax preselection from numpy's per-slice argmin/argmax (first occurrence)."""
    n = len(y)
    if n <= 2:
        return np.arange(n, dtype=np.int64)
    nb = n_out * r_ps // 2
    sel = {0, n - 1}
    for lo, hi in partition_by_inequality(n - 2, nb):
        if hi > lo:
            seg = y[1 + lo: 1 + hi]
            sel.add(1 + lo + int(np.argmin(seg)))
            sel.add(1 + lo + int(np.argmax(seg)))
    return np.array(sorted(sel), dtype=np.int64)


def exact_area2(xa, ya, xj, yj, mx, my) -> Fraction:
    """Twice the triangle area, exactly: |det [[xa, ya, 1], [xj, yj, 1], [mx, my, 1]]|."""
    d = xa * (yj - my) - ya * (xj - mx) + (xj * my - mx * yj)
    return abs(d)


def lttb_exact(xs, ys, n_out: int):
    """LTTB with exact rational arithmetic (means and areas exact), ties to the
    lowest position. xs, ys: sequences of ints/Fractions/floats (converted exactly)."""
    m = len(xs)
    if m <= n_out:
        return list(range(m))
    X = [Fraction(v) for v in xs]
    Y = [Fraction(v) for v in ys]
    B = n_out - 2
    buckets = [(1 + lo, 1 + hi) for lo, hi in partition_by_inequality(m - 2, B)]
    out = [0]
    a = 0
    for k in range(B):
        g0, g1 = buckets[k + 1] if k < B - 1 else (m - 1, m)
        c = g1 - g0
        mx = sum(X[g0:g1]) / c
        my = sum(Y[g0:g1]) / c
        best, sel = None, None
        for j in range(*buckets[k]):
            A = exact_area2(X[a], Y[a], X[j], Y[j], mx, my)
            if best is None or A > best:
                best, sel = A, j
        out.append(sel)
        a = sel
    out.append(m - 1)
    return out


def lttb_buckets(m: int, n_out: int):
    """Interior LTTB buckets over positions [1, m-1) as (lo, hi) ranges."""
    return [(1 + lo, 1 + hi) for lo, hi in partition_by_inequality(m - 2, n_out - 2)]


def check_lttb_near_optimal(xs_int, ys, out, n_out: int, rel=2.0 ** -44):
    """Each selection maximises the exact area within a rounding bound.

    Given the selections as made (the previous point a), exact means and exact
    areas are computed with rationals; the selected candidate's exact area must
    be within a relative rounding bound of every other candidate's, and no
    lower-indexed candidate may beat it by more than that bound."""
    m = len(xs_int)
    if m <= n_out:
        assert list(out) == list(range(m))
        return
    X = [Fraction(int(v)) if isinstance(v, (int, np.integer)) else Fraction(float(v)) for v in xs_int]
    Y = [Fraction(int(v)) if isinstance(v, (int, np.integer)) else Fraction(float(v)) for v in ys]
    B = n_out - 2
    buckets = lttb_buckets(m, n_out)
    assert out[0] == 0 and out[-1] == m - 1
    for k in range(B):
        a = out[k]
        sel = out[k + 1]
        lo, hi = buckets[k]
        assert lo <= sel < hi
        g0, g1 = buckets[k + 1] if k < B - 1 else (m - 1, m)
        c = g1 - g0
        mx = sum(X[g0:g1]) / c
        my = sum(Y[g0:g1]) / c
        areas = {}
        scale = {}
        for j in range(lo, hi):
            areas[j] = exact_area2(X[a], Y[a], X[j], Y[j], mx, my)
            t = (abs(X[a] - mx) * abs(Y[j] - Y[a]) + abs(X[a] - X[j]) * abs(my - Y[a])
                 + (abs(X[a]) + abs(X[j]) + abs(mx)) * (abs(Y[j] - Y[a]) + abs(my - Y[a]))
                 + (abs(Y[a]) + abs(Y[j]) + abs(my)) * (abs(X[a] - mx) + abs(X[a] - X[j])))
            scale[j] = t
        for j in range(lo, hi):
            tol = (scale[j] + scale[sel]) * Fraction(rel)
            assert areas[j] <= areas[sel] + tol, (k, j, sel)


def check_output_invariants(out, n: int, n_out: int):
    out = list(out)
    assert len(out) == min(n, n_out)
    if n <= n_out:
        assert out == list(range(n))
        return
    assert out[0] == 0 and out[-1] == n - 1
    assert all(b > a for a, b in zip(out, out[1:]))


def m4_by_numpy(y: np.ndarray, n_out: int) -> np.ndarray:
    """M4 from numpy: per part of all points, first, last, first-occurrence argmin/argmax."""
    n = len(y)
    if n <= n_out:
        return np.arange(n, dtype=np.int64)
    sel = set()
    for lo, hi in partition_by_inequality(n, n_out // 4):
        if hi > lo:
            seg = y[lo:hi]
            sel.update({lo, hi - 1, lo + int(np.argmin(seg)), lo + int(np.argmax(seg))})
    return np.array(sorted(sel), dtype=np.int64)


def everynth_by_parts(n: int, n_out: int) -> np.ndarray:
    """EveryNth as the first index of each part of an n_out-part balanced partition."""
    if n <= n_out:
        return np.arange(n, dtype=np.int64)
    return np.array([lo for lo, _ in partition_by_inequality(n, n_out)], dtype=np.int64)


def xbin_starts(x: np.ndarray, nb: int) -> np.ndarray:
    """Start index of each of nb equal x-width bins over the interior points,
    edges in exact Python integers, located with numpy's searchsorted."""
    n = len(x)
    x1, xl = int(x[1]), int(x[n - 1])
    edges = [x1 + (b * (xl - x1)) // nb for b in range(nb + 1)]
    inner = x[1:n - 1]
    starts = np.searchsorted(inner, np.array(edges[:-1], dtype=np.int64), side="left") + 1
    return np.append(starts, n - 1).astype(np.int64)


def minmax_xbins_by_numpy(y: np.ndarray, x: np.ndarray, n_out: int, r_ps: int) -> np.ndarray:
    n = len(y)
    if n <= 2:
        return np.arange(n, dtype=np.int64)
    nb = n_out * r_ps // 2
    st = xbin_starts(x, nb)
    sel = {0, n - 1}
    for b in range(nb):
        lo, hi = int(st[b]), int(st[b + 1])
        if hi > lo:
            seg = y[lo:hi]
            sel.add(lo + int(np.argmin(seg)))
            sel.add(lo + int(np.argmax(seg)))
    return np.array(sorted(sel), dtype=np.int64)


def means_by_fsum(v: np.ndarray, n_out: int) -> np.ndarray:
    """LTTB next-bucket means over all points from math.fsum (a correctly
    rounded sum) divided by the count; last interior bucket: the last point."""
    import math

    m = len(v)
    bk = lttb_buckets(m, n_out)
    out = []
    for k in range(n_out - 2):
        g0, g1 = bk[k + 1] if k < n_out - 3 else (m - 1, m)
        out.append(math.fsum(float(t) for t in v[g0:g1]) / (g1 - g0))
    return np.array(out, dtype=np.float64)


def vw_exact(xs, ys, n_out: int):
    """Visvalingam-Whyatt with exact rational areas: the remaining points kept
    as a list, the smallest doubled area removed (lowest index on ties)."""
    X = [Fraction(v) for v in xs]
    Y = [Fraction(v) for v in ys]
    keep = list(range(len(X)))

    def area(a, j, b):
        return abs((X[a] - X[b]) * (Y[j] - Y[a]) - (X[a] - X[j]) * (Y[b] - Y[a]))

    while len(keep) > n_out:
        best = None
        for t in range(1, len(keep) - 1):
            A = area(keep[t - 1], keep[t], keep[t + 1])
            if best is None or A < best[0]:
                best = (A, t)
        keep.pop(best[1])
    return keep


def dp_exact(xs, ys, n_out: int):
    """Douglas-Peucker with a point budget, exact rational squared distances:
    split the segment whose farthest point is farthest from its chord."""
    X = [Fraction(v) for v in xs]
    Y = [Fraction(v) for v in ys]
    kept = [0, len(X) - 1]
    while len(kept) < n_out:
        best = None
        for a, b in zip(kept, kept[1:]):
            cand = None
            for j in range(a + 1, b):
                c = abs((X[b] - X[a]) * (Y[j] - Y[a]) - (X[j] - X[a]) * (Y[b] - Y[a]))
                if cand is None or c > cand[0]:
                    cand = (c, j)
            if cand is None:
                continue
            key = cand[0] ** 2 / ((X[b] - X[a]) ** 2 + (Y[b] - Y[a]) ** 2)
            if best is None or key > best[0]:
                best = (key, cand[1])
        kept = sorted(kept + [best[1]])
    return kept


def llb_brute(X, Y, n_out: int, digits: int = 60):
    """Every path through the LTTB buckets (one point each, first and last
    fixed) with its length summed in `digits`-digit decimal arithmetic.
    Returns [(length, path), ...] sorted by decreasing length."""
    import itertools
    from decimal import Decimal, getcontext

    getcontext().prec = digits
    m = len(X)
    buckets = [[0]] + [list(range(lo, hi)) for lo, hi in lttb_buckets(m, n_out)] + [[m - 1]]
    D = [(Decimal(float(x)), Decimal(float(y))) for x, y in zip(X, Y)]
    out = []
    for path in itertools.product(*buckets):
        t = Decimal(0)
        for i, j in zip(path, path[1:]):
            dx, dy = D[j][0] - D[i][0], D[j][1] - D[i][1]
            t += (dx * dx + dy * dy).sqrt()
        out.append((t, list(path)))
    out.sort(key=lambda r: r[0], reverse=True)
    return out
