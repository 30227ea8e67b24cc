"""Plant plausible mistakes in copies of the oracle (CPU only) and show that
the pins reject every one of them: a dropped term, a wrong sign, a transposed
operand, a wrong tie rule, a wrong bucket, a wrong bin count or boundary, a
wrong rounding, a lost chain update."""
from __future__ import annotations

import faulthandler
import math
import multiprocessing

import numpy as np
import pytest

import oracle
from paper_2305_00332_amd import synth
from tests import pins

# sums whose exact value lies half-way between two binary64 neighbours, or that
# cancel: rounding ties to even and exactness both show
HALFWAY_CASES = [
    [2.0 ** 53, 1.0],
    [2.0 ** 53, 3.0],
    [2.0 ** 60, 2.0 ** 7, 2.0 ** 6],
    [1.0, 2.0 ** -60, -1.0],
    [2.0 ** 100, 1.0, -(2.0 ** 100)],
]

MUTANTS = {
    "min_tie_highest": ("if (y[i] < y[imin]) /* strict", "if (y[i] <= y[imin]) /* strict"),
    "max_tie_highest": ("if (y[i] > y[imax])\n                    imax = i;\n            }\n        }\n        bmin[b] = imin;",
                        "if (y[i] >= y[imax])\n                    imax = i;\n            }\n        }\n        bmin[b] = imin;"),
    "empty_bin_kept": ("        if (bmin[b] < 0) /* empty bin */\n            continue;\n", ""),
    "max_dropped_when_distinct": ("        if (bmax[b] != bmin[b])\n            P[cnt++] = bmax[b];\n", ""),
    "m4_min_tie_highest": ("if (y[i] < y[imin]) /* lowest index on ties (R12) */",
                           "if (y[i] <= y[imin]) /* lowest index on ties (R12) */"),
    "m4_max_tie_highest": ("if (y[i] > y[imax]) /* lowest index on ties (R12) */",
                           "if (y[i] >= y[imax]) /* lowest index on ties (R12) */"),
    "ceil_boundaries": ("return (int64_t)(((__int128)k * (__int128)len) / (__int128)parts);",
                        "return (int64_t)(((__int128)k * (__int128)len + parts - 1) / (__int128)parts);"),
    "nb_not_halved": ("int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 2); /* R1 */",
                      "int64_t nb = (int64_t)(((__int128)n_out * r_ps) / 1); /* R1 */"),
    "area_dropped_term": ("fabs((Xa - MX[k]) * (Yj - Ya) - (Xa - Xj) * (MY[k] - Ya))",
                          "fabs((Xa - MX[k]) * (Yj - Ya))"),
    "area_wrong_sign": ("fabs((Xa - MX[k]) * (Yj - Ya) - (Xa - Xj) * (MY[k] - Ya))",
                        "fabs((Xa - MX[k]) * (Yj - Ya) + (Xa - Xj) * (MY[k] - Ya))"),
    "area_transposed": ("fabs((Xa - MX[k]) * (Yj - Ya) - (Xa - Xj) * (MY[k] - Ya))",
                        "fabs((Xa - MY[k]) * (Yj - Ya) - (Xa - Xj) * (MX[k] - Ya))"),
    "area_tie_highest": ("if (area > best) { /* strict", "if (area >= best) { /* strict"),
    "typed_area_tie_highest": ("if (area > best) { /* lowest index on ties (R8) */",
                               "if (area >= best) { /* lowest index on ties (R8) */"),
    "mean_of_current_bucket": ("g0 = 1 + floor_frac(k + 1, m - 2, B);\n            g1 = 1 + floor_frac(k + 2, m - 2, B);",
                               "g0 = 1 + floor_frac(k, m - 2, B);\n            g1 = 1 + floor_frac(k + 1, m - 2, B);", 0, 2),
    "typed_mean_of_current_bucket": ("g0 = 1 + floor_frac(k + 1, m - 2, B);\n            g1 = 1 + floor_frac(k + 2, m - 2, B);",
                               "g0 = 1 + floor_frac(k, m - 2, B);\n            g1 = 1 + floor_frac(k + 1, m - 2, B);", 1, 2),
    "last_mean_two_points": ("g0 = m - 1;\n            g1 = m;", "g0 = m - 2;\n            g1 = m;", 0, 2),
    "typed_last_mean_two_points": ("g0 = m - 1;\n            g1 = m;", "g0 = m - 2;\n            g1 = m;", 1, 2),
    "mean_count_off_by_one": ("double c = (double)(g1 - g0);", "double c = (double)(g1 - g0 + 1);", 0, 2),
    "typed_mean_count_off_by_one": ("double c = (double)(g1 - g0);", "double c = (double)(g1 - g0 + 1);", 1, 2),
    "chain_not_updated": ("out[k + 1] = sel;\n        a = sel;", "out[k + 1] = sel;\n        a = 0;", 0, 2),
    "typed_chain_not_updated": ("out[k + 1] = sel;\n        a = sel;", "out[k + 1] = sel;\n        a = 0;", 1, 2),
    "round_half_up": ("if (round_bit && (sticky || (mant & 1u)))", "if (round_bit)"),
    "sum_in_double": ("MY[k] = exact_sum_f32(ys + g0, g1 - g0) / c;",
                      "{ double s_ = 0; for (int64_t q = g0; q < g1; q++) s_ += (double)ys[q]; MY[k] = s_ / c; }"),
    "subnormal_shift": ("mant = frac;\n            shift = 0;", "mant = frac;\n            shift = 1;", 0, 2),
    "f64_subnormal_shift": ("mant = frac;\n            shift = 0;", "mant = frac;\n            shift = 1;", 1, 2),
    "gather_wrong_x": ("xs[i] = (xk == XK_INT64) ? x[P[i]] : P[i];", "xs[i] = (xk == XK_INT64) ? x[i] : P[i];"),
    "no_first_point": ("    P[cnt++] = 0;\n    for (int64_t b = 0;", "    for (int64_t b = 0;", 0, 2),
    "typed_no_first_point": ("    P[cnt++] = 0;\n    for (int64_t b = 0;", "    for (int64_t b = 0;", 1, 2),
    "m4_no_last": ("        out[cnt++] = hi - 1;\n", ""),
    "m4_bins_not_quartered": ("    int64_t nb = n_out / 4;", "    int64_t nb = n_out / 2;"),
    "xbin_edges_from_first_point": ("int64_t right = x_edge(x[1], x[n - 1], b + 1, nb);",
                                    "int64_t right = x_edge(x[0], x[n - 1], b + 1, nb);"),
    "xbin_right_edge_inclusive": ("while (hi < n - 1 && x[hi] < right)", "while (hi < n - 1 && x[hi] <= right)"),
    "xbin_min_tie_highest": ("if (y[i] < y[imin]) /* lowest index on ties (R14, R3) */",
                             "if (y[i] <= y[imin]) /* lowest index on ties (R14, R3) */"),
    "typed_min_tie_highest": ("if (y_less(yk, y, i, imin)) /* lowest index on ties (R15, R3) */",
                              "if (!y_less(yk, y, imin, i)) /* lowest index on ties (R15, R3) */"),
    "typed_sum_f64_in_double": ("MY[k] = exact_sum_f64(Y + g0, g1 - g0) / c;",
                                "MY[k] = 0.0;\n        for (int64_t q = g0; q < g1; q++)\n            MY[k] += Y[q];\n        MY[k] /= c;"),
    "f64_sum_high_part_dropped": ("        big_add_u32_shifted(dst, (uint32_t)(mant >> 32), shift + 32);\n", ""),
    "typed_i32_as_float": ("    return (double)((const int32_t *)y)[i];", "    return (double)(float)((const int32_t *)y)[i];"),
    "vw_tie_highest": ("if (alive[i] && (sel < 0 || area[i] < area[sel]))", "if (alive[i] && (sel < 0 || area[i] <= area[sel]))"),
    "vw_neighbour_not_updated": ("        if (b < m - 1)\n            area[b] = vw_area(X, Y, a, b, next[b]);\n", ""),
    "vw_area_wrong_vertex": ("return fabs((X[a] - X[b]) * (Y[j] - Y[a]) - (X[a] - X[j]) * (Y[b] - Y[a])); /* R16 */",
                             "return fabs((X[a] - X[b]) * (Y[j] - Y[a]) - (X[a] - X[j]) * (Y[j] - Y[a])); /* R16 */"),
    "dp_key_not_normalised": ("*key = best * best / (dx * dx + dy * dy);", "*key = best * best;"),
    "dp_farthest_tie_highest": ("if (c > best) { /* lowest index on ties (R17) */", "if (c >= best) { /* lowest index on ties (R17) */"),
    "llb_squared_length": ("double t = L[i] + sqrt(dx * dx + dy * dy); /* R18 */", "double t = L[i] + (dx * dx + dy * dy); /* R18 */"),
    "llb_no_accumulation": ("double t = L[i] + sqrt(dx * dx + dy * dy); /* R18 */", "double t = sqrt(dx * dx + dy * dy); /* R18 */"),
    "everynth_ceil": ("        out[k] = floor_frac(k, n, n_out);", "        out[k] = (k * n + n_out - 1) / n_out;"),
}


def _passes_pins(v) -> bool:
    try:
        # MinMax vs numpy
        for seed in range(12):
            rng = np.random.default_rng(seed)
            n = int(rng.integers(3, 400))
            n_out = int(rng.integers(3, 60))
            r_ps = int(rng.integers(2, 9))
            y = synth.to_numpy([synth.random_walk, synth.ties_series, synth.subnormal_series][seed % 3](n, seed))
            if not np.array_equal(v.minmax(y, n_out, r_ps), pins.minmax_by_numpy(y, n_out, r_ps)):
                return False
        # sums and means vs fsum / Python ints
        for seed in range(6):
            y = synth.to_numpy(synth.extreme_series(200, seed))
            if v.exact_sum_f32(y) != math.fsum(float(t) for t in y):
                return False
            ys = synth.to_numpy(synth.subnormal_series(100, seed))
            if v.exact_sum_f32(ys) != math.fsum(float(t) for t in ys):
                return False
        for case in HALFWAY_CASES:
            a = np.array(case, dtype=np.float32)
            if v.exact_sum_f32(a) != math.fsum(float(t) for t in a):
                return False
        for seed in range(6):
            m, n_out = 300, 20 + seed
            y = synth.to_numpy(synth.random_walk(m, seed) if seed % 2 else synth.extreme_series(m, seed))
            MX, MY = v.lttb_means(y, n_out)
            bk = pins.lttb_buckets(m, n_out)
            B = n_out - 2
            for k in range(B):
                g0, g1 = bk[k + 1] if k < B - 1 else (m - 1, m)
                if MX[k] != float(sum(range(g0, g1))) / (g1 - g0):
                    return False
                if MY[k] != math.fsum(float(t) for t in y[g0:g1]) / (g1 - g0):
                    return False
        # M4 and EveryNth vs numpy / partition starts
        for seed in range(6):
            gen = synth.ties_series if seed % 2 else synth.random_walk
            y = synth.to_numpy(gen(300 + 97 * seed, seed))
            if not np.array_equal(v.m4(y, 8 + 4 * seed), pins.m4_by_numpy(y, 8 + 4 * seed)):
                return False
            if not np.array_equal(v.everynth(1000 + seed, 7 + seed), pins.everynth_by_parts(1000 + seed, 7 + seed)):
                return False
        # x-equal-width bins vs numpy
        for seed in range(6):
            n = 400 + 131 * seed
            gen = synth.ties_series if seed % 2 else synth.random_walk
            y = synth.to_numpy(gen(n, seed))
            x = np.cumsum(1 + (np.arange(n) * 7919 + seed) % 13).astype(np.int64)
            if not np.array_equal(v.minmax_xbins(y, x, 10 + seed, 4), pins.minmax_xbins_by_numpy(y, x, 10 + seed, 4)):
                return False
        # other value types: exact binary64 sums, numpy MinMax, float32 reduction, cancellation means
        import math as _m
        for seed in range(6):
            rng = np.random.default_rng(seed)
            vals = rng.standard_normal(50 + seed) * 10.0 ** rng.integers(-30, 30, size=50 + seed)
            if v.exact_sum_f64(vals) != _m.fsum(vals):
                return False
            subs = rng.standard_normal(40) * 5e-324 * 2.0 ** rng.integers(0, 70, size=40)
            if v.exact_sum_f64(subs) != _m.fsum(subs):
                return False
            yi = (rng.integers(-2 ** 31, 2 ** 31 - 1, size=400 + 17 * seed)).astype(np.int32)
            if not np.array_equal(v.minmax_typed(yi, 20, 2), pins.minmax_by_numpy(yi, 20, 2)):
                return False
            yt = synth.to_numpy(synth.ties_series(300 + 29 * seed, seed)).astype(np.float64)
            if not np.array_equal(v.minmax_typed(yt, 20, 4), pins.minmax_by_numpy(yt, 20, 4)):
                return False
            y32 = synth.to_numpy(synth.random_walk(500 + 31 * seed, seed))
            if not np.array_equal(v.minmaxlttb_typed(y32.astype(np.float64), 17, 4), v.minmaxlttb(y32, 17, 4)):
                return False
            # means that cancel: values 1e17 +- small, where a running binary64 sum loses the small parts
            ph = np.arange(400) % 3  # +1e17, a small value (lost by a running sum), -1e17
            yc = np.where(ph == 0, 1e17, np.where(ph == 2, -1e17, rng.standard_normal(400)))
            xc = np.cumsum(rng.random(400) + 0.5) + 1e15
            MX, MY = v.lttb_means_typed(yc, 13, xc)
            if not (np.array_equal(MX, pins.means_by_fsum(xc, 13)) and np.array_equal(MY, pins.means_by_fsum(yc, 13))):
                return False
            yi = synth.to_numpy(synth.int_series(300, seed, scale=1e9))
            if not np.array_equal(v.lttb_means_typed(yi, 11)[1], pins.means_by_fsum(yi.astype(np.float64), 11)):
                return False
        # other simplifiers: collinear closed forms, exact-rational VW / DP, LLB brute force
        Xc = np.arange(50, dtype=np.float64)
        if list(v.simplify_points("vw", Xc, 3.0 * Xc - 7.0, 10)) != [0] + list(range(41, 50)):
            return False
        if list(v.simplify_points("dp", Xc, 3.0 * Xc - 7.0, 10)) != list(range(9)) + [49]:
            return False
        for seed in range(12):
            rng = np.random.default_rng(300 + seed)
            m = int(rng.integers(6, 40))
            X = np.cumsum(rng.integers(1, 9, size=m)).astype(np.float64)
            Y = rng.integers(-40, 41, size=m).astype(np.float64)
            if seed % 3 == 0:
                Y = np.round(Y / 8)
            k = int(rng.integers(3, m))
            if list(v.simplify_points("vw", X, Y, k)) != pins.vw_exact(X.tolist(), Y.tolist(), k):
                return False
            if list(v.simplify_points("dp", X, Y, k)) != pins.dp_exact(X.tolist(), Y.tolist(), k):
                return False
            k = 3 + seed % 3
            mm = k + 1 + seed % (2 * (k - 2))
            Xl = np.cumsum(rng.random(mm) + 0.1)
            Yl = rng.standard_normal(mm) * 3
            paths = pins.llb_brute(Xl, Yl, k)
            if len(paths) > 1 and float(paths[0][0] - paths[1][0]) > 1e-9 * 100:
                if list(v.simplify_points("llb", Xl, Yl, k)) != paths[0][1]:
                    return False
        # exact-regime LTTB vs rationals
        for seed in range(30):
            rng = np.random.default_rng(seed)
            B = int(rng.integers(1, 20))
            w = int(2 ** rng.integers(0, 4))
            m = B * w + 2
            y = rng.integers(-1024, 1025, size=m).astype(np.float32)
            if seed % 3 == 0:
                y = np.round(y / 256).astype(np.float32)
            x = np.cumsum(rng.integers(1, 64, size=m)).astype(np.int64) if seed % 2 else None
            xs = np.arange(m) if x is None else x
            want = pins.lttb_exact([int(t) for t in xs], [int(t) for t in y], B + 2)
            if list(v.lttb(y, B + 2, x)) != want:
                return False
            # the typed path with every point preselected (nb >= m - 2), binary64 and int32 y
            r_big = 2 * m
            xf = None if x is None else x.astype(np.float64)
            if list(v.minmaxlttb_typed(y.astype(np.float64), B + 2, r_big, xf)) != want:
                return False
            if list(v.minmaxlttb_typed(y.astype(np.int32), B + 2, r_big, x)) != want:
                return False
        # MinMaxLTTB invariants + near-optimality over P
        for seed in range(8):
            rng = np.random.default_rng(50 + seed)
            n = int(rng.integers(50, 2000))
            n_out = int(rng.integers(3, 60))
            y = synth.to_numpy(synth.random_walk(n, seed))
            x = synth.to_numpy(synth.irregular_x(n, seed)) if seed % 2 else None
            out = v.minmaxlttb(y, n_out, 4, x)
            pins.check_output_invariants(out, n, n_out)
            P = pins.minmax_by_numpy(y, n_out, 4)
            if not set(out.tolist()) <= set(P.tolist()):
                return False
            pos = np.searchsorted(P, out)
            pins.check_lttb_near_optimal(P if x is None else x[P], y[P], list(pos), n_out)
    except (AssertionError, oracle.OracleError):
        return False
    return True


def _run_isolated(src: str, so_path: str) -> bool:
    """Compile the variant and run the pins in a child process; a crash of the
    child (a mutant can overrun a buffer) counts as a failed pin."""
    ctx = multiprocessing.get_context("fork")
    q = ctx.Queue()

    def child():
        # a mutant that overruns a buffer may abort here; that exit code is the
        # expected outcome, so keep pytest's fault handler from printing a trace
        faulthandler.disable()
        q.put(_passes_pins(oracle.compile_variant(src, so_path)))

    p = ctx.Process(target=child)
    p.start()
    p.join(300)
    if p.is_alive():
        p.kill()
        p.join()
        return False
    if p.exitcode != 0:
        return False
    return q.get(timeout=5)


def test_unmodified_oracle_passes(tmp_path):
    assert _run_isolated(oracle.source_text(), str(tmp_path / "unmodified.so"))


def _plant(src: str, spec) -> str:
    """(old, new) replaces the one occurrence of old; (old, new, k, count)
    replaces occurrence k of old, which must occur exactly count times."""
    old, new = spec[0], spec[1]
    k, count = (spec[2], spec[3]) if len(spec) > 2 else (0, 1)
    assert src.count(old) == count, f"mutation site {old!r} found {src.count(old)} times, expected {count}"
    at = -1
    for _ in range(k + 1):
        at = src.index(old, at + 1)
    return src[:at] + new + src[at + len(old):]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = _plant(oracle.source_text(), MUTANTS[name])
    assert not _run_isolated(src, str(tmp_path / f"mut_{name}.so")), f"pins did not catch the planted mistake {name}"
