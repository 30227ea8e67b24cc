"""ctypes wrapper around the plain C oracle -- TEST INFRASTRUCTURE ONLY.

Each function takes numpy arrays (y float32, x int64 or None for an implicit
x = 0..n-1) and returns numpy int64 index arrays. See ``mmlttb_oracle.c`` for
the definitions and the readings R1-R10 they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

XK_IMPLICIT = 0
XK_INT64 = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mmlttb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with -fopenmp: the independent MinMax bin loop (and the
# finiteness check) run on all cores; everything else, and every result, is the
# single-threaded oracle's. Timed beside it as the paper's parallel CPU case.
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

# No fast-math and no contraction: every double operation is one IEEE binary64
# operation rounded to nearest-even.
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Werror"]


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so`` and, with
    -fopenmp, ``oracle/liboracle_omp.so``."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} returned {rc}")
        self.rc = rc


_i64p = ctypes.POINTER(ctypes.c_int64)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)


def _bind(path: str):
    lib = ctypes.CDLL(path)
    lib.oracle_minmax.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p]
    lib.oracle_lttb.argtypes = [ctypes.c_int, _i64p, _f32p, ctypes.c_int64, ctypes.c_int64, _i64p]
    lib.oracle_minmaxlttb.argtypes = [ctypes.c_int, _i64p, _f32p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int32, _i64p]
    lib.oracle_lttb_means.argtypes = [ctypes.c_int, _i64p, _f32p, ctypes.c_int64, ctypes.c_int64, _f64p, _f64p]
    lib.oracle_exact_sum_f32.argtypes = [_f32p, ctypes.c_int64, _f64p]
    lib.oracle_exact_sum_i64.argtypes = [_i64p, ctypes.c_int64, _f64p]
    lib.oracle_m4.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int64, _i64p, _i64p]
    _vp = ctypes.c_void_p
    lib.oracle_minmax_typed.argtypes = [ctypes.c_int, _vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p]
    lib.oracle_minmaxlttb_typed.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int32, _i64p]
    lib.oracle_exact_sum_f64.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, _f64p]
    lib.oracle_minmax_simplify.argtypes = [ctypes.c_int, ctypes.c_int, _i64p, _f32p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int32, _i64p]
    lib.oracle_simplify_points.argtypes = [ctypes.c_int, _f64p, _f64p, ctypes.c_int64, ctypes.c_int64, _i64p]
    lib.oracle_lttb_means_typed.argtypes = [ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.c_int64, ctypes.c_int64,
                                            _f64p, _f64p]
    lib.oracle_minmax_xbins.argtypes = [_i64p, _f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p]
    lib.oracle_minmaxlttb_xbins.argtypes = [_i64p, _f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _i64p,
                                            _i64p]
    lib.oracle_everynth.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p]
    lib.oracle_threads.argtypes = []
    for f in ("oracle_minmax", "oracle_lttb", "oracle_minmaxlttb", "oracle_lttb_means",
              "oracle_exact_sum_f32", "oracle_exact_sum_i64", "oracle_m4", "oracle_everynth",
              "oracle_minmax_xbins", "oracle_minmaxlttb_xbins", "oracle_minmax_typed", "oracle_minmaxlttb_typed",
              "oracle_exact_sum_f64", "oracle_lttb_means_typed", "oracle_minmax_simplify",
              "oracle_simplify_points", "oracle_threads"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = None
_lib_omp = None


def _load():
    global _lib
    if _lib is None:
        # A test may point this at an instrumented build of the same source
        # (address and undefined-behaviour sanitizers); results are the same.
        override = os.environ.get("MMLTTB_ORACLE_LIB")
        if override:
            _lib = _bind(override)
            return _lib
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


def load_openmp():
    """The OpenMP build of the same source (pass it as ``_lib_override``)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build(force=False)
        _lib_omp = _bind(_LIB_OMP)
    return _lib_omp


def threads(lib=None) -> int:
    """Threads the given build's parallel loops may use (1 for the plain build)."""
    return int((lib or _load()).oracle_threads())


def compile_variant(src_text: str, out_path: str):
    """Compile a (test-modified) copy of the oracle source and return a module-like
    namespace with minmax/lttb/minmaxlttb/lttb_means bound to it. Used only by the
    test that plants mistakes in the oracle to show the pins catch them."""
    c_path = out_path[:-3] + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    flags = [f for f in CFLAGS if f != "-Werror"]
    subprocess.check_call(["gcc", *flags, "-w", "-o", out_path, c_path, "-lm"])
    lib = _bind(out_path)

    class _Variant:
        pass

    v = _Variant()
    v.minmax = lambda y, n_out, r_ps: minmax(y, n_out, r_ps, _lib_override=lib)
    v.lttb = lambda y, n_out, x=None: lttb(y, n_out, x, _lib_override=lib)
    v.minmaxlttb = lambda y, n_out, r_ps, x=None: minmaxlttb(y, n_out, r_ps, x, _lib_override=lib)
    v.lttb_means = lambda y, n_out, x=None: lttb_means(y, n_out, x, _lib_override=lib)
    v.m4 = lambda y, n_out: m4(y, n_out, _lib_override=lib)
    v.minmax_typed = lambda y, n_out, r_ps: minmax_typed(y, n_out, r_ps, _lib_override=lib)
    v.minmaxlttb_typed = lambda y, n_out, r_ps, x=None: minmaxlttb_typed(y, n_out, r_ps, x, _lib_override=lib)
    v.exact_sum_f64 = lambda a: exact_sum_f64(a, _lib_override=lib)
    v.minmax_simplify = lambda alg, y, n_out, r_ps, x=None: minmax_simplify(alg, y, n_out, r_ps, x, _lib_override=lib)
    v.simplify_points = lambda alg, X, Y, n_out: simplify_points(alg, X, Y, n_out, _lib_override=lib)
    v.lttb_means_typed = lambda y, n_out, x=None: lttb_means_typed(y, n_out, x, _lib_override=lib)
    v.minmax_xbins = lambda y, x, n_out, r_ps: minmax_xbins(y, x, n_out, r_ps, _lib_override=lib)
    v.minmaxlttb_xbins = lambda y, x, n_out, r_ps: minmaxlttb_xbins(y, x, n_out, r_ps, _lib_override=lib)
    v.everynth = lambda n, n_out: everynth(n, n_out, _lib_override=lib)
    v.exact_sum_f32 = lambda a: exact_sum_f32(a, _lib_override=lib)
    v.exact_sum_i64 = lambda a: exact_sum_i64(a, _lib_override=lib)
    return v


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def _f32(y) -> np.ndarray:
    y = np.ascontiguousarray(y)
    if y.dtype != np.float32:
        raise TypeError("y must be float32")
    return y


def _x(x):
    if x is None:
        return XK_IMPLICIT, None, None
    x = np.ascontiguousarray(x)
    if x.dtype != np.int64:
        raise TypeError("x must be int64")
    return XK_INT64, x, x.ctypes.data_as(_i64p)


def _ptr(a, t):
    # a zero-length array still needs a valid pointer
    return a.ctypes.data_as(t) if a.size else ctypes.cast(ctypes.create_string_buffer(16), t)


def minmax(y, n_out: int, r_ps: int, _lib_override=None) -> np.ndarray:
    """Sorted distinct MinMax preselection P (readings R1-R4); r_ps = 1 is the
    MinMax downsampler (R11)."""
    y = _f32(y)
    n = y.shape[0]
    nb = (n_out * r_ps) // 2
    P = np.empty(max(2 * nb + 2, n if n <= 2 else 0, 1), dtype=np.int64)
    m = ctypes.c_int64(0)
    rc = (_lib_override or _load()).oracle_minmax(_ptr(y, _f32p), n, n_out, r_ps, P.ctypes.data_as(_i64p), ctypes.byref(m))
    if rc != 0:
        raise OracleError(rc, "minmax")
    return P[: m.value].copy()


_YKINDS = {np.dtype(np.float32): 0, np.dtype(np.float64): 1, np.dtype(np.int32): 2}
_XKINDS = {np.dtype(np.int64): 1, np.dtype(np.float64): 2}


def _typed_y(y):
    y = np.ascontiguousarray(y)
    if y.dtype not in _YKINDS:
        raise TypeError("y must be float32, float64 or int32")
    return y, _YKINDS[y.dtype]


def minmax_typed(y, n_out: int, r_ps: int, _lib_override=None) -> np.ndarray:
    """MinMax preselection for float32, float64 or int32 y (reading R15)."""
    y, yk = _typed_y(y)
    n = y.shape[0]
    nb = n_out * r_ps // 2
    P = np.empty(max(2 * nb + 2, n if n <= 2 else 0, 1), dtype=np.int64)
    m = ctypes.c_int64(0)
    rc = (_lib_override or _load()).oracle_minmax_typed(yk, y.ctypes.data, n, n_out, r_ps, P.ctypes.data_as(_i64p),
                                                        ctypes.byref(m))
    if rc != 0:
        raise OracleError(rc, "minmax_typed")
    return P[: m.value].copy()


def minmaxlttb_typed(y, n_out: int, r_ps: int, x=None, _lib_override=None) -> np.ndarray:
    """MinMaxLTTB for float32, float64 or int32 y and implicit, int64 or
    float64 x (reading R15)."""
    y, yk = _typed_y(y)
    n = y.shape[0]
    xk, xp = 0, None
    if x is not None:
        x = np.ascontiguousarray(x)
        if x.dtype not in _XKINDS or x.shape[0] != n:
            raise TypeError("x must be int64 or float64, as long as y")
        xk, xp = _XKINDS[x.dtype], x.ctypes.data
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    rc = (_lib_override or _load()).oracle_minmaxlttb_typed(xk, xp, yk, y.ctypes.data, n, n_out, r_ps,
                                                            out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "minmaxlttb_typed")
    return out[: min(n, n_out)].copy()


def lttb_means_typed(y, n_out: int, x=None, _lib_override=None):
    """(MX, MY): LTTB's next-bucket means over all m = len(y) points, any value type (R6, R15)."""
    y, yk = _typed_y(y)
    m = y.shape[0]
    xk, xp = 0, None
    if x is not None:
        x = np.ascontiguousarray(x)
        if x.dtype not in _XKINDS or x.shape[0] != m:
            raise TypeError("x must be int64 or float64, as long as y")
        xk, xp = _XKINDS[x.dtype], x.ctypes.data
    B = max(n_out - 2, 1)
    MX = np.empty(B, dtype=np.float64)
    MY = np.empty(B, dtype=np.float64)
    rc = (_lib_override or _load()).oracle_lttb_means_typed(xk, xp, yk, y.ctypes.data, m, n_out,
                                                            MX.ctypes.data_as(_f64p), MY.ctypes.data_as(_f64p))
    if rc != 0:
        raise OracleError(rc, "lttb_means_typed")
    return MX, MY


SIMPLIFIERS = {"vw": 1, "dp": 2, "llb": 3}


def _alg(alg):
    a = SIMPLIFIERS.get(alg, alg)
    if a not in (1, 2, 3):
        raise ValueError(f"unknown simplifier {alg!r}")
    return a


def minmax_simplify(alg, y, n_out: int, r_ps: int, x=None, _lib_override=None) -> np.ndarray:
    """MinMax preselection, then Visvalingam-Whyatt ("vw"), Douglas-Peucker
    ("dp") or Longest-Line-Bucket ("llb") on the preselected points (R16-R18)."""
    y = _f32(y)
    n = y.shape[0]
    xk, xarr, xp = _x(x)
    assert xarr is None or xarr.shape[0] == n
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    rc = (_lib_override or _load()).oracle_minmax_simplify(_alg(alg), xk, xp, _ptr(y, _f32p), n, n_out, r_ps,
                                                           out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "minmax_simplify")
    return out[: min(n, n_out)].copy()


def simplify_points(alg, X, Y, n_out: int, _lib_override=None) -> np.ndarray:
    """The simplifier alone over m > n_out binary64 points (positions)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    out = np.empty(n_out, dtype=np.int64)
    rc = (_lib_override or _load()).oracle_simplify_points(_alg(alg), X.ctypes.data_as(_f64p), Y.ctypes.data_as(_f64p),
                                                           X.shape[0], n_out, out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "simplify_points")
    return out


def exact_sum_f64(a, _lib_override=None) -> float:
    """RN(exact sum) of binary64 values (reading R15)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    r = ctypes.c_double(0.0)
    (_lib_override or _load()).oracle_exact_sum_f64(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.shape[0],
                                                    ctypes.byref(r))
    return r.value


def minmax_xbins(y, x, n_out: int, r_ps: int, _lib_override=None) -> np.ndarray:
    """MinMax preselection with bins of equal x width (reading R14)."""
    y = _f32(y)
    x = np.ascontiguousarray(x, dtype=np.int64)
    n = y.shape[0]
    assert x.shape[0] == n
    nb = n_out * r_ps // 2
    P = np.empty(max(2 * nb + 2, n if n <= 2 else 0, 1), dtype=np.int64)
    m = ctypes.c_int64(0)
    rc = (_lib_override or _load()).oracle_minmax_xbins(x.ctypes.data_as(_i64p), _ptr(y, _f32p), n, n_out, r_ps,
                                                        P.ctypes.data_as(_i64p), ctypes.byref(m))
    if rc != 0:
        raise OracleError(rc, "minmax_xbins")
    return P[: m.value].copy()


def minmaxlttb_xbins(y, x, n_out: int, r_ps: int, _lib_override=None) -> np.ndarray:
    """MinMaxLTTB with MinMax bins of equal x width (reading R14)."""
    y = _f32(y)
    x = np.ascontiguousarray(x, dtype=np.int64)
    n = y.shape[0]
    assert x.shape[0] == n
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    cnt = ctypes.c_int64(0)
    rc = (_lib_override or _load()).oracle_minmaxlttb_xbins(x.ctypes.data_as(_i64p), _ptr(y, _f32p), n, n_out, r_ps,
                                                            out.ctypes.data_as(_i64p), ctypes.byref(cnt))
    if rc != 0:
        raise OracleError(rc, "minmaxlttb_xbins")
    return out[: cnt.value].copy()


def m4(y, n_out: int, _lib_override=None) -> np.ndarray:
    """M4: per bin first, last, min and max (reading R12)."""
    y = _f32(y)
    n = y.shape[0]
    out = np.empty(max(4 * (n_out // 4), n if n <= n_out else 0, 1), dtype=np.int64)
    cnt = ctypes.c_int64(0)
    rc = (_lib_override or _load()).oracle_m4(_ptr(y, _f32p), n, n_out, out.ctypes.data_as(_i64p), ctypes.byref(cnt))
    if rc != 0:
        raise OracleError(rc, "m4")
    return out[: cnt.value].copy()


def everynth(n: int, n_out: int, _lib_override=None) -> np.ndarray:
    """EveryNth: n_out evenly spaced indices (reading R13)."""
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    rc = (_lib_override or _load()).oracle_everynth(n, n_out, out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "everynth")
    return out[: min(n, n_out)].copy()


def lttb(y, n_out: int, x=None, _lib_override=None) -> np.ndarray:
    """Plain LTTB over all points (readings R5-R9)."""
    y = _f32(y)
    xk, x, xp = _x(x)
    n = y.shape[0]
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    rc = (_lib_override or _load()).oracle_lttb(xk, xp, _ptr(y, _f32p), n, n_out, out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "lttb")
    return out[: min(n, n_out)].copy()


def minmaxlttb(y, n_out: int, r_ps: int, x=None, _lib_override=None) -> np.ndarray:
    """MinMaxLTTB: MinMax preselection, then LTTB on the preselected points."""
    y = _f32(y)
    xk, x, xp = _x(x)
    n = y.shape[0]
    out = np.empty(max(min(n, n_out), 1), dtype=np.int64)
    rc = (_lib_override or _load()).oracle_minmaxlttb(xk, xp, _ptr(y, _f32p), n, n_out, r_ps, out.ctypes.data_as(_i64p))
    if rc != 0:
        raise OracleError(rc, "minmaxlttb")
    return out[: min(n, n_out)].copy()


def minmaxlttb_segments(fetch, segs, workers: int = 1, slab_points: int = 1 << 27, _lib_override=None):
    """minmaxlttb of many segments of one long series pair, in segment order.

    segs holds (offset, n, n_out, r_ps) per segment (segments may overlap and
    come in any order); fetch(lo, hi) returns the host arrays (y[lo:hi],
    x[lo:hi] or None) of an element range. Segments are taken in offset order
    and grouped into slabs of about slab_points elements, each fetched once;
    the segments of a slab run on `workers` threads (the C calls release the
    GIL, and the oracle keeps no shared state). No arithmetic happens here:
    each result is minmaxlttb of that segment alone."""
    from concurrent.futures import ThreadPoolExecutor

    order = sorted(range(len(segs)), key=lambda i: (int(segs[i][0]), i))
    results = [None] * len(segs)
    pool = ThreadPoolExecutor(max_workers=max(1, workers)) if workers > 1 else None
    try:
        k = 0
        while k < len(order):
            lo = int(segs[order[k]][0])
            hi = lo + int(segs[order[k]][1])
            j = k + 1
            while j < len(order):
                o, n = int(segs[order[j]][0]), int(segs[order[j]][1])
                if max(hi, o + n) - lo > slab_points:
                    break
                hi = max(hi, o + n)
                j += 1
            ys, xs = fetch(lo, hi)

            def one(i, ys=ys, xs=xs, lo=lo):
                o, n, n_out, r_ps = (int(v) for v in segs[i])
                xi = None if xs is None else xs[o - lo: o - lo + n]
                return i, minmaxlttb(ys[o - lo: o - lo + n], n_out, r_ps, xi, _lib_override=_lib_override)

            batch = order[k:j]
            done = pool.map(one, batch) if pool else map(one, batch)
            for i, r in done:
                results[i] = r
            k = j
    finally:
        if pool:
            pool.shutdown()
    return results


def lttb_means(y, n_out: int, x=None, _lib_override=None):
    """(MX, MY) next-bucket means of LTTB over the given points (reading R6)."""
    y = _f32(y)
    xk, x, xp = _x(x)
    m = y.shape[0]
    B = n_out - 2
    MX = np.empty(B, dtype=np.float64)
    MY = np.empty(B, dtype=np.float64)
    rc = (_lib_override or _load()).oracle_lttb_means(xk, xp, _ptr(y, _f32p), m, n_out, MX.ctypes.data_as(_f64p),
                                   MY.ctypes.data_as(_f64p))
    if rc != 0:
        raise OracleError(rc, "lttb_means")
    return MX, MY


def exact_sum_f32(v, _lib_override=None) -> float:
    v = _f32(v)
    out = ctypes.c_double(0.0)
    (_lib_override or _load()).oracle_exact_sum_f32(_ptr(v, _f32p), v.shape[0], ctypes.byref(out))
    return out.value


def exact_sum_i64(v, _lib_override=None) -> float:
    v = np.ascontiguousarray(v, dtype=np.int64)
    out = ctypes.c_double(0.0)
    (_lib_override or _load()).oracle_exact_sum_i64(_ptr(v, _i64p), v.shape[0], ctypes.byref(out))
    return out.value
