"""GPU == oracle for the other value types, element by element: float64,
int32 and float32 y with implicit, int64 and float64 x (mmlttb_minmax_typed,
mmlttb_minmaxlttb_typed). Random shapes over several work items per bin and
ragged tails; subnormal, huge, tied and signed-zero float64 values; extreme
int32 values; both LTTB pass forms; launch-geometry sweeps; the typed float32
path against the float32 library path; 1e8 points; argument errors."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
DMAX = sys.float_info.max


def _y(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "f64walk":
        return synth.to_numpy(synth.random_walk(n, seed, dtype=torch.float64))
    if kind == "f64wide":  # magnitudes 1e-300..1e300, subnormals, signed zeros
        v = rng.standard_normal(n) * 10.0 ** rng.integers(-300, 300, size=n)
        v[rng.random(n) < 0.05] = 5e-324 * rng.integers(-100, 100)
        v[rng.random(n) < 0.05] = -0.0
        return v
    if kind == "f64ties":
        return np.round(rng.standard_normal(n) * 2) / 4 * (1 + 2.0 ** -40)
    if kind == "i32walk":
        return synth.to_numpy(synth.int_series(n, seed))
    if kind == "i32extreme":
        return rng.choice(np.array([-2 ** 31, 2 ** 31 - 1, 0, -1, 1], dtype=np.int32), size=n)
    return synth.to_numpy(synth.random_walk(n, seed))  # f32


def _x(kind, n, seed):
    if kind == "int64":
        return synth.to_numpy(synth.irregular_x(n, seed))
    if kind == "f64":
        return synth.to_numpy(synth.float_x(n, seed))
    return None


YKINDS = ["f64walk", "f64wide", "f64ties", "i32walk", "i32extreme", "f32"]
XKINDS = [None, "int64", "f64"]


def _dev(a, offset=0):
    t = torch.from_numpy(np.ascontiguousarray(a))
    buf = torch.empty(len(a) + offset, dtype=t.dtype, device=DEV)
    buf[offset:] = t.to(DEV)
    return buf[offset:]


@pytest.fixture(params=[ops.CHAIN_SEQUENTIAL, ops.CHAIN_SEGMENTED], ids=["seqchain", "segchain"])
def chain_mode(request):
    old = ops.get_tuning()
    ops.set_tuning(0, 0, request.param)
    yield request.param
    ops.set_tuning(*old)


def _cases(count, seed0, nmax):
    rng = np.random.default_rng(seed0)
    out = []
    for c in range(count):
        n = max(1, int(np.exp(rng.uniform(0, np.log(nmax)))))
        n_out = int(rng.integers(3, max(4, min(n + 5, 3000))))
        r_ps = int(rng.choice([2, 2, 4, 4, 8, 16]))
        out.append((seed0 + c, YKINDS[c % len(YKINDS)], XKINDS[(c // 2) % 3], n, n_out, r_ps, int(rng.integers(0, 2))))
    return out


def _ids(c):
    return f"s{c[0]}-{c[1]}-{c[2]}-n{c[3]}-o{c[4]}-r{c[5]}-a{c[6]}"


def _check(y, x, n_out, r_ps, off=0):
    yd = _dev(y, off)
    xd = None if x is None else _dev(x)
    P, m = ops.minmax_typed(yd, n_out, r_ps)
    want_p = oracle.minmax_typed(y, n_out, r_ps)
    assert m == len(want_p)
    np.testing.assert_array_equal(P.cpu().numpy(), want_p)
    got = ops.minmaxlttb_typed(yd, n_out, r_ps, x=xd).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmaxlttb_typed(y, n_out, r_ps, x))


@pytest.mark.parametrize("case", _cases(120, 70_000, 300_000), ids=_ids)
def test_typed_random(case, chain_mode):
    seed, yk, xk, n, n_out, r_ps, off = case
    _check(_y(yk, n, seed), _x(xk, n, seed), n_out, r_ps, off)


@pytest.mark.parametrize("case", _cases(30, 71_000, 100_000), ids=_ids)
def test_typed_minmax_r1(case):
    seed, yk, _, n, n_out, _, off = case
    y = _y(yk, n, seed)
    P, m = ops.minmax_typed(_dev(y, off), n_out, 1)
    np.testing.assert_array_equal(P.cpu().numpy(), oracle.minmax_typed(y, n_out, 1))


@pytest.mark.parametrize("n,n_out,r_ps", [(1, 3, 2), (2, 3, 2), (3, 3, 2), (4, 3, 2), (5, 3, 2), (7, 5, 4),
                                          (100, 99, 2), (100, 101, 2), (1000, 3, 200), (4099, 1000, 2),
                                          (100_000, 3, 2), (100_000, 5000, 16)])
@pytest.mark.parametrize("yk", ["f64walk", "f64ties", "i32extreme"])
def test_typed_edges(n, n_out, r_ps, yk, chain_mode):
    _check(_y(yk, n, n + n_out), _x("f64", n, n) if n % 2 else None, n_out, r_ps)


def test_typed_float32_equals_float32_path():
    for seed, n, n_out, r_ps in [(1, 1_000_003, 1000, 4), (2, 77_777, 97, 2), (3, 500_001, 3000, 8)]:
        y = _dev(_y("f32", n, seed), seed % 4)
        x = _dev(_x("int64", n, seed)) if seed % 2 else None
        assert torch.equal(ops.minmaxlttb_typed(y, n_out, r_ps, x=x), ops.minmaxlttb(y, n_out, r_ps, x=x))
        P, m = ops.minmax_typed(y, n_out, r_ps)
        Q, mq = ops.minmax(y, n_out, r_ps)
        assert m == mq and torch.equal(P, Q)


def test_overflowing_means_follow_the_same_rule():
    # values near DBL_MAX: next-bucket sums overflow, some areas are NaN
    rng = np.random.default_rng(5)
    for n, n_out, r_ps in [(5000, 50, 4), (300_000, 20, 200)]:
        y = rng.choice(np.array([DMAX, -DMAX, DMAX / 2, 0.0, 1e308]), size=n)
        for x in (None, _x("f64", n, 3)):
            for mode in (ops.CHAIN_SEQUENTIAL, ops.CHAIN_SEGMENTED):
                old = ops.get_tuning()
                try:
                    ops.set_tuning(0, 0, mode)
                    got = ops.minmaxlttb_typed(_dev(y), n_out, r_ps, x=None if x is None else _dev(x))
                finally:
                    ops.set_tuning(*old)
                np.testing.assert_array_equal(got.cpu().numpy(), oracle.minmaxlttb_typed(y, n_out, r_ps, x))


@pytest.mark.parametrize("unroll,chunk", [(1, 256), (2, 512), (4, 16384), (8, 65536), (2, 1 << 20)])
def test_typed_independent_of_launch_geometry(unroll, chunk):
    old = ops.get_tuning()
    try:
        ops.set_tuning(unroll, chunk)
        for seed, n, n_out, r_ps, yk, xk in [(1, 2_000_003, 1000, 4, "f64walk", "f64"),
                                             (2, 777_777, 97, 2, "i32walk", None),
                                             (3, 123_457, 4000, 8, "f64ties", "int64")]:
            _check(_y(yk, n, seed), _x(xk, n, seed), n_out, r_ps, seed % 2)
    finally:
        ops.set_tuning(*old)


def test_hundred_million_points_f64():
    print("typed: 1e8 float64 points with float64 x", file=sys.stderr, flush=True)
    n = 100_000_000
    y = synth.random_walk(n, 11, device=DEV, dtype=torch.float64)
    x = synth.float_x(n, 11, device=DEV)
    y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
    for n_out, r_ps in [(2000, 4), (1000, 8)]:
        got = ops.minmaxlttb_typed(y, n_out, r_ps, x=x).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.minmaxlttb_typed(y_np, n_out, r_ps, x_np))
    yi = synth.int_series(n, 12, device=DEV)
    got = ops.minmaxlttb_typed(yi, 2000, 4).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmaxlttb_typed(yi.cpu().numpy(), 2000, 4))
    del y, x, yi
    torch.cuda.empty_cache()


def test_typed_errors():
    y = _dev(_y("f64walk", 1000, 1))
    with pytest.raises(TypeError):
        ops.minmax_typed(y.to(torch.float16), 100, 4)
    with pytest.raises(RuntimeError, match="r_ps"):
        ops.minmaxlttb_typed(y, 100, 1)
    with pytest.raises(RuntimeError, match="workspace"):
        ops.minmaxlttb_typed(y, 100, 4, ws=torch.empty(8, dtype=torch.uint8, device=DEV))
    with pytest.raises(RuntimeError, match="aligned"):
        _misaligned_f64_call()
    np.testing.assert_array_equal(ops.minmaxlttb_typed(y, 100, 4).cpu().numpy(),
                                  oracle.minmaxlttb_typed(y.cpu().numpy(), 100, 4))


def _misaligned_f64_call():
    from paper_2305_00332_amd import _lib

    lib = _lib.load()
    buf = torch.zeros(1000, dtype=torch.float64, device=DEV)
    out = torch.empty(100, dtype=torch.int64, device=DEV)
    ws = torch.empty(ops.typed_workspace_size(999, 100, 4), dtype=torch.uint8, device=DEV)
    # a binary64 series starting 4 bytes into an allocation: refused on the host
    _lib.check(lib.mmlttb_minmaxlttb_typed(_lib.X_IMPLICIT, None, _lib.Y_F64, buf.data_ptr() + 4, 999, 100, 4,
                                           out.data_ptr(), ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
