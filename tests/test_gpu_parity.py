"""GPU path == oracle, element by element (tolerance 0: indices are integers).

Randomised small and medium shapes spanning several work items per bin and
ragged tails, plus the edge cases of the method: tiny n, n_out at and around
n, every point preselected, constant and tied series, signed zeros,
subnormals, extreme magnitudes, epoch-nanosecond timestamps, misaligned
series starts, and launch-geometry sweeps (results must not move)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import ops, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _dev(y_np, offset=0):
    """Device copy of y starting `offset` floats into its allocation (misaligned start)."""
    buf = torch.empty(len(y_np) + offset, dtype=torch.float32, device=DEV)
    buf[offset:] = torch.from_numpy(np.ascontiguousarray(y_np)).to(DEV)
    return buf[offset:]


def _devx(x_np):
    return None if x_np is None else torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)


@pytest.fixture(params=[ops.CHAIN_SEQUENTIAL, ops.CHAIN_SEGMENTED], ids=["seqchain", "segchain"])
def chain_mode(request):
    """Both forms of the LTTB pass must give the oracle's picks."""
    old = ops.get_tuning()
    ops.set_tuning(0, 0, request.param)
    yield request.param
    ops.set_tuning(*old)


KINDS = ["walk", "ties", "subnormal", "extreme", "composite", "constant"]


def _series(kind, n, seed):
    if kind == "walk":
        return synth.to_numpy(synth.random_walk(n, seed))
    if kind == "ties":
        return synth.to_numpy(synth.ties_series(n, seed))
    if kind == "subnormal":
        return synth.to_numpy(synth.subnormal_series(n, seed))
    if kind == "extreme":
        return synth.to_numpy(synth.extreme_series(n, seed))
    if kind == "composite":
        return synth.to_numpy(synth.composite_series(n, seed, with_x=False)[1])
    return np.full(n, -0.0 if seed % 2 else 3.5, dtype=np.float32)


def _x_for(seed, n):
    k = seed % 3
    if k == 0:
        return None
    if k == 1:
        return synth.to_numpy(synth.irregular_x(n, seed))
    return synth.to_numpy(synth.epoch_x(n, seed))


def _cases(count, seed0, nmax):
    rng = np.random.default_rng(seed0)
    out = []
    for c in range(count):
        n = int(np.exp(rng.uniform(0, np.log(nmax))))
        n_out = int(rng.integers(3, max(4, min(n + 3, 3000))))
        r_ps = int(rng.choice([2, 2, 3, 4, 4, 6, 8, 16]))
        out.append((seed0 + c, KINDS[c % len(KINDS)], max(n, 1), n_out, r_ps, int(rng.integers(0, 4))))
    return out


def _check_minmax(y_np, n_out, r_ps, offset):
    P, m = ops.minmax(_dev(y_np, offset), n_out, r_ps)
    want = oracle.minmax(y_np, n_out, r_ps)
    got = P.cpu().numpy()
    assert m == len(want)
    np.testing.assert_array_equal(got, want)


def _check_mmlttb(y_np, n_out, r_ps, x_np, offset):
    got = ops.minmaxlttb(_dev(y_np, offset), n_out, r_ps, x=_devx(x_np)).cpu().numpy()
    want = oracle.minmaxlttb(y_np, n_out, r_ps, x_np)
    np.testing.assert_array_equal(got, want)


def _check_lttb(y_np, n_out, x_np, offset):
    got = ops.lttb(_dev(y_np, offset), n_out, x=_devx(x_np)).cpu().numpy()
    want = oracle.lttb(y_np, n_out, x_np)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("case", _cases(120, 10_000, 200_000), ids=lambda c: f"s{c[0]}-{c[1]}-n{c[2]}-o{c[3]}-r{c[4]}-a{c[5]}")
def test_minmax_random(case):
    seed, kind, n, n_out, r_ps, off = case
    _check_minmax(_series(kind, n, seed), n_out, r_ps, off)


@pytest.mark.parametrize("case", _cases(120, 20_000, 200_000), ids=lambda c: f"s{c[0]}-{c[1]}-n{c[2]}-o{c[3]}-r{c[4]}-a{c[5]}")
def test_minmaxlttb_random(case, chain_mode):
    seed, kind, n, n_out, r_ps, off = case
    _check_mmlttb(_series(kind, n, seed), n_out, r_ps, _x_for(seed, n), off)


@pytest.mark.parametrize("case", _cases(60, 30_000, 100_000), ids=lambda c: f"s{c[0]}-{c[1]}-n{c[2]}-o{c[3]}-a{c[5]}")
def test_lttb_random(case, chain_mode):
    seed, kind, n, n_out, _r, off = case
    _check_lttb(_series(kind, n, seed), n_out, _x_for(seed, n), off)


EDGE = [
    # (n, n_out, r_ps)
    (1, 3, 2), (2, 3, 2), (3, 3, 2), (4, 3, 2), (5, 3, 2), (6, 3, 2), (5, 4, 2), (7, 5, 3),
    (100, 99, 2), (100, 100, 2), (100, 101, 2), (100, 98, 2), (1000, 3, 2), (1000, 3, 200),
    (10_001, 5000, 2), (10_000, 4999, 2), (4002, 1000, 4), (4003, 1000, 4), (4001, 1000, 4),
    (65_537, 3, 2), (300_000, 7, 3), (1 << 20, 1000, 4), ((1 << 20) + 3, 1001, 5),
]


@pytest.mark.parametrize("n,n_out,r_ps", EDGE)
@pytest.mark.parametrize("kind", ["walk", "ties", "constant", "subnormal"])
def test_edge_shapes(n, n_out, r_ps, kind, chain_mode):
    seed = n * 7 + n_out
    y = _series(kind, n, seed)
    x = _x_for(seed, n)
    _check_minmax(y, n_out, r_ps, n % 4)
    _check_mmlttb(y, n_out, r_ps, x, (n + 1) % 4)
    if n <= 300_000:
        _check_lttb(y, n_out, x, (n + 2) % 4)


def _takes_fused_tail(n, n_out, r_ps):
    """Whether the library runs this call's tail as one fused launch (at most
    3840 bins, a segmented chain, and a chain segment's points with the
    bucket before and after within 640 staging slots)."""
    nb = n_out * r_ps // 2
    B = n_out - 2
    mbb = (2 * nb + B - 1) // B
    return nb < n - 2 and nb <= 3840 and mbb <= 64 and 34 * mbb + 2 <= 640


@pytest.mark.parametrize("n_out,r_ps", [(1920, 4), (1921, 4), (3, 2), (4, 2), (5, 3), (33, 2), (34, 2),
                                        (70, 16), (70, 17), (400, 17), (400, 18), (227, 16), (3840, 2),
                                        (3841, 2)])
def test_fused_tail_on_both_sides_of_its_limits(n_out, r_ps, chain_mode):
    """The fused tail (one workgroup per chain segment, the last one linking)
    and the three-launch form around the fused tail's limits: 3840 bins,
    640 staged points per segment, 1, 2 and many segments; both equal to the
    oracle, for implicit and int64 x and two alignments of y."""
    n = 1_200_007
    y = _series("walk", n, n_out * 7 + r_ps)
    x = synth.to_numpy(synth.irregular_x(n, n_out))
    fused = _takes_fused_tail(n, n_out, r_ps)
    assert fused == ((n_out, r_ps) in {(1920, 4), (3, 2), (4, 2), (5, 3), (33, 2), (34, 2), (70, 16), (70, 17),
                                       (400, 17), (227, 16), (3840, 2)})
    for off, xs in ((0, None), (3, x)):
        _check_mmlttb(y, n_out, r_ps, xs, off)


def test_signed_zero_and_planted_extremes(chain_mode):
    n = 50_000
    y = np.zeros(n, dtype=np.float32)
    y[::3] = -0.0
    y[777] = 5.0
    y[778] = 5.0  # tie: 777 must win
    y[40_000] = -7.0
    y[40_001] = -7.0
    for n_out, r_ps in [(10, 2), (100, 4), (1000, 8)]:
        _check_minmax(y, n_out, r_ps, 1)
        _check_mmlttb(y, n_out, r_ps, None, 2)


@pytest.mark.parametrize("unroll,chunk", [(1, 256), (2, 512), (4, 1024), (4, 16384), (8, 2048), (8, 65536), (4, 1 << 22)])
def test_results_do_not_depend_on_launch_geometry(unroll, chunk):
    old = ops.get_tuning()
    try:
        ops.set_tuning(unroll, chunk)
        for seed, n, n_out, r_ps in [(1, 2_000_003, 1000, 4), (2, 777_777, 97, 3), (3, 123_457, 4000, 8)]:
            y = _series("ties" if seed == 2 else "walk", n, seed)
            _check_minmax(y, n_out, r_ps, seed % 4)
            _check_mmlttb(y, n_out, r_ps, None, 0)
    finally:
        ops.set_tuning(*old)


def test_repeated_calls_identical():
    y = _dev(_series("walk", 3_000_001, 9))
    first = ops.minmaxlttb(y, 2000, 4).clone()
    for _ in range(5):
        assert torch.equal(ops.minmaxlttb(y, 2000, 4), first)


def test_errors_on_gpu():
    y = _dev(_series("walk", 1000, 1))
    with pytest.raises(RuntimeError):
        ops.minmaxlttb(y, 2, 4)
    with pytest.raises(RuntimeError):
        ops.minmaxlttb(y, 10, 1)
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(RuntimeError, match="workspace"):
        ops.minmaxlttb(y, 100, 4, ws=small)
    # a failed call leaves the next one unaffected
    np.testing.assert_array_equal(ops.minmaxlttb(y, 100, 4).cpu().numpy(),
                                  oracle.minmaxlttb(y.cpu().numpy(), 100, 4))


def test_profile_call_spans_cover_their_kernels():
    """Each successful call leaves one whole-call span, at least as long as the
    kernels launched inside it; a call rejected on the host leaves none."""
    y = _dev(_series("walk", 2_000_001, 5))
    names = ("init_keys", "minmax_bin_reduce", "preselect_tail", "preselect_compact_means", "lttb_chain_seg",
             "lttb_chain")
    ops.minmaxlttb(y, 1000, 4)
    torch.cuda.synchronize()
    ops.profile_enable(True)
    try:
        ops.profile_reset()
        for _ in range(4):
            ops.minmaxlttb(y, 1000, 4)
        with pytest.raises(RuntimeError):
            ops.minmaxlttb(y, 1000, 1)
        ops.minmaxlttb(y[:500], 1000, 4)  # n <= n_out: one iota launch, still one span
        torch.cuda.synchronize()
        spans = ops.profile_samples("call_minmaxlttb")
        per_kernel = {k: ops.profile_samples(k) for k in names}
    finally:
        ops.profile_enable(False)
        ops.profile_reset()
    assert len(spans) == 5
    launched = [k for k in names if per_kernel[k]]
    for k in launched:
        assert len(per_kernel[k]) == 4, k
    for i in range(4):
        inside = sum(per_kernel[k][i] for k in launched)
        assert spans[i] >= 0.95 * inside, (i, spans[i], inside)
    assert spans[4] > 0


@pytest.mark.parametrize("unroll,chunk", [(4, 1 << 22), (1, 256)], ids=["item-per-bin", "items-per-bin"])
@pytest.mark.parametrize("fill", [0x00, 0xFF, 0x5A])
def test_stale_workspace_bytes_do_not_leak(unroll, chunk, fill):
    """With 1500-2000 bins and chunks longer than a bin, each bin is one work
    item that stores its keys (no initialising launch); with 256-point chunks
    bins of 500-2000 points are several items merging into initialised keys.
    Either way, bytes left in the workspace (all zeros, all ones, a pattern)
    never reach the result."""
    old = ops.get_tuning()
    try:
        ops.set_tuning(unroll, chunk)
        for seed, n, n_out, r_ps, m4_out in [(11, 1_000_003, 1000, 4, 8000), (12, 3_000_001, 1500, 2, 6000)]:
            y_np = _series("ties" if seed % 2 else "walk", n, seed)
            y = _dev(y_np)
            ws = torch.full((ops.workspace_size(n, n_out, r_ps),), fill, dtype=torch.uint8, device=DEV)
            got = ops.minmaxlttb(y, n_out, r_ps, ws=ws)
            np.testing.assert_array_equal(got.cpu().numpy(), oracle.minmaxlttb(y_np, n_out, r_ps))
            ws.fill_(fill)
            P, m = ops.minmax(y, n_out, r_ps, ws=ws)
            np.testing.assert_array_equal(P[: int(m)].cpu().numpy(), oracle.minmax(y_np, n_out, r_ps))
            m4_ws = torch.full((ops.m4_workspace_size(n, m4_out),), fill, dtype=torch.uint8, device=DEV)
            idx4, m4 = ops.m4(y, m4_out, ws=m4_ws)  # 2000 / 1500 M4 bins
            np.testing.assert_array_equal(idx4[: int(m4)].cpu().numpy(), oracle.m4(y_np, m4_out))
    finally:
        ops.set_tuning(*old)


@pytest.mark.parametrize("unroll,chunk,n_out,r_ps", [(4, 1 << 20, 3000, 4), (4, 65536, 1000, 4), (2, 1 << 20, 4000, 8)],
                         ids=["whole-bins", "split-bins", "r8"])
def test_waves_looping_over_long_items(unroll, chunk, n_out, r_ps):
    """Items of >= 32768 points and more than 2048 of them: the stream grid is
    capped at 2048 waves and each wave loops over several items (whole bins
    storing their keys, or bin pieces merging by atomics); with r_ps = 8 the
    16000 items of 12500 points keep one wave each."""
    n = 200_000_003
    y_np = _series("walk", n, 21)
    y = _dev(y_np)
    old = ops.get_tuning()
    try:
        ops.set_tuning(unroll, chunk)
        got = ops.minmaxlttb(y, n_out, r_ps)
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.minmaxlttb(y_np, n_out, r_ps))
        P, m = ops.minmax(y, n_out, r_ps)
        np.testing.assert_array_equal(P[: int(m)].cpu().numpy(), oracle.minmax(y_np, n_out, r_ps))
        idx4, m4 = ops.m4(y, 4 * n_out * r_ps // 2)
        np.testing.assert_array_equal(idx4[: int(m4)].cpu().numpy(), oracle.m4(y_np, 4 * n_out * r_ps // 2))
    finally:
        ops.set_tuning(*old)


@pytest.mark.parametrize("n_out,r_ps", [(8192, 4), (16385, 2), (10240, 4), (10241, 4), (20000, 4), (5000, 16)],
                         ids=lambda v: str(v))
@pytest.mark.parametrize("xk", [0, 1, 2])
def test_tiled_compaction_around_its_threshold(n_out, r_ps, xk):
    """More than 16384 bins take the tiled compaction (tiles of 4096 bins:
    counts, slots, tiles) and the means over many workgroups; 16384 bins
    (n_out = 8192, r_ps = 4) the one-workgroup form. Ragged last tiles, bins of
    a few points, and every x kind."""
    n = 300_001 + xk
    seed = 600 + 3 * n_out + xk
    y_np = _series("ties" if xk == 1 else "walk", n, seed)
    x_np = _x_for(xk, n)
    y, x = _dev(y_np, xk), _devx(x_np)
    got = ops.minmaxlttb(y, n_out, r_ps, x=x).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, n_out, r_ps, x_np))
    P, m = ops.minmax(y, n_out, r_ps, x=x)
    np.testing.assert_array_equal(P[: int(m)].cpu().numpy(), oracle.minmax(y_np, n_out, r_ps))


@pytest.mark.parametrize("n_out", [32770, 32802, 32866, 70002], ids=lambda v: f"o{v}")
def test_two_level_link_of_long_chains(n_out):
    """More than 1024 chain segments (32 buckets each) link in two levels:
    chunk maps of 64 transitions, a chain over the chunks, then each chunk's
    segment starts. n_out = 32770 keeps 1024 segments (one level); 32802 and
    32866 give 1025 and 1027 (16 full chunks, then a ragged 17th)."""
    n = 400_003
    seed = 31 + n_out
    y_np = _series("walk", n, seed)
    x_np = _x_for(1, n)
    y, x = _dev(y_np), _devx(x_np)
    got = ops.minmaxlttb(y, n_out, 2, x=x).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.minmaxlttb(y_np, n_out, 2, x_np))
    got_l = ops.lttb(y, n_out).cpu().numpy()  # buckets of ~12 points: the segmented pass over all points
    np.testing.assert_array_equal(got_l, oracle.lttb(y_np, n_out))
