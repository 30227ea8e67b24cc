"""mmlttb_minmaxlttb_noalloc (workspace in the library's fixed device array)
against mmlttb_minmaxlttb (caller workspace) and the oracle, through the C ABI:
two calls in a row, the second on a smaller input, so the second call runs on
the array the first one left behind."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2305_00332_amd import _lib, ops, synth

pytestmark = pytest.mark.gpu


def _series(n, seed, with_x):
    if with_x:
        x, y = synth.composite_series(n, seed, device="cuda")
        return x, y
    return None, synth.random_walk(n, seed, device="cuda")


def _noalloc(y, n_out, r_ps, x=None):
    lib = _lib.load()
    n = y.numel()
    out = torch.full((max(min(n, n_out), 1),), -7, dtype=torch.int64, device=y.device)
    xk = _lib.X_INT64 if x is not None else _lib.X_IMPLICIT
    rc = lib.mmlttb_minmaxlttb_noalloc(xk, _lib.ptr(x), y.data_ptr(), n, n_out, r_ps, out.data_ptr(),
                                       _lib.stream_ptr())
    return rc, out[: min(n, n_out)]


@pytest.mark.parametrize("with_x", [False, True])
@pytest.mark.parametrize("first,second", [
    ((1_000_003, 1000, 4), (200_003, 500, 2)),
    ((3_000_000, 4000, 4), (50_000, 1000, 4)),
    ((20_000_000, 16384, 4), (1_000_000, 2000, 8)),
])
def test_two_calls_in_a_row_equal_the_workspace_call(with_x, first, second):
    for k, (n, n_out, r_ps) in enumerate((first, second)):
        x, y = _series(n, 100 + k, with_x)
        print(f"noalloc n={n} n_out={n_out} r_ps={r_ps} x={'int64' if with_x else 'implicit'}", flush=True)
        rc, got = _noalloc(y, n_out, r_ps, x)
        assert rc == _lib.OK, _lib.last_error()
        want = ops.minmaxlttb(y, n_out, r_ps, x=x)
        torch.cuda.synchronize()
        got, want = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(got, want)
        if n <= 3_000_000:
            x_np = None if x is None else x.cpu().numpy()
            assert np.array_equal(got, oracle.minmaxlttb(y.cpu().numpy(), n_out, r_ps, x_np))


def test_small_and_identity_inputs():
    for n, n_out, r_ps in [(1, 3, 2), (2, 3, 2), (3, 3, 2), (5, 3, 2), (7, 5, 200), (1000, 998, 2)]:
        y = synth.random_walk(n, 9, device="cuda")
        rc, got = _noalloc(y, n_out, r_ps)
        assert rc == _lib.OK, _lib.last_error()
        want = ops.minmaxlttb(y, n_out, r_ps).cpu().numpy()
        assert np.array_equal(got.cpu().numpy(), want)


def test_sizes_beyond_the_array_are_rejected_before_anything_runs():
    lib = _lib.load()
    y = synth.random_walk(10_000_000, 3, device="cuda")
    n_out, r_ps = 65536, 4
    assert lib.mmlttb_workspace_size(y.numel(), n_out, r_ps) > _lib.NOALLOC_SCRATCH_BYTES
    rc, out = _noalloc(y, n_out, r_ps)
    torch.cuda.synchronize()
    assert rc == _lib.EINVAL
    assert "fixed scratch" in _lib.last_error()
    assert bool((out == -7).all())


def test_allocates_nothing_on_the_device():
    y = synth.random_walk(2_000_000, 4, device="cuda")
    out = torch.empty(1000, dtype=torch.int64, device="cuda")
    ops.minmaxlttb_noalloc(y, 1000, 4, out=out)  # first call on the device looks the array up
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    free_before = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        ops.minmaxlttb_noalloc(y, 1000, 4, out=out)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    assert torch.cuda.mem_get_info()[0] == free_before
    assert np.array_equal(out.cpu().numpy(), ops.minmaxlttb(y, 1000, 4).cpu().numpy())


def test_argument_errors_match_the_workspace_call():
    lib = _lib.load()
    y = synth.random_walk(1000, 5, device="cuda")
    out = torch.empty(1000, dtype=torch.int64, device="cuda")
    for n_out, r_ps in [(2, 4), (100, 1), (100, 0)]:
        rc = lib.mmlttb_minmaxlttb_noalloc(0, None, y.data_ptr(), 1000, n_out, r_ps, out.data_ptr(), None)
        assert rc == _lib.EINVAL
    rc = lib.mmlttb_minmaxlttb_noalloc(1, None, y.data_ptr(), 1000, 100, 4, out.data_ptr(), None)
    assert rc == _lib.EINVAL
    rc = lib.mmlttb_minmaxlttb_noalloc(0, None, y.data_ptr(), 1000, 100, 4, None, None)
    assert rc == _lib.EINVAL
    assert ctypes.c_int(rc).value == _lib.EINVAL
