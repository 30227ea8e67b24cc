"""Python front end of libmmlttb on torch tensors (device memory + current stream).

    idx = minmaxlttb(y, n_out=1000, r_ps=4)            # y: float32 cuda tensor
    idx = minmaxlttb(y, n_out=2000, r_ps=4, x=x)       # x: int64 cuda tensor
    P, m = minmax(y, n_out, r_ps)
    idx = lttb(y, n_out, x=x)
    P, m = minmax(y, n_out, 1)                          # the MinMax downsampler
    idx, m = m4(y, n_out)
    idx = everynth(n, n_out, device=y.device)

Each call only checks tensor types and passes pointers; the C library checks
the arguments again and runs the whole path in HIP kernels on the current
stream. Results are int64 device tensors of indices into the series.
"""
from __future__ import annotations

from typing import NamedTuple

import torch

from . import _lib


def _as_series(y, x):
    if not isinstance(y, torch.Tensor) or y.dtype != torch.float32 or not y.is_cuda:
        raise TypeError("y must be a float32 CUDA (HIP) tensor")
    if y.dim() != 1 or not y.is_contiguous():
        raise ValueError("y must be 1-D and contiguous")
    if x is not None:
        if not isinstance(x, torch.Tensor) or x.dtype != torch.int64 or x.device != y.device:
            raise TypeError("x must be an int64 tensor on y's device")
        if x.dim() != 1 or not x.is_contiguous() or x.numel() != y.numel():
            raise ValueError("x must be 1-D, contiguous and as long as y")
    return (_lib.X_INT64 if x is not None else _lib.X_IMPLICIT)


def workspace_size(n: int, n_out: int, r_ps: int) -> int:
    return int(_lib.load().mmlttb_workspace_size(n, n_out, r_ps))


def lttb_workspace_size(n: int, n_out: int) -> int:
    return int(_lib.load().mmlttb_lttb_workspace_size(n, n_out))


def _workspace(nbytes: int, device, ws):
    if ws is not None:
        return ws
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def minmax(y, n_out: int, r_ps: int, x=None, out=None, count=None, ws=None, sync: bool = True):
    """MinMax preselection. Returns (P, m): P holds the sorted distinct indices in
    P[:m]. With sync=False, m is returned as the device scalar tensor instead."""
    lib = _lib.load()
    xk = _as_series(y, x)
    n = y.numel()
    nb = n_out * r_ps // 2
    cap = max(2 * nb + 2, min(n, 2), 1)
    out = out if out is not None else torch.empty(cap, dtype=torch.int64, device=y.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmax(xk, _lib.ptr(x), y.data_ptr(), n, n_out, r_ps, out.data_ptr(), count.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    if not sync:
        return out, count
    m = int(count.item())
    return out[:m], m


_YKIND = {torch.float32: _lib.Y_F32, torch.float64: _lib.Y_F64, torch.int32: _lib.Y_I32}
_XKIND = {torch.int64: _lib.X_INT64, torch.float64: _lib.X_F64}


def _typed_series(y, x):
    if not isinstance(y, torch.Tensor) or not y.is_cuda or y.dtype not in _YKIND:
        raise TypeError("y must be a float32, float64 or int32 CUDA (HIP) tensor")
    if y.dim() != 1 or not y.is_contiguous():
        raise ValueError("y must be 1-D and contiguous")
    if x is None:
        return _lib.X_IMPLICIT, _YKIND[y.dtype]
    if not isinstance(x, torch.Tensor) or x.dtype not in _XKIND or x.device != y.device:
        raise TypeError("x must be an int64 or float64 tensor on y's device")
    if x.dim() != 1 or not x.is_contiguous() or x.numel() != y.numel():
        raise ValueError("x must be 1-D, contiguous and as long as y")
    return _XKIND[x.dtype], _YKIND[y.dtype]


SIMPLIFIERS = {"vw": 1, "dp": 2, "llb": 3}


def simplify_workspace_size(n: int, n_out: int, r_ps: int) -> int:
    return int(_lib.load().mmlttb_simplify_workspace_size(n, n_out, r_ps))


def minmax_simplify(alg: str, y, n_out: int, r_ps: int, x=None, out=None, ws=None):
    """MinMax preselection, then Visvalingam-Whyatt ("vw"), Douglas-Peucker
    ("dp") or Longest-Line-Bucket ("llb") on the preselected points."""
    lib = _lib.load()
    xk = _as_series(y, x)
    n = y.numel()
    code = SIMPLIFIERS.get(alg, alg)
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_simplify_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmax_simplify(code, xk, _lib.ptr(x), y.data_ptr(), n, n_out, r_ps, out.data_ptr(),
                                          ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    return out[: min(n, n_out)]


def typed_workspace_size(n: int, n_out: int, r_ps: int) -> int:
    return int(_lib.load().mmlttb_typed_workspace_size(n, n_out, r_ps))


def minmax_typed(y, n_out: int, r_ps: int, out=None, count=None, ws=None, sync: bool = True):
    """MinMax preselection for float32, float64 or int32 y. Returns (P, m) as minmax()."""
    lib = _lib.load()
    _, yk = _typed_series(y, None)
    n = y.numel()
    cap = max(2 * (n_out * r_ps // 2) + 2, min(n, 2), 1)
    out = out if out is not None else torch.empty(cap, dtype=torch.int64, device=y.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_typed_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmax_typed(yk, y.data_ptr(), n, n_out, r_ps, out.data_ptr(), count.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    if not sync:
        return out, count
    m = int(count.item())
    return out[:m], m


def minmaxlttb_typed(y, n_out: int, r_ps: int, x=None, out=None, ws=None):
    """MinMaxLTTB for float32, float64 or int32 y and implicit, int64 or float64 x."""
    lib = _lib.load()
    xk, yk = _typed_series(y, x)
    n = y.numel()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_typed_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmaxlttb_typed(xk, _lib.ptr(x), yk, y.data_ptr(), n, n_out, r_ps, out.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    return out[: min(n, n_out)]


def xbins_workspace_size(n: int, n_out: int, r_ps: int) -> int:
    return int(_lib.load().mmlttb_xbins_workspace_size(n, n_out, r_ps))


def _xbins_series(y, x):
    if x is None:
        raise TypeError("bins of equal x width need x (int64, strictly increasing)")
    _as_series(y, x)


def minmax_xbins(y, x, n_out: int, r_ps: int, out=None, count=None, ws=None, sync: bool = True):
    """MinMax preselection with bins of equal x width. Returns (P, m) as minmax()."""
    lib = _lib.load()
    _xbins_series(y, x)
    n = y.numel()
    cap = max(2 * (n_out * r_ps // 2) + 2, min(n, 2), 1)
    out = out if out is not None else torch.empty(cap, dtype=torch.int64, device=y.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_xbins_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmax_xbins(x.data_ptr(), y.data_ptr(), n, n_out, r_ps, out.data_ptr(), count.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    if not sync:
        return out, count
    m = int(count.item())
    return out[:m], m


def minmaxlttb_xbins(y, x, n_out: int, r_ps: int, out=None, count=None, ws=None, sync: bool = True):
    """MinMaxLTTB with MinMax bins of equal x width. Returns the selected
    indices (fewer than n_out when gaps leave fewer preselected points); with
    sync=False, (out, device count) instead."""
    lib = _lib.load()
    _xbins_series(y, x)
    n = y.numel()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_xbins_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmaxlttb_xbins(x.data_ptr(), y.data_ptr(), n, n_out, r_ps, out.data_ptr(),
                                           count.data_ptr(), ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    if not sync:
        return out, count
    return out[: int(count.item())]


def m4_workspace_size(n: int, n_out: int) -> int:
    return int(_lib.load().mmlttb_m4_workspace_size(n, n_out))


def m4(y, n_out: int, out=None, count=None, ws=None, sync: bool = True):
    """M4: per equal-index bin the first, last, min and max point. Returns
    (idx, m) with the sorted distinct indices in idx[:m]; with sync=False, m is
    the device scalar tensor instead."""
    lib = _lib.load()
    _as_series(y, None)
    n = y.numel()
    out = out if out is not None else torch.empty(max(n_out, 1), dtype=torch.int64, device=y.device)
    count = count if count is not None else torch.empty(1, dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_m4_workspace_size(n, n_out), y.device, ws)
    _lib.check(lib.mmlttb_m4(y.data_ptr(), n, n_out, out.data_ptr(), count.data_ptr(), ws.data_ptr(), ws.numel(),
                             _lib.stream_ptr()))
    if not sync:
        return out, count
    m = int(count.item())
    return out[:m], m


def everynth(n: int, n_out: int, out=None, device="cuda"):
    """EveryNth: the min(n, n_out) indices floor(k*n/n_out)."""
    lib = _lib.load()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=device)
    _lib.check(lib.mmlttb_everynth(n, n_out, out.data_ptr(), _lib.stream_ptr()))
    return out[: min(n, n_out)]


def lttb_means(y, n_out: int, x=None, MX=None, MY=None):
    """(MX, MY): the next-bucket means LTTB takes over the m = len(y) given
    points (m > n_out), float64 device tensors of n_out - 2 values."""
    lib = _lib.load()
    xk = _as_series(y, x)
    B = n_out - 2
    MX = MX if MX is not None else torch.empty(max(B, 1), dtype=torch.float64, device=y.device)
    MY = MY if MY is not None else torch.empty(max(B, 1), dtype=torch.float64, device=y.device)
    _lib.check(lib.mmlttb_lttb_means(xk, _lib.ptr(x), y.data_ptr(), y.numel(), n_out, MX.data_ptr(), MY.data_ptr(),
                                     _lib.stream_ptr()))
    return MX[:B], MY[:B]


def lttb(y, n_out: int, x=None, out=None, ws=None):
    """Plain LTTB over every point (the comparator)."""
    lib = _lib.load()
    xk = _as_series(y, x)
    n = y.numel()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_lttb_workspace_size(n, n_out), y.device, ws)
    _lib.check(lib.mmlttb_lttb(xk, _lib.ptr(x), y.data_ptr(), n, n_out, out.data_ptr(), ws.data_ptr(), ws.numel(),
                               _lib.stream_ptr()))
    return out[: min(n, n_out)]


def minmaxlttb(y, n_out: int, r_ps: int, x=None, out=None, ws=None):
    """MinMaxLTTB: MinMax preselection then LTTB on the preselected points."""
    lib = _lib.load()
    xk = _as_series(y, x)
    n = y.numel()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    ws = _workspace(lib.mmlttb_workspace_size(n, n_out, r_ps), y.device, ws)
    _lib.check(lib.mmlttb_minmaxlttb(xk, _lib.ptr(x), y.data_ptr(), n, n_out, r_ps, out.data_ptr(), ws.data_ptr(),
                                     ws.numel(), _lib.stream_ptr()))
    return out[: min(n, n_out)]


def minmaxlttb_noalloc(y, n_out: int, r_ps: int, x=None, out=None):
    """MinMaxLTTB with the library's fixed device scratch as its workspace:
    the call allocates nothing in the library (pass `out` to allocate nothing
    at all). Calls that overlap on one device race on that scratch."""
    lib = _lib.load()
    xk = _as_series(y, x)
    n = y.numel()
    out = out if out is not None else torch.empty(max(min(n, n_out), 1), dtype=torch.int64, device=y.device)
    _lib.check(lib.mmlttb_minmaxlttb_noalloc(xk, _lib.ptr(x), y.data_ptr(), n, n_out, r_ps, out.data_ptr(),
                                             _lib.stream_ptr()))
    return out[: min(n, n_out)]


def segment_table(segs):
    """Build the C segment array from (offset, n, n_out, r_ps) tuples; output
    slots are packed in order. Returns (ctypes array, out_offsets, total_out)."""
    arr = (_lib.Segment * len(segs))()
    out_offsets = []
    pos = 0
    for i, (offset, n, n_out, r_ps) in enumerate(segs):
        arr[i].offset = int(offset)
        arr[i].n = int(n)
        arr[i].n_out = int(n_out)
        arr[i].r_ps = int(r_ps)
        arr[i].reserved = 0
        arr[i].out_offset = pos
        out_offsets.append(pos)
        pos += min(int(n), int(n_out))
    return arr, out_offsets, pos


def batched_workspace_size(segs) -> int:
    arr, _, _ = segment_table(segs)
    return int(_lib.load().mmlttb_batched_workspace_size(arr, len(segs)))


def minmaxlttb_batched(y_base, segs, x_base=None, out=None, ws=None, table=None):
    """MinMaxLTTB over many series in one call.

    y_base (and x_base) hold the series back to back; segs lists
    (offset, n, n_out, r_ps) per series. Returns (out, out_offsets): series i's
    min(n, n_out) segment-local indices are out[out_offsets[i]:...]."""
    lib = _lib.load()
    if not isinstance(y_base, torch.Tensor) or y_base.dtype != torch.float32 or not y_base.is_cuda:
        raise TypeError("y_base must be a float32 CUDA (HIP) tensor")
    if x_base is not None and (x_base.dtype != torch.int64 or x_base.device != y_base.device):
        raise TypeError("x_base must be an int64 tensor on y_base's device")
    arr, out_offsets, total = table if table is not None else segment_table(segs)
    xk = _lib.X_INT64 if x_base is not None else _lib.X_IMPLICIT
    out = out if out is not None else torch.empty(max(total, 1), dtype=torch.int64, device=y_base.device)
    ws = _workspace(lib.mmlttb_batched_workspace_size(arr, len(arr)), y_base.device, ws)
    _lib.check(lib.mmlttb_minmaxlttb_batched(xk, _lib.ptr(x_base), y_base.data_ptr(), arr, len(arr), out.data_ptr(),
                                             ws.data_ptr(), ws.numel(), _lib.stream_ptr()))
    return out, out_offsets


def set_graph_cache(max_graphs: int):
    """Capture batched calls on non-default streams into HIP graphs and replay
    repeated ones (0 disables and releases the cache)."""
    _lib.check(_lib.load().mmlttb_set_graph_cache(int(max_graphs)))


def graph_cache_stats():
    """(entries, replays, captures)"""
    import ctypes

    v = [ctypes.c_int64(0) for _ in range(3)]
    _lib.check(_lib.load().mmlttb_graph_cache_stats(*[ctypes.byref(t) for t in v]))
    return tuple(t.value for t in v)


CHAIN_SEQUENTIAL, CHAIN_SEGMENTED, CHAIN_AUTO = 1, 2, 3


class Tuning(NamedTuple):
    unroll: int
    chunk: int
    chain: int
    tile: int
    batch_unroll: int
    batch_chunk: int


def set_tuning(unroll: int = 0, chunk: int = 0, chain: int = 0, tile: int = 0, batch_unroll: int = 0,
               batch_chunk: int = 0):
    """Execution tuning (results never depend on it): single-series MinMax loads
    in flight per lane and points per work item, LTTB pass form (1 sequential,
    2 segmented, 3 automatic), small-bin tile points (batched series, and
    single series' short bins), batched large-bin
    loads in flight and points per work item. Zero keeps the current value, so
    set_tuning(*get_tuning()) restores a saved setting exactly."""
    _lib.check(_lib.load().mmlttb_set_tuning(unroll, chunk, chain, tile, batch_unroll, batch_chunk))


def get_tuning() -> Tuning:
    import ctypes

    ints = [ctypes.c_int(0) for _ in range(4)]
    longs = [ctypes.c_int64(0) for _ in range(2)]
    u, ch, t, bu = ints
    c, bc = longs
    _lib.check(_lib.load().mmlttb_get_tuning(ctypes.byref(u), ctypes.byref(c), ctypes.byref(ch), ctypes.byref(t),
                                             ctypes.byref(bu), ctypes.byref(bc)))
    return Tuning(u.value, c.value, ch.value, t.value, bu.value, bc.value)


def profile_enable(on: bool = True):
    _lib.check(_lib.load().mmlttb_profile_enable(1 if on else 0))


def profile_reset():
    _lib.check(_lib.load().mmlttb_profile_reset())


def profile_read(kernel: str):
    """(total milliseconds, launch count) of `kernel` since the last reset."""
    import ctypes

    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _lib.check(_lib.load().mmlttb_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def profile_samples(name: str):
    """The individual durations (milliseconds, launch order) recorded under
    `name` since the last reset: a kernel name, or "call_minmaxlttb" for whole
    minmaxlttb calls."""
    import ctypes

    lib = _lib.load()
    cnt = ctypes.c_int64(0)
    _lib.check(lib.mmlttb_profile_samples(name.encode(), None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_float * max(cnt.value, 1))()
    _lib.check(lib.mmlttb_profile_samples(name.encode(), buf, cnt.value, ctypes.byref(cnt)))
    return [float(buf[i]) for i in range(min(cnt.value, len(buf)))]
