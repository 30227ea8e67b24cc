"""Autotuner for libmmlttb's execution parameters.

Parameters (none changes any result; see mmlttb_set_tuning):
  unroll  16-byte loads in flight per lane in the MinMax stream (points per
          thread per batch = 4 * unroll)
  chunk   points per MinMax work item (one wave each)
  tile    points a workgroup stages in LDS for batched series with small bins
          (bins per workgroup = tile / bin size, a power of two <= 256)

tune_single() sweeps unroll x chunk on one resident series, timing the stream
kernel with the library's HIP events; tune_typed() does the same for the
stream of the other value types (classes "typed_f64", "typed_i32");
tune_batched() sweeps tile x chunk x unroll on a batch, timing whole batched
calls (the batched class sets the batched stream's own unroll and chunk).
Results are cached as JSON, keyed by GPU architecture, HIP runtime and
library version and the workload class; apply(kind) sets the cached choice,
and the binding applies the single-series and batched entries when it loads
the library (on_load, under MMLTTB_TUNE=off|use|retune).

    python -m paper_2305_00332_amd.autotune --out tune_cache.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")


def device_key() -> str:
    import torch

    from . import _lib

    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", props.name)
    return f"{arch}|hip {torch.version.hip}|{_lib.version()}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_entry(kind: str, entry: dict, path: str = CACHE):
    cache = load_cache(path)
    cache.setdefault(device_key(), {})[kind] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


# Cache fields of each workload class -> mmlttb_set_tuning arguments. The
# typed streams ("typed_f64", "typed_i32") share the single-series settings.
_FIELDS = {
    "single": {"unroll": "unroll", "chunk": "chunk"},
    "typed_f64": {"unroll": "unroll", "chunk": "chunk"},
    "typed_i32": {"unroll": "unroll", "chunk": "chunk"},
    "batched": {"unroll": "batch_unroll", "chunk": "batch_chunk", "tile": "tile"},
}
LOAD_CLASSES = ("single", "batched")


def select(cache: dict, key: str, kind: str):
    """set_tuning keyword arguments of the cached best entry for (device key,
    workload class), or None when the cache holds no such entry."""
    entry = cache.get(key, {}).get(kind)
    if not entry:
        return None
    best = entry["best"]
    return {arg: int(best[f]) for f, arg in _FIELDS[kind].items() if f in best}


def apply(kind: str, path: str = CACHE):
    """Set the cached tuning for this device and workload class; returns the
    applied parameters, or None when the cache has no entry."""
    from . import ops

    args = select(load_cache(path), device_key(), kind)
    if args is None:
        return None
    ops.set_tuning(**args)
    return args


def on_load(path: str = CACHE) -> str:
    """Tuning policy applied when the library loads, from MMLTTB_TUNE:
    "off" keeps the compiled defaults (the settings measured best on MI355X);
    "use" (the default) applies the cached entries of this device for the
    single-series and batched classes, warning when there is none;
    "retune" measures both classes again on synthetic inputs on this device,
    stores them in the cache and applies them. Returns what was done."""
    import torch

    mode = os.environ.get("MMLTTB_TUNE", "use").strip().lower()
    if mode not in ("off", "use", "retune"):
        raise ValueError(f"MMLTTB_TUNE must be off, use or retune, not {mode!r}")
    if mode == "off" or not torch.cuda.is_available():
        return "compiled defaults"
    if mode == "retune":
        retune(path)
    applied = [k for k in LOAD_CLASSES if apply(k, path) is not None]
    if not applied:
        import warnings

        warnings.warn(f"libmmlttb: the tuning cache {path} has no entry for {device_key()}; the compiled defaults "
                      "are in use (MMLTTB_TUNE=retune measures this device)", RuntimeWarning, stacklevel=3)
        return "compiled defaults (no cache entry)"
    return "cache: " + ", ".join(applied)


def retune(path: str = CACHE, n: int = 250_000_000, batch_series: int = 1024, log=None):
    """Measure the single-series and batched classes on this device (a
    random-walk series of n points; a batch of the batched workload's recipe
    with batch_series series) and store the results in the cache."""
    import torch

    from . import synth

    y = synth.random_walk(n, 3, device="cuda")
    torch.cuda.synchronize()
    save_entry("single", tune_single(y, 1000, 4, log=log), path)
    del y
    lengths = synth.batch_lengths(batch_series, 1e3, 1e7, 4)
    n_outs = synth.choice([200, 500, 1000, 2000], batch_series, 40)
    x, yb, offsets = synth.batch_series(lengths, 4, device="cuda")
    torch.cuda.synchronize()
    segs = [(int(o), int(m), int(no), 4) for o, m, no in zip(offsets, lengths, n_outs)]
    save_entry("batched", tune_batched(yb, segs, x, log=log), path)


def _median_ms(fn, reps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(times)


def tune_single(y, n_out: int, r_ps: int, unrolls=(2, 4, 8), chunks=(16384, 65536, 262144, 1 << 20, 1 << 22), reps=5,
                log=None):
    """Sweep the stream kernel's parameters on one resident series."""
    import torch

    from . import ops

    old = ops.get_tuning()
    out = torch.empty(n_out, dtype=torch.int64, device=y.device)
    ws = torch.empty(ops.workspace_size(y.numel(), n_out, r_ps), dtype=torch.uint8, device=y.device)
    results = []
    try:
        for u, c in itertools.product(unrolls, chunks):
            ops.set_tuning(unroll=u, chunk=c)
            ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws)
            torch.cuda.synchronize()
            ops.profile_enable(True)
            ops.profile_reset()
            for _ in range(reps):
                ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws)
            torch.cuda.synchronize()
            ops.profile_enable(False)
            tot, cnt = ops.profile_read("minmax_bin_reduce")
            ms = tot / max(cnt, 1)
            results.append({"unroll": u, "chunk": ops.get_tuning()[1], "kernel_ms": round(ms, 5)})
            if log:
                log(f"  unroll={u} chunk={c}: {ms:.4f} ms")
    finally:
        ops.profile_enable(False)
        ops.set_tuning(*old)
    best = min(results, key=lambda r: r["kernel_ms"])
    return {"best": {"unroll": best["unroll"], "chunk": best["chunk"]}, "metric": "minmax_bin_reduce kernel ms",
            "workload": {"n": int(y.numel()), "n_out": n_out, "r_ps": r_ps}, "sweep": results}


def tune_typed(y, n_out: int, r_ps: int, unrolls=(1, 2, 4, 8), chunks=(65536, 262144, 1 << 20), reps=5, log=None):
    """Sweep the typed stream kernel's parameters on one resident series
    (float64 or int32 y, implicit x)."""
    import torch

    from . import ops

    old = ops.get_tuning()
    out = torch.empty(n_out, dtype=torch.int64, device=y.device)
    ws = torch.empty(ops.typed_workspace_size(y.numel(), n_out, r_ps), dtype=torch.uint8, device=y.device)
    results = []
    try:
        for u, c in itertools.product(unrolls, chunks):
            ops.set_tuning(unroll=u, chunk=c)
            ops.minmaxlttb_typed(y, n_out, r_ps, out=out, ws=ws)
            torch.cuda.synchronize()
            ops.profile_enable(True)
            ops.profile_reset()
            for _ in range(reps):
                ops.minmaxlttb_typed(y, n_out, r_ps, out=out, ws=ws)
            torch.cuda.synchronize()
            ops.profile_enable(False)
            tot, cnt = ops.profile_read("typed_bin_reduce")
            ms = tot / max(cnt, 1)
            results.append({"unroll": u, "chunk": ops.get_tuning()[1], "kernel_ms": round(ms, 5)})
            if log:
                log(f"  unroll={u} chunk={c}: {ms:.4f} ms")
    finally:
        ops.profile_enable(False)
        ops.set_tuning(*old)
    best = min(results, key=lambda r: r["kernel_ms"])
    return {"best": {"unroll": best["unroll"], "chunk": best["chunk"]}, "metric": "typed_bin_reduce kernel ms",
            "workload": {"n": int(y.numel()), "dtype": str(y.dtype), "n_out": n_out, "r_ps": r_ps},
            "sweep": results}


def tune_batched(y, segs, x=None, tiles=(2048, 4096, 8192), chunks=(16384, 65536, 262144), unrolls=(2, 4, 8), reps=3,
                 log=None):
    """Sweep the batched stream parameters on one batch (whole-call time)."""
    import torch

    from . import ops

    old = ops.get_tuning()
    table = ops.segment_table(segs)
    out = torch.empty(max(table[2], 1), dtype=torch.int64, device=y.device)
    ws = torch.empty(ops.batched_workspace_size(segs), dtype=torch.uint8, device=y.device)
    results = []
    try:
        for t, c, u in itertools.product(tiles, chunks, unrolls):
            ops.set_tuning(batch_unroll=u, batch_chunk=c, tile=t)
            ms = _median_ms(lambda: ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table), reps)
            results.append({"tile": t, "chunk": ops.get_tuning().batch_chunk, "unroll": u, "call_ms": round(ms, 4)})
            if log:
                log(f"  tile={t} chunk={c} unroll={u}: {ms:.3f} ms")
    finally:
        ops.set_tuning(*old)
    best = min(results, key=lambda r: r["call_ms"])
    return {"best": {"tile": best["tile"], "chunk": best["chunk"], "unroll": best["unroll"]},
            "metric": "batched call ms", "workload": {"series": len(segs), "points": int(sum(s[1] for s in segs))},
            "sweep": results}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--n", type=float, default=1e9)
    ap.add_argument("--batch-series", type=int, default=4096)
    ap.add_argument("--only", default="single,typed_f64,typed_i32,batched",
                    help="comma-separated workload classes to tune")
    args = ap.parse_args()
    only = set(args.only.split(","))

    import torch

    from . import _lib, synth

    def log(m):
        print(m, file=sys.stderr, flush=True)

    _lib.load()
    log(f"device {device_key()}")
    n = int(args.n)
    if "single" in only:
        log(f"single: {n} points")
        y = synth.random_walk(n, 3, device="cuda")
        torch.cuda.synchronize()
        save_entry("single", tune_single(y, 1000, 4, log=log), args.out)
        del y
        torch.cuda.empty_cache()
    for kind, make in (("typed_f64", lambda: synth.random_walk(n, 3, device="cuda", dtype=torch.float64)),
                       ("typed_i32", lambda: synth.int_series(n, 3, device="cuda"))):
        if kind in only:
            log(f"{kind}: {n} points")
            y = make()
            torch.cuda.synchronize()
            save_entry(kind, tune_typed(y, 1000, 4, log=log), args.out)
            del y
            torch.cuda.empty_cache()
    if "batched" not in only:
        print(json.dumps(load_cache(args.out).get(device_key(), {}), indent=1))
        return
    lengths = synth.batch_lengths(args.batch_series, 1e3, 1e7, 4)
    n_outs = synth.choice([200, 500, 1000, 2000], args.batch_series, 40)
    log(f"batched: {args.batch_series} series, {int(lengths.sum())} points")
    x, yb, offsets = synth.batch_series(lengths, 4, device="cuda")
    torch.cuda.synchronize()
    segs = [(int(o), int(m), int(no), 4) for o, m, no in zip(offsets, lengths, n_outs)]
    save_entry("batched", tune_batched(yb, segs, x, log=log), args.out)
    print(json.dumps(load_cache(args.out)[device_key()], indent=1))


if __name__ == "__main__":
    main()
