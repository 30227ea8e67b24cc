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
calls. Results are cached as JSON, keyed by GPU architecture, HIP runtime and
library version and the workload class; apply(kind) sets the cached choice.

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


def apply(kind: str, path: str = CACHE):
    """Set the cached tuning for this device and workload class; returns the
    applied parameters, or None when the cache has no entry."""
    from . import ops

    entry = load_cache(path).get(device_key(), {}).get(kind)
    if not entry:
        return None
    best = entry["best"]
    ops.set_tuning(unroll=best.get("unroll", 0), chunk=best.get("chunk", 0), tile=best.get("tile", 0))
    return best


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
            ops.set_tuning(unroll=u, chunk=c, tile=t)
            ms = _median_ms(lambda: ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table), reps)
            results.append({"tile": t, "chunk": ops.get_tuning()[1], "unroll": u, "call_ms": round(ms, 4)})
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
