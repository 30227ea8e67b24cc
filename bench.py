"""Benchmark: MinMaxLTTB on one series of 1e9 float32 points (random walk,
implicit x, 4 GB resident in HBM), n_out=1000, r_ps=4.

    python bench.py [--steps K] [--warmup W] [--n N] [--n-out O] [--r-ps R]

A step is one mmlttb_minmaxlttb call (MinMax preselection, compaction,
next-bucket means, LTTB chain) on the resident series. Prints one JSON line:
throughput in Gpts/s over the K timed steps (nothing recorded around the
calls), the MinMax stream kernel against the HBM roofline (its duration
measured with HIP events recorded by the library on the launch stream during
a second pass of K steps), and the CPU oracle timed on the host as a baseline.
Every timed output is checked against the oracle (tolerance 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpts/s & HBM GB/s, MinMaxLTTB n=1e9; batched/served vs plain; p50/p99 ms"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "minmax_bin_reduce_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2305_00332_amd", "csrc", f)
                  for f in ("minmax.hip", "minmax_device.hpp", "device_common.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu_model() -> str:
    """CPU model name and logical core count of the host the oracle ran on."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical cores visible)"


# Freed device memory stays in torch's cache between sections (no
# empty_cache): a 1e9-point stream over memory that had been handed back to
# the driver and allocated again ran 5% slower (0.598 vs 0.568 ms) than over
# memory allocated once, at the same address too, so every section reads
# memory that has not been through a release.
_WALKS = {}


def shared_walk(n: int, seed: int, dev):
    """The float32 random walk that the single-series sections share (headline,
    n_out = 4000, other downsamplers, x-width bins, simplifiers), generated once
    and kept resident, so every section streams the same allocation: a fresh
    4 GB allocation made after others were freed streamed up to 5% slower in
    some sections than the first one."""
    from paper_2305_00332_amd import synth

    key = (n, seed, str(dev))
    if key not in _WALKS:
        _WALKS[key] = synth.random_walk(n, seed, device=dev)
    return _WALKS[key]


def oracle_seconds(fn, reps: int = 5):
    """Median wall time of `reps` runs of fn() after one warm-up, and its result."""
    import statistics

    out = fn()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times), out


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(launch_points: int, unroll: int, chunk: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when it is missing or was taken on another kernel source, size or tuning."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha") != kernel_source_sha() or t.get("n") != launch_points
            or t.get("unroll") != unroll or t.get("chunk") != chunk):
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=float, default=1e9)
    ap.add_argument("--n-out", type=int, default=1000)
    ap.add_argument("--r-ps", type=int, default=4)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--skip-headline", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-comparator", action="store_true")
    ap.add_argument("--skip-served", action="store_true")
    ap.add_argument("--skip-shapes", action="store_true")
    ap.add_argument("--skip-downsamplers", action="store_true")
    ap.add_argument("--skip-xbins", action="store_true")
    ap.add_argument("--skip-typed", action="store_true")
    ap.add_argument("--skip-simplifiers", action="store_true")
    ap.add_argument("--batch-series", type=int, default=4096)
    ap.add_argument("--pool-series", type=int, default=512)
    ap.add_argument("--rates", type=str, default="100,250,500,1000,2000,5000")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="requests per rate: max(--serve-min-requests, rate x this)")
    ap.add_argument("--serve-min-requests", type=int, default=2000)
    ap.add_argument("--serve-arena", type=int, default=1 << 30, help="device arena bytes of each serving form")
    ap.add_argument("--serve-oracle-sample", type=int, default=256)
    ap.add_argument("--serve-chunks", type=int, default=4,
                    help="each rate's stream in this many consecutive chunks, both forms on each, order alternating")
    ap.add_argument("--burst", type=int, default=2000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (the reference kernel for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: libmmlttb has no multi-GPU path; splitting the bins (one "
              "series) or the series (batches) across GPUs is a design, not code here.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2305_00332_amd import _lib

    torch.cuda.set_device(0)
    _lib.load()
    result = {"metric": METRIC}
    if not args.skip_headline:
        result.update(bench_headline(args))
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": 1 << 30, "write": 1 << 30}
        del src, dst
    if not args.skip_shapes:
        result["shapes"] = bench_shapes(args)
    if not args.skip_downsamplers:
        result["downsamplers"] = bench_downsamplers(args)
    if not args.skip_xbins:
        result["xbins"] = bench_xbins(args)
    if not args.skip_typed:
        result["typed"] = bench_typed(args)
    if not args.skip_simplifiers:
        result["simplifiers"] = bench_simplifiers(args)
    if not args.skip_comparator:
        result["comparator"] = bench_comparator(args)
    if not args.skip_batched:
        result["batched"] = bench_batched(args)
    if not args.skip_served:
        result["served"] = bench_served(args)
    print(json.dumps(result), flush=True)


def bench_headline(args):
    """One 1e9-point series: MinMaxLTTB steps, the stream kernel's roofline,
    the CPU oracle baseline and parity."""
    import numpy as np
    import torch

    from paper_2305_00332_amd import _lib, ops, synth

    n, n_out, r_ps = int(args.n), args.n_out, args.r_ps
    nb = n_out * r_ps // 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    _lib.load()

    log(f"tuning: {ops.get_tuning()} (set by: {_lib.tuning_source})")
    log(f"generating y: float32 random walk, n={n}, seed={args.seed}")
    y = shared_walk(n, args.seed, dev)
    torch.cuda.synchronize()
    out = torch.empty(n_out, dtype=torch.int64, device=dev)
    ws = torch.empty(ops.workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws)
    torch.cuda.synchronize()
    ref_out = out.clone()

    # value: K steps with the library's timing events off (nothing but the calls)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    stable_off = bool(torch.equal(out, ref_out))
    # per-kernel durations: the same K steps again with timing events around every launch
    log(f"timing {args.steps} steps with per-kernel events")
    ops.profile_enable(True)
    ops.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ops.profile_enable(False)
    ms_per_step_profiled = (t1 - t0) * 1e3 / args.steps
    kern = {}
    for k in ("init_keys", "minmax_bin_reduce", "preselect_tail", "preselect_compact_means", "preselect_all",
              "bucket_mean", "lttb_chain", "lttb_chain_seg"):
        tot, cnt = ops.profile_read(k)
        kern[k] = round(tot / cnt, 5) if cnt else None
    # device time of each timed call (events before its first and after its last launch)
    spans = ops.profile_samples("call_minmaxlttb")
    step_ms = ({"median": round(float(np.median(spans)), 5), "min": round(min(spans), 5),
                "max": round(max(spans), 5), "calls": len(spans)} if spans else None)
    stable = stable_off and bool(torch.equal(out, ref_out))

    # the LTTB pass in its sequential form on the same data (identical picks):
    # the tail after the stream, fused (compaction, means, segmented chain) or
    # compaction and means followed by the sequential chain
    seg_ms = (kern["preselect_tail"] or 0.0) + (kern["preselect_compact_means"] or 0.0) + \
        (kern["lttb_chain_seg"] or 0.0)
    old_tuning = ops.get_tuning()
    ops.set_tuning(chain=ops.CHAIN_SEQUENTIAL)
    out_seq = torch.empty_like(out)
    ops.minmaxlttb(y, n_out, r_ps, out=out_seq, ws=ws)
    torch.cuda.synchronize()
    ops.profile_enable(True)
    ops.profile_reset()
    for _ in range(5):
        ops.minmaxlttb(y, n_out, r_ps, out=out_seq, ws=ws)
    torch.cuda.synchronize()
    ops.profile_enable(False)
    tot, cnt = ops.profile_read("lttb_chain")
    tc, cc = ops.profile_read("preselect_compact_means")
    ops.set_tuning(*old_tuning)
    seq_ms = tot / max(cnt, 1) + tc / max(cc, 1)
    chain_forms = {"what": "tail after the stream: compaction, means and chain",
                   "sequential_ms": round(seq_ms, 5), "segmented_ms": round(seg_ms, 5),
                   "speedup": round(seq_ms / seg_ms, 2) if seg_ms else None,
                   "identical": bool(torch.equal(out_seq, out))}

    mm_ms = kern["minmax_bin_reduce"]
    alg_bytes = 4 * n + 16 * nb  # y read once + the bins' key pair
    achieved = alg_bytes / (mm_ms * 1e-3) / 1e9
    tun = ops.get_tuning()
    traffic = measured_traffic(n, tun[0], tun[1])
    roofline = {"bound": "hbm", "kernel": "minmax_bin_reduce", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": alg_bytes, "avg_ms": mm_ms}

    result = {
        "value": round(n / (ms_per_step * 1e-3) / 1e9, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"one series, n={n}, float32 random walk (sigma=1, seed={args.seed}), "
                               f"implicit x, resident in HBM; MinMaxLTTB n_out={n_out}, r_ps={r_ps}",
                   "n": n, "n_out": n_out, "r_ps": r_ps, "mode": "plain single-series call"},
        "kernel_avg_ms": kern,
        "ms_per_step_profiled": round(ms_per_step_profiled, 5),
        "step_device_ms": step_ms,
        "chain_forms": chain_forms,
        "tuning": ops.get_tuning()._asdict(),
        "roofline": roofline,
        "repeat_identical": stable,
    }

    if not args.no_cpu_baseline:
        import oracle

        log("copying y to the host for the oracle")
        y_np = y.cpu().numpy()
        result["config"]["y_sha256"] = hashlib.sha256(memoryview(y_np).cast("B")).hexdigest()
        times = []
        want = None
        for _ in range(max(1, args.cpu_reps)):
            c0 = time.perf_counter()
            want = oracle.minmaxlttb(y_np, n_out, r_ps)
            times.append(time.perf_counter() - c0)
        t = float(np.median(times))
        omp = oracle.load_openmp()
        omp_times = []
        for _ in range(max(1, args.cpu_reps)):
            c0 = time.perf_counter()
            want_omp = oracle.minmaxlttb(y_np, n_out, r_ps, _lib_override=omp)
            omp_times.append(time.perf_counter() - c0)
        t_omp = float(np.median(omp_times))
        result["cpu_baseline"] = {"value": round(n / t / 1e9, 4), "unit": "Gpts/s", "cores": 1, "kind": "oracle",
                                  "host_cpu": host_cpu_model(),
                                  "sample": f"the full workload (n={n}) run {len(times)} times single-threaded, "
                                            f"median {t:.3f} s"}
        result["cpu_openmp"] = {"value": round(n / t_omp / 1e9, 4), "unit": "Gpts/s", "cores": oracle.threads(omp),
                                "kind": "oracle source built with -fopenmp: the MinMax bin loop and the finiteness "
                                        "check on all threads, the rest single-threaded",
                                "sample": f"the full workload run {len(omp_times)} times, median {t_omp:.3f} s",
                                "identical": bool(np.array_equal(want_omp, want))}
        result["parity_vs_oracle"] = bool(np.array_equal(out.cpu().numpy(), want))
        del y_np
    del y, ws
    return result


def bench_shapes(args):
    """The other single-series shapes the method is quoted on: a 1e6-point
    random walk (4 MB, cache-resident, so launch-latency-bound) with MinMaxLTTB
    and whole-series LTTB, and the 1e9-point walk with n_out = 4000 (8000 bins
    of 125000 points, 3998 LTTB buckets). Host-clock time per call over
    back-to-back calls, median and min of the device spans of the calls, and
    parity with the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    dev = torch.device("cuda", 0)
    res = {}

    def timed_calls(fn, reps, span):
        """Host-clock time per call with the timing events off; then a second,
        profiled pass for the per-kernel times and the device spans."""
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        ops.profile_enable(True)
        ops.profile_reset()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        wall_profiled = (time.perf_counter() - t0) * 1e3 / reps
        ops.profile_enable(False)
        spans = ops.profile_samples(span) if span else []
        kern = {}
        for k in ("minmax_bin_reduce", "preselect_tail", "preselect_compact_means", "lttb_chain_seg", "lttb_chain",
                  "bucket_mean", "bucket_mean_wide", "lttb_scan", "lttb_hull", "lttb_tables", "lttb_table_walk",
                  "lttb_chain_wide"):
            tot, c = ops.profile_read(k)
            if c:
                kern[k] = round(tot / c, 5)
        e = {"call_ms": round(wall, 5), "call_ms_profiled": round(wall_profiled, 5), "kernel_avg_ms": kern}
        if spans:
            e["device_ms"] = {"median": round(float(np.median(spans)), 5), "min": round(min(spans), 5)}
        return e

    n, n_out, r_ps = 1_000_000, 1000, 4
    log(f"shapes: n={n}")
    y = synth.random_walk(n, 1, device=dev)
    torch.cuda.synchronize()
    out = torch.empty(n_out, dtype=torch.int64, device=dev)
    ws = torch.empty(ops.workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)
    # 64 copies (256 MB) taken in turn, so no call finds its input in the caches
    copies = [y.clone() for _ in range(64)]
    turn = iter(range(1 << 30))

    def next_copy():
        return copies[next(turn) % len(copies)]

    e = timed_calls(lambda: ops.minmaxlttb(next_copy(), n_out, r_ps, out=out, ws=ws), 200, "call_minmaxlttb")
    e["gpts_per_s"] = round(n / (e["call_ms"] * 1e-3) / 1e9, 3)
    same = timed_calls(lambda: ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws), 200, "call_minmaxlttb")
    e["one_buffer_call_ms"] = same["call_ms"]
    got = out.cpu().numpy()
    out_l = torch.empty(n_out, dtype=torch.int64, device=dev)
    ws_l = torch.empty(ops.lttb_workspace_size(n, n_out), dtype=torch.uint8, device=dev)
    el = timed_calls(lambda: ops.lttb(next_copy(), n_out, out=out_l, ws=ws_l), 200, None)
    el["gpts_per_s"] = round(n / (el["call_ms"] * 1e-3) / 1e9, 3)
    if not args.no_cpu_baseline:
        y_np = y.cpu().numpy()
        omp = oracle.load_openmp()
        for entry, fn, gpu_out in ((e, lambda lib: oracle.minmaxlttb(y_np, n_out, r_ps, _lib_override=lib), got),
                                   (el, lambda lib: oracle.lttb(y_np, n_out, _lib_override=lib),
                                    out_l.cpu().numpy())):
            t_one, want = oracle_seconds(lambda: fn(None))
            t_omp, want_omp = oracle_seconds(lambda: fn(omp))
            entry["parity_vs_oracle"] = bool(np.array_equal(gpu_out, want))
            entry["cpu_oracle_s"] = round(t_one, 5)
            entry["cpu_openmp_s"] = round(t_omp, 5)
            entry["cpu_openmp_identical"] = bool(np.array_equal(want_omp, want))
        res["cpu"] = {"host_cpu": host_cpu_model(), "openmp_threads": oracle.threads(omp),
                      "protocol": "median of 5 runs after one warm-up"}
    res["n1e6"] = {"workload": f"one series, n={n}, float32 random walk (seed 1), implicit x; n_out={n_out}, "
                               f"r_ps={r_ps}; 200 back-to-back calls over 64 copies of it in turn (256 MB)",
                   "minmaxlttb": e, "lttb": el}
    del y, out, ws, out_l, ws_l, copies

    n, n_out, r_ps = int(args.n), 4000, 4
    log(f"shapes: n={n}, n_out={n_out}")
    y = shared_walk(n, args.seed, dev)
    torch.cuda.synchronize()
    out = torch.empty(n_out, dtype=torch.int64, device=dev)
    ws = torch.empty(ops.workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)
    e = timed_calls(lambda: ops.minmaxlttb(y, n_out, r_ps, out=out, ws=ws), 20, "call_minmaxlttb")
    e["gpts_per_s"] = round(n / (e["call_ms"] * 1e-3) / 1e9, 3)
    nb = n_out * r_ps // 2
    mm = e["kernel_avg_ms"].get("minmax_bin_reduce")
    if mm:
        gbs = (4 * n + 16 * nb) / (mm * 1e-3) / 1e9
        e["stream_roofline"] = {"kernel": "minmax_bin_reduce", "algorithmic_bytes": 4 * n + 16 * nb,
                                "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if not args.no_cpu_baseline:
        e["parity_vs_oracle"] = bool(np.array_equal(out.cpu().numpy(), oracle.minmaxlttb(y.cpu().numpy(), n_out,
                                                                                           r_ps)))
    res["n1e9_nout4000"] = {"workload": f"one series, n={n}, float32 random walk (seed {args.seed}), implicit x; "
                                        f"n_out={n_out}, r_ps={r_ps}", "minmaxlttb": e}
    del y, out, ws
    return res


def bench_downsamplers(args, reps: int = 10):
    """The other Table 1 downsamplers on the headline series (n=1e9 float32
    random walk, n_out as the headline): MinMax alone (r_ps = 1), M4 and
    EveryNth. Whole-call and stream-kernel times, the stream kernel's HBM
    roofline fraction, and parity of each output with the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    n, n_out = int(args.n), args.n_out
    dev = torch.device("cuda", 0)
    log(f"downsamplers: generating y, n={n}")
    y = shared_walk(n, args.seed, dev)
    torch.cuda.synchronize()
    y_np = y.cpu().numpy() if not args.no_cpu_baseline else None
    out = torch.empty(max(n_out + 2, 2 * (n_out // 2) + 2), dtype=torch.int64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    res = {}

    def run(name, call, kernel, alg_bytes, want_fn):
        call()
        torch.cuda.synchronize()
        ops.profile_enable(True)
        ops.profile_reset()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        ops.profile_enable(False)
        tot, c = ops.profile_read(kernel)
        k_ms = tot / max(c, 1)
        entry = {"call_ms": round(wall, 5), "kernel": kernel, "kernel_ms": round(k_ms, 5),
                 "gpts_per_s": round(n / (wall * 1e-3) / 1e9, 3)}
        if alg_bytes is not None:
            gbs = alg_bytes / (k_ms * 1e-3) / 1e9
            entry.update({"algorithmic_bytes": alg_bytes, "achieved_GBps": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)})
        if want_fn is not None:
            m = int(cnt.item()) if name != "everynth" else min(n, n_out)
            entry["parity_vs_oracle"] = bool(np.array_equal(out[:m].cpu().numpy(), want_fn()))
        res[name] = entry
        log(f"  {name}: {entry}")

    ws_mm = torch.empty(ops.workspace_size(n, n_out, 1), dtype=torch.uint8, device=dev)
    ws_m4 = torch.empty(ops.m4_workspace_size(n, n_out), dtype=torch.uint8, device=dev)
    nb1, nb4 = n_out // 2, n_out // 4
    run("minmax_r1", lambda: ops.minmax(y, n_out, 1, out=out, count=cnt, ws=ws_mm, sync=False), "minmax_bin_reduce",
        4 * n + 16 * nb1, (lambda: oracle.minmax(y_np, n_out, 1)) if y_np is not None else None)
    run("m4", lambda: ops.m4(y, n_out, out=out, count=cnt, ws=ws_m4, sync=False), "m4_bin_reduce",
        4 * n + 16 * nb4, (lambda: oracle.m4(y_np, n_out)) if y_np is not None else None)
    run("everynth", lambda: ops.everynth(n, n_out, out=out), "everynth", None,
        (lambda: oracle.everynth(n, n_out)) if y_np is not None else None)
    del y, y_np, ws_mm, ws_m4
    return {"workload": f"one series, n={n}, float32 random walk (seed={args.seed}), n_out={n_out}", **res}


def bench_xbins(args, reps: int = 10):
    """MinMaxLTTB with MinMax bins of equal x width on n=1e9 points with
    bursty int64 timestamps (exponential gaps, mean 1000, plus outages of
    1e6-1e9 at 0.1% of the points): call time, the stream kernel's HBM
    roofline fraction (it reads y only: 4 B per point), the edge search, and
    parity with the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    n, n_out, r_ps = int(args.n), args.n_out, args.r_ps
    nb = n_out * r_ps // 2
    dev = torch.device("cuda", 0)
    log(f"xbins: generating y and bursty x, n={n}")
    x = synth.bursty_x(n, args.seed, device=dev)
    y = shared_walk(n, args.seed, dev)
    torch.cuda.synchronize()
    out = torch.empty(n_out, dtype=torch.int64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    ws = torch.empty(ops.xbins_workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)

    def call():
        ops.minmaxlttb_xbins(y, x, n_out, r_ps, out=out, count=cnt, ws=ws, sync=False)

    call()
    torch.cuda.synchronize()
    ops.profile_enable(True)
    ops.profile_reset()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / reps
    ops.profile_enable(False)
    kern = {}
    for k in ("xbin_bounds", "init_keys", "xbin_reduce", "xbin_compact", "lttb_chain_seg", "lttb_chain",
              "xbin_finish"):
        tot, c = ops.profile_read(k)
        kern[k] = round(tot / c, 5) if c else None
    alg = 4 * n + 16 * nb
    gbs = alg / (kern["xbin_reduce"] * 1e-3) / 1e9
    res = {"workload": f"one series, n={n}, float32 random walk, bursty int64 x (seed={args.seed}); "
                       f"MinMaxLTTB n_out={n_out}, r_ps={r_ps}, bins of equal x width",
           "call_ms": round(wall, 5), "gpts_per_s": round(n / (wall * 1e-3) / 1e9, 3), "kernel_avg_ms": kern,
           "stream_roofline": {"kernel": "xbin_reduce", "algorithmic_bytes": alg, "achieved_GBps": round(gbs, 1),
                               "frac": round(gbs / HBM_PEAK_GBS, 4)},
           "count": int(cnt.item())}
    if not args.no_cpu_baseline:
        y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
        c0 = time.perf_counter()
        want = oracle.minmaxlttb_xbins(y_np, x_np, n_out, r_ps)
        res["oracle_s"] = round(time.perf_counter() - c0, 3)
        res["parity_vs_oracle"] = bool(np.array_equal(out[: int(cnt.item())].cpu().numpy(), want))
        del y_np, x_np
    log(f"  xbins: {res}")
    del x, y, ws
    return res


def bench_typed(args, reps: int = 10):
    """MinMaxLTTB on other value types at the headline size (n=1e9, n_out and
    r_ps as the headline): float64 y with float64 timestamps, and int32 y with
    implicit x. Call and stream-kernel times, the stream's HBM roofline
    fraction (it reads y once: 8 or 4 B per point), parity with the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    n, n_out, r_ps = int(args.n), args.n_out, args.r_ps
    dev = torch.device("cuda", 0)
    res = {}
    for name, make_y, make_x, ybytes in [
        ("f64_y_f64_x", lambda: synth.random_walk(n, args.seed, device=dev, dtype=torch.float64),
         lambda: synth.float_x(n, args.seed, device=dev), 8),
        ("i32_y", lambda: synth.int_series(n, args.seed, device=dev), lambda: None, 4),
    ]:
        log(f"typed: {name}, n={n}, tuning {ops.get_tuning()}")
        y, x = make_y(), make_x()
        torch.cuda.synchronize()
        out = torch.empty(n_out, dtype=torch.int64, device=dev)
        ws = torch.empty(ops.typed_workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)

        def call():
            ops.minmaxlttb_typed(y, n_out, r_ps, x=x, out=out, ws=ws)

        call()
        torch.cuda.synchronize()
        ops.profile_enable(True)
        ops.profile_reset()
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        ops.profile_enable(False)
        kern = {}
        for k in ("typed_bin_reduce", "typed_bin_merge", "typed_compact", "typed_bucket_means", "lttb_chain_seg",
                  "lttb_chain"):
            tot, c = ops.profile_read(k)
            kern[k] = round(tot / c, 5) if c else None
        alg = ybytes * n
        gbs = alg / (kern["typed_bin_reduce"] * 1e-3) / 1e9
        entry = {"call_ms": round(wall, 5), "gpts_per_s": round(n / (wall * 1e-3) / 1e9, 3), "kernel_avg_ms": kern,
                 "tuning": ops.get_tuning()._asdict(),
                 "stream_roofline": {"kernel": "typed_bin_reduce", "algorithmic_bytes": alg,
                                     "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        if not args.no_cpu_baseline:
            y_np = y.cpu().numpy()
            x_np = None if x is None else x.cpu().numpy()
            c0 = time.perf_counter()
            want = oracle.minmaxlttb_typed(y_np, n_out, r_ps, x_np)
            entry["oracle_s"] = round(time.perf_counter() - c0, 3)
            entry["parity_vs_oracle"] = bool(np.array_equal(out.cpu().numpy(), want))
            del y_np, x_np
        log(f"  {name}: {entry}")
        res[name] = entry
        del y, x, ws
    res["workload"] = (f"one series, n={n}: float64 random walk with float64 second timestamps, and int32 counts "
                       f"with implicit x (seed={args.seed}); MinMaxLTTB n_out={n_out}, r_ps={r_ps}")
    return res


def bench_simplifiers(args, reps: int = 10):
    """MinMax preselection followed by Visvalingam-Whyatt, Douglas-Peucker or
    Longest-Line-Bucket instead of LTTB, on the headline series (n=1e9,
    n_out and r_ps as the headline): call time, the simplifier kernels' time
    on the preselected points (VW and LLB: one wave; DP: the split tree in one
    workgroup, then the greedy loop's gated launch), parity with the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    n, n_out, r_ps = int(args.n), args.n_out, args.r_ps
    dev = torch.device("cuda", 0)
    log(f"simplifiers: generating y, n={n}")
    y = shared_walk(n, args.seed, dev)
    torch.cuda.synchronize()
    y_np = None if args.no_cpu_baseline else y.cpu().numpy()
    out = torch.empty(n_out, dtype=torch.int64, device=dev)
    ws = torch.empty(ops.simplify_workspace_size(n, n_out, r_ps), dtype=torch.uint8, device=dev)
    res = {"workload": f"one series, n={n}, float32 random walk (seed={args.seed}), implicit x; n_out={n_out}, "
                       f"r_ps={r_ps} ({2 * (n_out * r_ps // 2) + 2} preselected points)"}
    for alg in ("vw", "dp", "llb"):
        ops.minmax_simplify(alg, y, n_out, r_ps, out=out, ws=ws)
        torch.cuda.synchronize()
        ops.profile_enable(True)
        ops.profile_reset()
        t0 = time.perf_counter()
        for _ in range(reps):
            ops.minmax_simplify(alg, y, n_out, r_ps, out=out, ws=ws)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / reps
        ops.profile_enable(False)
        tot, c = ops.profile_read(f"simplify_{alg}")
        mm, cm = ops.profile_read("minmax_bin_reduce")
        entry = {"call_ms": round(wall, 5), "gpts_per_s": round(n / (wall * 1e-3) / 1e9, 3),
                 "simplify_kernel_ms": round(tot / max(c, 1), 5), "stream_kernel_ms": round(mm / max(cm, 1), 5)}
        if y_np is not None:
            c0 = time.perf_counter()
            want = oracle.minmax_simplify(alg, y_np, n_out, r_ps)
            entry["oracle_s"] = round(time.perf_counter() - c0, 3)
            entry["parity_vs_oracle"] = bool(np.array_equal(out.cpu().numpy(), want))
        log(f"  {alg}: {entry}")
        res[alg] = entry
    del y, y_np, ws
    return res


def bench_comparator(args):
    """Whole-series LTTB vs MinMaxLTTB on one 1e8-point series (random walk +
    sinusoids + noise + spikes, int64 irregular timestamps), n_out=2000: GPU
    times for both, and the oracle's single-thread CPU times for both (the
    paper's comparison, section 3.2), every output checked against the oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2305_00332_amd import ops, synth

    n, n_out = 100_000_000, 2000
    log(f"comparator: generating {n} points")
    x, y = synth.composite_series(n, 2, device="cuda")
    torch.cuda.synchronize()
    y_np, x_np = y.cpu().numpy(), x.cpu().numpy()
    input_sha256 = {"y": hashlib.sha256(memoryview(y_np).cast("B")).hexdigest(),
                    "x": hashlib.sha256(memoryview(x_np).cast("B")).hexdigest()}

    def gpu_time(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out

    omp = oracle.load_openmp()
    res = {"workload": f"one series, n={n}, float32 random walk + 3 sinusoids + noise + 0.01% spikes (seed 2), "
                       f"int64 irregular x; n_out={n_out}", "n": n, "n_out": n_out,
           "cpu_openmp_threads": oracle.threads(omp), "input_sha256": input_sha256}
    log("comparator: GPU whole-series LTTB")
    t_l, out_l = gpu_time(lambda: ops.lttb(y, n_out, x=x), 3)
    c0 = time.perf_counter()
    want_l = oracle.lttb(y_np, n_out, x_np)
    t_lc = time.perf_counter() - c0
    ops.profile_enable(True)
    ops.profile_reset()
    ops.lttb(y, n_out, x=x)
    torch.cuda.synchronize()
    ops.profile_enable(False)
    k_l = {}
    for k in ("lttb_scan", "bucket_mean_wide", "lttb_hull", "lttb_tables", "lttb_table_walk"):
        tot, cnt = ops.profile_read(k)
        if cnt:
            k_l[k] = round(tot / cnt, 4)
    old = ops.get_tuning()
    ops.set_tuning(0, 0, ops.CHAIN_SEQUENTIAL)
    t_seq, out_seq = gpu_time(lambda: ops.lttb(y, n_out, x=x), 1)
    ops.set_tuning(*old)
    res["lttb"] = {"gpu_ms": round(t_l * 1e3, 4), "gpu_gpts_per_s": round(n / t_l / 1e9, 3),
                   "kernel_ms": k_l, "form": "transition tables over hull candidates",
                   "sequential_form_ms": round(t_seq * 1e3, 3),
                   "sequential_form_identical": bool(torch.equal(out_seq, out_l)),
                   "cpu_oracle_s": round(t_lc, 3), "parity_vs_oracle": bool(np.array_equal(out_l.cpu().numpy(), want_l))}
    for r_ps in (2, 4, 8):
        log(f"comparator: MinMaxLTTB r_ps={r_ps}")
        t_m, out_m = gpu_time(lambda: ops.minmaxlttb(y, n_out, r_ps, x=x), 10)
        c0 = time.perf_counter()
        want_m = oracle.minmaxlttb(y_np, n_out, r_ps, x_np)
        t_mc = time.perf_counter() - c0
        c0 = time.perf_counter()
        want_omp = oracle.minmaxlttb(y_np, n_out, r_ps, x_np, _lib_override=omp)
        t_mo = time.perf_counter() - c0
        res[f"minmaxlttb_r{r_ps}"] = {
            "gpu_ms": round(t_m * 1e3, 4), "gpu_gpts_per_s": round(n / t_m / 1e9, 3), "cpu_oracle_s": round(t_mc, 3),
            "cpu_openmp_s": round(t_mo, 3),
            "gpu_speedup_vs_gpu_lttb": round(t_l / t_m, 2), "cpu_speedup_vs_cpu_lttb": round(t_lc / t_mc, 2),
            "cpu_openmp_speedup_vs_cpu_lttb": round(t_lc / t_mo, 2),
            "parity_vs_oracle": bool(np.array_equal(out_m.cpu().numpy(), want_m) and np.array_equal(want_omp, want_m))}
    del x, y, y_np, x_np
    res["paper_context"] = {
        "serial_speedup_vs_lttb": "about 10x",
        "parallel_speedup_vs_lttb": "30x",
        "source": "section 3.2: CPU implementations (a C LTTB, tsdownsample's MinMaxLTTB); hardware, core "
                  "count, N, n_out and r_ps are not stated",
        "here": "cpu_speedup_vs_cpu_lttb compares the two single-thread oracle runs; "
                "cpu_openmp_speedup_vs_cpu_lttb the oracle built with OpenMP over the MinMax bins (all host "
                "threads) against the single-thread LTTB oracle; gpu_speedup_vs_gpu_lttb the two GPU paths",
    }
    return res


def bench_batched(args):
    """Many series of uneven length: one batched call vs one call per series."""
    import numpy as np
    import torch

    from paper_2305_00332_amd import ops, synth

    count = args.batch_series
    lengths = synth.batch_lengths(count, 1e3, 1e7, 4)
    n_outs = synth.choice([200, 500, 1000, 2000], count, 40)
    log(f"batched: generating {count} series, {int(lengths.sum())} points")
    x, y, offsets = synth.batch_series(lengths, 4, device="cuda")
    torch.cuda.synchronize()
    segs = [(int(o), int(n), int(no), 4) for o, n, no in zip(offsets, lengths, n_outs)]
    table = ops.segment_table(segs)
    out = torch.empty(max(table[2], 1), dtype=torch.int64, device="cuda")
    ws = torch.empty(ops.batched_workspace_size(segs), dtype=torch.uint8, device="cuda")
    for _ in range(2):
        ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table)
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / reps
    ops.profile_enable(True)
    ops.profile_reset()
    ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table)
    torch.cuda.synchronize()
    ops.profile_enable(False)
    kern = {}
    for k in ("batch_init", "batch_minmax_large", "batch_minmax_small", "batch_compact", "batch_means",
              "batch_chain", "batch_chain_seq", "batch_link_emit"):
        tot, cnt = ops.profile_read(k)
        if cnt:
            kern[k] = round(tot / cnt, 4)
    # the same batch replayed from a captured graph (a dashboard refreshing the same series)
    gstream = torch.cuda.Stream()
    ops.set_graph_cache(2)
    with torch.cuda.stream(gstream):
        for _ in range(2):
            ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table)
    gstream.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(gstream):
        for _ in range(reps):
            ops.minmaxlttb_batched(y, segs, x_base=x, out=out, ws=ws, table=table)
    gstream.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    graph_stats = ops.graph_cache_stats()
    ops.set_graph_cache(0)
    # a serving-sized batch of 16 series: eager vs graph replay
    small = segs[:16]
    small_table = ops.segment_table(small)
    small_out = torch.empty(max(small_table[2], 1), dtype=torch.int64, device="cuda")
    small_ws = torch.empty(ops.batched_workspace_size(small), dtype=torch.uint8, device="cuda")

    def time_small(graph):
        ops.set_graph_cache(2 if graph else 0)
        with torch.cuda.stream(gstream):
            for _ in range(3):
                ops.minmaxlttb_batched(y, small, x_base=x, out=small_out, ws=small_ws, table=small_table)
        gstream.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(gstream):
            for _ in range(50):
                ops.minmaxlttb_batched(y, small, x_base=x, out=small_out, ws=small_ws, table=small_table)
        gstream.synchronize()
        ops.set_graph_cache(0)
        return (time.perf_counter() - t0) / 50

    t_small_eager, t_small_graph = time_small(False), time_small(True)
    log("batched: plain per-series calls")
    plain = torch.empty_like(out)
    ws1 = torch.empty(max(ops.workspace_size(1, no, 4) for no in (200, 500, 1000, 2000)), dtype=torch.uint8,
                      device="cuda")
    outoff = table[1]

    def run_plain():
        for i, (o, n, no, r) in enumerate(segs):
            k = min(n, no)
            ops.minmaxlttb(y[o: o + n], no, r, x=x[o: o + n], out=plain[outoff[i]: outoff[i] + k], ws=ws1)

    run_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # the same per-series calls again, each bracketed by the library's events:
    # their summed device spans (the plain form's device time without host gaps)
    ops.profile_enable(True)
    ops.profile_reset()
    run_plain()
    torch.cuda.synchronize()
    ops.profile_enable(False)
    plain_spans = ops.profile_samples("call_minmaxlttb")
    # the plain form's kernels alone: the sum of every launch's own event-timed
    # duration (no host gaps inside or between calls)
    plain_kernel_ms = sum(ops.profile_read(k)[0] for k in (
        "iota", "init_keys", "minmax_bin_reduce", "preselect_tail", "preselect_all", "preselect_compact_means",
        "preselect_compact", "bucket_mean", "lttb_chain", "lttb_chain_seg"))
    pts = int(lengths.sum())
    res = {"workload": f"{count} series, lengths log-uniform in [1e3, 1e7] (seed 4), float32 random walk + "
                       f"N(0, 0.5^2), int64 irregular x; n_out in {{200, 500, 1000, 2000}}, r_ps=4",
           "points": pts, "ms": round(t_batched * 1e3, 4), "gpts_per_s": round(pts / t_batched / 1e9, 3),
           "plain_ms": round(t_plain * 1e3, 4), "plain_gpts_per_s": round(pts / t_plain / 1e9, 3),
           "speedup_vs_plain": round(t_plain / t_batched, 3),
           "plain_device_ms": round(float(sum(plain_spans)), 4) if len(plain_spans) == len(segs) else None,
           "plain_device_ms_note": "summed call spans, with every launch bracketed by timing events (the host's "
                                   "launch gaps inside a call included)",
           "plain_kernel_ms": round(plain_kernel_ms, 4),
           "plain_kernel_ms_note": "sum of every launch's event-timed duration (the events add a few us per launch)",
           "speedup_vs_plain_kernels": round(plain_kernel_ms / (t_batched * 1e3), 3),
           "kernel_ms": kern,
           "tuning": ops.get_tuning()._asdict(),
           "graph_replay_ms": round(t_graph * 1e3, 4), "graph_stats": list(graph_stats),
           "small_batch_16": {"eager_ms": round(t_small_eager * 1e3, 4), "graph_ms": round(t_small_graph * 1e3, 4),
                              "points": int(sum(n for _, n, _, _ in small))},
           "identical_to_plain": bool(torch.equal(out[: table[2]], plain[: table[2]]))}
    if not args.no_cpu_baseline:
        res.update(batched_oracle(args, x, y, segs, out, table[1]))
    del x, y, out, plain, ws, ws1
    return res


def batched_oracle(args, x, y, segs, out, outoff):
    """Every series of the batch through the oracle on the host: parity with
    the batched output, and the oracle's time single-threaded, in its OpenMP
    build (bins of each series across threads), and single-threaded builds on
    a pool of threads over the series."""
    import numpy as np

    import oracle

    log("batched: copying the batch to the host for the oracle")
    y_h, x_h = y.cpu().numpy(), x.cpu().numpy()
    got = out.cpu().numpy()

    def fetch(lo, hi):
        return y_h[lo:hi], x_h[lo:hi]

    omp = oracle.load_openmp()
    workers = min(16, os.cpu_count() or 1)
    log("batched: oracle, single thread")
    t0 = time.perf_counter()
    want = oracle.minmaxlttb_segments(fetch, segs, workers=1, slab_points=1 << 40)
    t_one = time.perf_counter() - t0
    log("batched: oracle, OpenMP build")
    t0 = time.perf_counter()
    want_omp = oracle.minmaxlttb_segments(fetch, segs, workers=1, slab_points=1 << 40, _lib_override=omp)
    t_omp = time.perf_counter() - t0
    log(f"batched: oracle, {workers} threads over the series")
    t0 = time.perf_counter()
    want_par = oracle.minmaxlttb_segments(fetch, segs, workers=workers, slab_points=1 << 40)
    t_par = time.perf_counter() - t0
    bad = [i for i, (o, n, no, r) in enumerate(segs)
           if not np.array_equal(got[outoff[i]: outoff[i] + min(n, no)], want[i])]
    pts = sum(n for _, n, _, _ in segs)
    return {"parity_vs_oracle": not bad, "oracle_mismatches": len(bad),
            "cpu_oracle_s": round(t_one, 3), "cpu_openmp_s": round(t_omp, 3),
            "cpu_series_parallel_s": round(t_par, 3), "cpu_series_parallel_threads": workers,
            "cpu_oracle_gpts_per_s": round(pts / t_one / 1e9, 4),
            "cpu_identical": bool(all(np.array_equal(a, b) and np.array_equal(a, c)
                                      for a, b, c in zip(want, want_omp, want_par))),
            "cpu_host": host_cpu_model(), "cpu_openmp_threads": oracle.threads(omp),
            "cpu_sample": f"all {len(segs)} series, each its own oracle call, inputs already in host memory"}


def bench_served(args):
    """Poisson request streams against a resident pool: continuous batching
    vs one single-series call per request, p50/p99 latency, Gpts/s and the
    fraction of the run with work on the device; every result of the two forms
    compared, and a seeded sample of requests compared with the oracle (which
    is also timed on that sample)."""
    import numpy as np
    import torch

    from paper_2305_00332_amd import synth
    from paper_2305_00332_amd.serve import GpuExecutor, PlainGpuExecutor, Scheduler, latency_summary, \
        poisson_requests

    count = args.pool_series
    lengths = synth.batch_lengths(count, 1e4, 1e8, 5)
    log(f"served: generating pool of {count} series, {int(lengths.sum())} points")
    x, y, offsets = synth.batch_series(lengths, 5, device="cuda", sinusoids=True)
    torch.cuda.synchronize()
    rates = [float(r) for r in args.rates.split(",") if r]
    slots = 4
    forms = {"batched": (GpuExecutor(y, offsets, lengths, x=x, n_slots=slots, arena_bytes=args.serve_arena), None),
             "plain": (PlainGpuExecutor(y, offsets, lengths, x=x, n_slots=slots, arena_bytes=args.serve_arena), 1)}

    def serve(name, reqs, max_batch=None):
        ex, mb = forms[name]
        sched = Scheduler(ex, n_slots=slots, max_batch=max_batch if max_batch is not None else mb)
        fresh = [type(r)(r.rid, r.series, r.lo, r.hi, r.n_out, r.r_ps, r.arrival) for r in reqs]
        done = sched.run_open_loop(fresh, timeout=900)
        s = latency_summary(done)
        s["busy_frac"] = round(sched.busy_fraction(s.get("span_s", 0.0)), 4)
        s["steps"] = sched.steps_launched
        s["mean_batch"] = round(float(np.mean(sched.batch_sizes)), 2) if sched.batch_sizes else 0.0
        s["max_in_flight"] = sched.max_in_flight
        s["max_device_bytes"] = sched.max_ws_in_use
        return s, done

    def same(a, b):
        """Every request succeeded in both forms with equal indices."""
        ra, rb = {r.rid: r for r in a}, {r.rid: r for r in b}
        return ra.keys() == rb.keys() and all(
            ra[k].error is None and rb[k].error is None and np.array_equal(ra[k].result, rb[k].result) for k in ra)

    def combine(parts):
        """One summary of a form's runs over consecutive chunks of a stream."""
        done = [r for _, d in parts for r in d]
        ok = [r for r in done if r.error is None]
        lat = np.array([r.latency for r in ok], dtype=np.float64) * 1e3
        span = sum(sm["span_s"] for sm, _ in parts)
        steps = sum(sm["steps"] for sm, _ in parts)
        out = {"requests": len(ok), "errors": len(done) - len(ok)}
        if lat.size:
            out.update({"p50_ms": round(float(np.percentile(lat, 50)), 4),
                        "p99_ms": round(float(np.percentile(lat, 99)), 4),
                        "mean_ms": round(float(lat.mean()), 4),
                        "gpts_per_s": round(sum(r.n for r in ok) / max(span, 1e-9) / 1e9, 3)})
        out.update({"span_s": round(span, 4),
                    "busy_frac": round(sum(sm["busy_frac"] * sm["span_s"] for sm, _ in parts) / max(span, 1e-9), 4),
                    "steps": steps, "mean_batch": round(len(done) / max(steps, 1), 2),
                    "max_in_flight": max(sm["max_in_flight"] for sm, _ in parts),
                    "max_device_bytes": max(sm["max_device_bytes"] for sm, _ in parts)})
        return out, done

    per_rate = {}
    identical = True
    chunks = max(1, args.serve_chunks)
    for rate in rates:
        n_req = max(args.serve_min_requests, int(rate * args.serve_seconds))
        reqs = poisson_requests(rate, n_req, lengths, seed=50 + int(rate))
        warm = poisson_requests(rate, 50, lengths, seed=7)
        for name in forms:
            serve(name, warm)
        # the stream in consecutive chunks, each served by both forms in
        # alternating order, so drift in the machine's state falls on both
        runs = {name: [] for name in forms}
        for c, idx in enumerate(np.array_split(np.arange(n_req), chunks)):
            if idx.size == 0:
                continue
            t0 = reqs[idx[0]].arrival
            sub = [type(r)(r.rid, r.series, r.lo, r.hi, r.n_out, r.r_ps, r.arrival - t0) for r in (reqs[i] for i in idx)]
            for name in (list(forms) if c % 2 == 0 else list(forms)[::-1]):
                log(f"served: rate {rate:g}/s, chunk {c + 1}/{chunks} ({idx.size} requests), {name}")
                runs[name].append(serve(name, sub))
        entry, results = {}, {}
        for name in forms:
            entry[name], results[name] = combine(runs[name])
        entry["interleaved_chunks"] = chunks
        identical = identical and same(results["batched"], results["plain"])
        b, p = entry["batched"], entry["plain"]
        entry["p99_ratio_plain_over_batched"] = round(p["p99_ms"] / b["p99_ms"], 3) if b.get("p99_ms") else None
        entry["throughput_ratio_vs_plain"] = (round(b["gpts_per_s"] / p["gpts_per_s"], 3)
                                              if p.get("gpts_per_s") else None)
        per_rate[f"{rate:g}"] = entry
    # saturation: a burst of requests all arriving at t=0, served to completion
    burst = poisson_requests(1e12, args.burst, lengths, seed=77)
    burst_entry, burst_results = {}, {}
    for name in forms:
        serve(name, burst[:64], max_batch=256 if name == "batched" else None)
        log(f"served: burst of {args.burst} requests, {name}")
        burst_entry[name], burst_results[name] = serve(name, burst, max_batch=256 if name == "batched" else None)
    identical = identical and same(burst_results["batched"], burst_results["plain"])
    burst_entry["throughput_ratio_vs_plain"] = round(burst_entry["batched"]["gpts_per_s"] /
                                                     burst_entry["plain"]["gpts_per_s"], 3)
    errors = sum(e[k]["errors"] for e in per_rate.values() for k in ("batched", "plain")) + \
        sum(burst_entry[k]["errors"] for k in ("batched", "plain"))
    res = {"workload": f"pool of {count} series resident in HBM, lengths log-uniform in [1e4, 1e8] (seed 5), "
                       f"float32 random walk + sinusoids + noise, int64 irregular x; Poisson arrivals; per request "
                       f"a series, a log-uniform sub-range, n_out uniform in [100, 4000], r_ps in {{2, 4}}",
           "pool_points": int(lengths.sum()), "slots": slots, "arena_bytes_per_form": args.serve_arena,
           "requests_per_rate": f"max({args.serve_min_requests}, {args.serve_seconds:g} s x rate)",
           "rates": per_rate, "burst": burst_entry, "errors": errors,
           "identical_to_plain": bool(identical and errors == 0)}
    if not args.no_cpu_baseline:
        res.update(served_oracle(x, y, offsets, burst_results["batched"], args.serve_oracle_sample))
    del forms, x, y
    return res


def served_oracle(x, y, offsets, done, sample):
    """A seeded sample of served requests (from the burst, so most ran inside
    batched steps) through the oracle: parity, and its time single-threaded and
    in the OpenMP build on that sample."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(2024)
    pick = sorted(rng.choice(len(done), size=min(sample, len(done)), replace=False).tolist())
    reqs = [done[i] for i in pick]
    segs = [(int(offsets[r.series]) + r.lo, r.n, r.n_out, r.r_ps) for r in reqs]
    log(f"served: copying {len(segs)} sampled sub-ranges to the host for the oracle")
    host = {}
    for o, n, _, _ in segs:
        if o not in host or host[o][0].shape[0] < n:
            host[o] = (y[o: o + n].cpu().numpy(), x[o: o + n].cpu().numpy())

    def fetch(lo, hi):
        ys, xs = host[lo]
        return ys[: hi - lo], xs[: hi - lo]

    omp = oracle.load_openmp()
    log("served: oracle on the sample, single thread")
    t0 = time.perf_counter()
    want = oracle.minmaxlttb_segments(fetch, segs, workers=1, slab_points=0)
    t_one = time.perf_counter() - t0
    log("served: oracle on the sample, OpenMP build")
    t0 = time.perf_counter()
    want_omp = oracle.minmaxlttb_segments(fetch, segs, workers=1, slab_points=0, _lib_override=omp)
    t_omp = time.perf_counter() - t0
    bad = [r.rid for r, w in zip(reqs, want) if r.error is not None or not np.array_equal(r.result, w)]
    pts = sum(r.n for r in reqs)
    return {"parity_vs_oracle": not bad, "oracle_mismatches": len(bad),
            "oracle_sample": {"requests": len(reqs), "points": int(pts),
                              "above_1e7_points": sum(1 for r in reqs if r.n > 10 ** 7),
                              "in_batched_steps": sum(1 for r in reqs if r.batch > 1),
                              "how": "seeded sample of the burst's requests (batched form), each sub-range "
                                     "through the oracle alone"},
            "cpu_oracle_s": round(t_one, 3), "cpu_openmp_s": round(t_omp, 3),
            "cpu_oracle_gpts_per_s": round(pts / t_one / 1e9, 4), "cpu_openmp_gpts_per_s": round(pts / t_omp / 1e9, 4),
            "cpu_identical": bool(all(np.array_equal(a, b) for a, b in zip(want, want_omp))),
            "cpu_host": host_cpu_model(), "cpu_openmp_threads": oracle.threads(omp)}


if __name__ == "__main__":
    main()
