"""Continuous-batching downsampling server over a device-resident series pool.

A request asks for MinMaxLTTB of one pool series' sub-range [lo, hi) with its
own n_out and r_ps. The scheduler keeps a FIFO of arrived requests and, on
every tick:
  1. completes steps whose device work has finished (indices land in pinned
     host memory; workspace bytes and the slot are released);
  2. while a slot (an in-flight step, each on its own HIP stream) is free,
     admits requests from the head of the queue as long as their workspace
     fits the remaining budget, and launches them as ONE batched call.
Requests that arrive while other steps run are admitted as soon as a slot
and memory free up, and steps overlap on the device. A request whose
arguments are invalid fails alone (checked on submit); one that can never fit
the budget fails alone; an executor failure fails the requests of that step
only and the server keeps serving.

The scheduler is plain host logic over an Executor (launch / poll / collect);
GpuExecutor runs the batched library call, PlainGpuExecutor one single-series
call per request (the comparator).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib


@dataclass
class Request:
    rid: int
    series: int
    lo: int
    hi: int
    n_out: int
    r_ps: int
    arrival: float = 0.0  # scheduled arrival, seconds from the run's start
    admitted: float | None = None
    done: float | None = None
    result: np.ndarray | None = None
    error: str | None = None

    @property
    def n(self) -> int:
        return self.hi - self.lo

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


def validate(req: Request, series_len: int) -> str | None:
    """Host-side argument check with the library's rules (one request alone)."""
    n = req.hi - req.lo
    if req.lo < 0 or req.hi > series_len or n < 1:
        return f"sub-range [{req.lo}, {req.hi}) is empty or outside the series (length {series_len})"
    if not (3 <= req.n_out <= 2 ** 31 - 1):
        return f"n_out must be in [3, 2^31-1], got {req.n_out}"
    if req.r_ps < 2:
        return f"r_ps must be >= 2, got {req.r_ps}"
    nb = req.n_out * req.r_ps // 2
    if nb > 2 ** 31 - 1:
        return "floor(n_out*r_ps/2) must be <= 2^31-1"
    if n > 2:
        L = n - 2
        nbe = min(nb, L)
        if -(-L // nbe) >= 2 ** 32:
            return "MinMax bins exceed 2^32-1 points"
    return None


@dataclass
class Step:
    slot: int
    reqs: list
    ws_bytes: int
    handle: object = None


class Scheduler:
    def __init__(self, executor, n_slots: int = 2, ws_budget: int = 256 << 20, max_batch: int | None = None,
                 clock=time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        self.ws_budget = ws_budget
        self.max_batch = max_batch
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.free_slots = list(range(n_slots))
        self.in_flight: list[Step] = []
        self.ws_in_use = 0
        self.t0 = None
        self.completed: list[Request] = []
        self.steps_launched = 0
        self.max_in_flight = 0
        self.batch_sizes: list[int] = []

    def now(self) -> float:
        return self.clock() - self.t0

    def start(self):
        self.t0 = self.clock()

    def submit(self, req: Request):
        err = validate(req, self.ex.series_len(req.series))
        if err is None and self.ex.request_ws(req) > self.ws_budget:
            err = f"request needs {self.ex.request_ws(req)} workspace bytes, above the whole budget {self.ws_budget}"
        if err is not None:
            req.error = err
            req.done = self.now()
            self.completed.append(req)
            return
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        """Drop a request that is still queued (not yet admitted)."""
        for r in self.queue:
            if r.rid == rid:
                self.queue.remove(r)
                r.error = "cancelled"
                r.done = self.now()
                self.completed.append(r)
                return True
        return False

    def _complete(self):
        still = []
        for st in self.in_flight:
            if self.ex.poll(st.handle):
                t = self.now()
                try:
                    results = self.ex.collect(st.handle)
                    for r, res in zip(st.reqs, results):
                        r.result = res
                except Exception as e:  # the step failed: its requests fail, serving goes on
                    for r in st.reqs:
                        r.error = f"step failed: {e}"
                for r in st.reqs:
                    r.done = t
                    self.completed.append(r)
                self.ws_in_use -= st.ws_bytes
                self.free_slots.append(st.slot)
            else:
                still.append(st)
        self.in_flight = still

    def _admit(self):
        while self.free_slots and self.queue:
            batch, ws = [], 0
            while self.queue:
                r = self.queue[0]
                need = self.ex.request_ws(r)
                if self.ws_in_use + ws + need > self.ws_budget:
                    break
                if self.max_batch is not None and len(batch) >= self.max_batch:
                    break
                batch.append(self.queue.popleft())
                ws += need
            if not batch:
                return  # head does not fit until memory frees up
            slot = self.free_slots.pop(0)
            t = self.now()
            for r in batch:
                r.admitted = t
            st = Step(slot=slot, reqs=batch, ws_bytes=ws)
            try:
                st.handle = self.ex.launch(batch, slot)
            except Exception as e:
                for r in batch:
                    r.error = f"launch failed: {e}"
                    r.done = self.now()
                    self.completed.append(r)
                self.free_slots.append(slot)
                continue
            self.ws_in_use += ws
            self.in_flight.append(st)
            self.steps_launched += 1
            self.batch_sizes.append(len(batch))
            self.max_in_flight = max(self.max_in_flight, len(self.in_flight))

    def tick(self):
        self._complete()
        self._admit()

    def idle(self) -> bool:
        return not self.queue and not self.in_flight

    def run_open_loop(self, requests, timeout: float = 600.0):
        """Submit each request at its scheduled arrival time (seconds from start)
        and serve until all complete. Returns the completed requests."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        self.start()
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.now()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self.tick()
            if now > timeout:
                raise TimeoutError("serving run exceeded its time limit")
        return self.completed


def latency_summary(reqs) -> dict:
    lat = np.array([r.latency for r in reqs if r.error is None], dtype=np.float64) * 1e3
    pts = sum(r.n for r in reqs if r.error is None)
    if lat.size == 0:
        return {"requests": 0}
    first = min(r.arrival for r in reqs)
    last = max(r.done for r in reqs if r.done is not None)
    span = max(last - first, 1e-9)
    return {
        "requests": int(lat.size),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "mean_ms": round(float(lat.mean()), 4),
        "gpts_per_s": round(pts / span / 1e9, 3),
        "span_s": round(span, 4),
        "errors": sum(1 for r in reqs if r.error is not None),
    }


def poisson_requests(rate: float, count: int, pool_lengths, seed: int, n_out_range=(100, 4000), r_ps_choices=(2, 4),
                     min_len: int = 10_000):
    """Open-loop Poisson arrivals; each request picks a series, a sub-range of
    log-uniform length in [min(min_len, len), len] at a uniform start, n_out
    uniform in n_out_range, r_ps from r_ps_choices."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        s = int(rng.integers(0, len(pool_lengths)))
        L = int(pool_lengths[s])
        lo_len = min(min_len, L)
        n = int(math.floor(math.exp(rng.uniform(math.log(lo_len), math.log(L))))) if L > lo_len else L
        n = max(1, min(n, L))
        start = int(rng.integers(0, L - n + 1))
        n_out = int(rng.integers(n_out_range[0], n_out_range[1] + 1))
        r_ps = int(rng.choice(r_ps_choices))
        out.append(Request(rid=i, series=s, lo=start, hi=start + n, n_out=n_out, r_ps=r_ps, arrival=float(arrivals[i])))
    return out


# ------------------------------------------------------------------ executors

class GpuExecutor:
    """Runs each admitted set of requests as one batched call on the slot's
    stream (a set of one takes the single-series call, which launches fewer
    kernels and gives the same indices), then copies the indices to pinned
    host memory on that stream."""

    def __init__(self, y, offsets, lengths, x=None, n_slots: int = 2):
        import torch

        self.torch = torch
        self.y, self.x = y, x
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.lengths = np.asarray(lengths, dtype=np.int64)
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self._ws_cache = {}

    def series_len(self, s: int) -> int:
        return int(self.lengths[s])

    def request_ws(self, r: Request) -> int:
        key = (r.n_out, r.r_ps)
        v = self._ws_cache.get(key)
        if v is None:
            v = int(_lib.load().mmlttb_workspace_size(1, r.n_out, r.r_ps))
            self._ws_cache[key] = v
        return v

    def launch(self, reqs, slot):
        from .ops import minmaxlttb_batched, segment_table

        if len(reqs) == 1:
            return PlainGpuExecutor.launch(self, reqs, slot)
        torch = self.torch
        segs = [(int(self.offsets[r.series]) + r.lo, r.n, r.n_out, r.r_ps) for r in reqs]
        table = segment_table(segs)
        stream = self.streams[slot]
        with torch.cuda.stream(stream):
            out, outoff = minmaxlttb_batched(self.y, segs, x_base=self.x, table=table)
            host = torch.empty(out.numel(), dtype=torch.int64, pin_memory=True)
            host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, host, outoff, [min(r.n, r.n_out) for r in reqs], out)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle):
        _, host, outoff, counts, _ = handle
        h = host.numpy()
        return [h[o: o + c].copy() for o, c in zip(outoff, counts)]


class PlainGpuExecutor(GpuExecutor):
    """Comparator: one single-series call per request, in arrival order."""

    def launch(self, reqs, slot):
        from .ops import minmaxlttb

        torch = self.torch
        stream = self.streams[slot]
        outs = []
        with torch.cuda.stream(stream):
            for r in reqs:
                o = int(self.offsets[r.series]) + r.lo
                xs = None if self.x is None else self.x[o: o + r.n]
                outs.append(minmaxlttb(self.y[o: o + r.n], r.n_out, r.r_ps, x=xs))
            cat = torch.cat(outs) if len(outs) > 1 else outs[0]
            host = torch.empty(cat.numel(), dtype=torch.int64, pin_memory=True)
            host.copy_(cat, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        counts = [min(r.n, r.n_out) for r in reqs]
        offs = list(np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(int))
        return (ev, host, offs, counts, outs)
