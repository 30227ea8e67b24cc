"""Continuous-batching downsampling server over a device-resident series pool.

A request asks for MinMaxLTTB of one pool series' sub-range [lo, hi) with its
own n_out and r_ps. The scheduler keeps a FIFO of arrived requests and, on
every tick:
  1. completes steps whose device work has finished (indices land in pinned
     host memory; the step's device memory and slot are released);
  2. while a slot (an in-flight step, each on its own HIP stream) is free,
     admits requests from the head of the queue, spread over the free slots
     (a step takes ceil(queued / free slots) of them, so a lightly loaded
     server runs each request alone and batches form once slots are busy),
     reserves the step's exact device memory (workspace and output) from the
     executor, and launches the requests as ONE batched call.
Requests that arrive while other steps run are admitted as soon as a slot
and memory free up, and steps overlap on the device. A request whose
arguments are invalid fails alone (checked on submit); one that can never fit
the memory budget fails alone; an executor failure fails the requests of that
step only and the server keeps serving.

The scheduler is plain host logic over an Executor (reserve / launch / poll /
collect / release); GpuExecutor runs the batched library call with its
workspace and output carved out of one device arena allocated up front (the
budget is the arena: serving allocates no other device memory), and
PlainGpuExecutor one single-series call per request (the comparator).
"""
from __future__ import annotations

import collections
import ctypes
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
    batch: int = 0  # requests in the step that served it

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
    token: object = None
    handle: object = None
    launched: float = 0.0


class Scheduler:
    def __init__(self, executor, n_slots: int = 2, ws_budget: int | None = None, max_batch: int | None = None,
                 clock=time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        # bytes the executor may hold for in-flight steps (an executor with a
        # device arena bounds this by the arena's size)
        cap = getattr(executor, "capacity", None)
        if ws_budget is None:
            ws_budget = cap
        if ws_budget is None:
            raise ValueError("ws_budget is needed for an executor without a fixed capacity")
        if cap is not None and ws_budget > cap:
            raise ValueError(f"ws_budget {ws_budget} exceeds the executor's device arena of {cap} bytes")
        self.ws_budget = ws_budget
        self.max_batch = max_batch
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.free_slots = list(range(n_slots))
        self.in_flight: list[Step] = []
        self.ws_in_use = 0
        self.max_ws_in_use = 0
        self.t0 = None
        self.completed: list[Request] = []
        self.steps_launched = 0
        self.max_in_flight = 0
        self.batch_sizes: list[int] = []
        self.busy_since = None  # start of the current stretch with a step in flight
        self.busy_time = 0.0

    def now(self) -> float:
        return self.clock() - self.t0

    def start(self):
        self.t0 = self.clock()
        self.busy_since = None
        self.busy_time = 0.0

    def busy_fraction(self, span: float) -> float:
        """Fraction of `span` seconds during which at least one step was in
        flight (launched and not yet seen complete)."""
        busy = self.busy_time + ((self.now() - self.busy_since) if self.busy_since is not None else 0.0)
        return busy / span if span > 0 else 0.0

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
                self.ex.release(st.token)
                self.ws_in_use -= st.ws_bytes
                self.free_slots.append(st.slot)
            else:
                still.append(st)
        self.in_flight = still
        if not self.in_flight and self.busy_since is not None:
            self.busy_time += self.now() - self.busy_since
            self.busy_since = None

    def _take_batch(self):
        """Requests from the head of the queue for one step: ceil(queued / free
        slots) of them (at most max_batch), as long as their estimated memory
        fits what the budget has left."""
        want = -(-len(self.queue) // len(self.free_slots))
        if self.max_batch is not None:
            want = min(want, self.max_batch)
        batch, est = [], 0
        while self.queue and len(batch) < want:
            need = self.ex.request_ws(self.queue[0])
            if self.ws_in_use + est + need > self.ws_budget:
                break
            batch.append(self.queue.popleft())
            est += need
        return batch

    def _admit(self):
        while self.free_slots and self.queue:
            batch = self._take_batch()
            token = None
            while batch:
                token = self.ex.reserve(batch)  # exact bytes of the step, or None if they do not fit now
                if token is not None and self.ws_in_use + self.ex.token_bytes(token) <= self.ws_budget:
                    break
                if token is not None:
                    self.ex.release(token)
                    token = None
                self.queue.appendleft(batch.pop())  # shrink the step from its tail
            if not batch:
                return  # the head does not fit until memory frees up
            slot = self.free_slots.pop(0)
            t = self.now()
            for r in batch:
                r.admitted = t
                r.batch = len(batch)
            nbytes = self.ex.token_bytes(token)
            st = Step(slot=slot, reqs=batch, ws_bytes=nbytes, token=token, launched=t)
            try:
                st.handle = self.ex.launch(batch, slot, token)
            except Exception as e:
                for r in batch:
                    r.error = f"launch failed: {e}"
                    r.done = self.now()
                    self.completed.append(r)
                self.ex.release(token)
                self.free_slots.append(slot)
                continue
            self.ws_in_use += nbytes
            self.max_ws_in_use = max(self.max_ws_in_use, self.ws_in_use)
            if self.busy_since is None:
                self.busy_since = t
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
    """p50 / p99 / mean latency (ms) of the successful requests, their Gpts/s
    over the run's span, and the number of failed requests."""
    errors = sum(1 for r in reqs if r.error is not None)
    lat = np.array([r.latency for r in reqs if r.error is None], dtype=np.float64) * 1e3
    pts = sum(r.n for r in reqs if r.error is None)
    if lat.size == 0:
        return {"requests": 0, "errors": errors}
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
        "errors": errors,
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

class Arena:
    """First-fit allocator of byte ranges in [0, size), 256-byte aligned (host
    bookkeeping of one device allocation)."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)]  # sorted, non-adjacent (offset, length) holes
        self.used = 0

    @classmethod
    def round(cls, nbytes: int) -> int:
        return -(-max(int(nbytes), 1) // cls.ALIGN) * cls.ALIGN

    def alloc(self, nbytes: int):
        nbytes = self.round(nbytes)
        for i, (o, ln) in enumerate(self.free):
            if ln >= nbytes:
                if ln == nbytes:
                    del self.free[i]
                else:
                    self.free[i] = (o + nbytes, ln - nbytes)
                self.used += nbytes
                return o, nbytes
        return None

    def release(self, block):
        o, ln = block
        self.used -= ln
        holes = self.free
        i = 0
        while i < len(holes) and holes[i][0] < o:
            i += 1
        holes.insert(i, (o, ln))
        # merge with the neighbours
        if i + 1 < len(holes) and holes[i][0] + holes[i][1] == holes[i + 1][0]:
            holes[i] = (holes[i][0], holes[i][1] + holes[i + 1][1])
            del holes[i + 1]
        if i > 0 and holes[i - 1][0] + holes[i - 1][1] == holes[i][0]:
            holes[i - 1] = (holes[i - 1][0], holes[i - 1][1] + holes[i][1])
            del holes[i]


class _HipRuntime:
    """The process's HIP runtime (the one torch loaded: the same shared object,
    found by its soname) for the serving loop's stream-ordered copies of
    results to pinned host memory and its completion events, called without
    torch dispatch in between."""

    DEVICE_TO_HOST = 2
    DISABLE_TIMING = 2
    NOT_READY = 600

    def __init__(self):
        h = ctypes.CDLL("libamdhip64.so.7")
        vp = ctypes.c_void_p
        h.hipMemcpyAsync.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int, vp]
        h.hipMemcpyAsync.restype = ctypes.c_int
        h.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(vp), ctypes.c_uint]
        h.hipEventCreateWithFlags.restype = ctypes.c_int
        h.hipEventRecord.argtypes = [vp, vp]
        h.hipEventRecord.restype = ctypes.c_int
        h.hipEventQuery.argtypes = [vp]
        h.hipEventQuery.restype = ctypes.c_int
        h.hipEventDestroy.argtypes = [vp]
        h.hipEventDestroy.restype = ctypes.c_int
        self.h = h

    def event(self):
        ev = ctypes.c_void_p()
        rc = self.h.hipEventCreateWithFlags(ctypes.byref(ev), self.DISABLE_TIMING)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
        return ev

    def copy_to_host(self, dst, src, nbytes, stream):
        rc = self.h.hipMemcpyAsync(dst, src, nbytes, self.DEVICE_TO_HOST, stream)
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({rc})")

    def record(self, ev, stream):
        rc = self.h.hipEventRecord(ev, stream)
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def done(self, ev) -> bool:
        rc = self.h.hipEventQuery(ev)
        if rc == self.NOT_READY:
            return False
        if rc != 0:
            raise RuntimeError(f"step failed on the device (hipEventQuery: {rc})")
        return True


class GpuExecutor:
    """Runs each admitted set of requests as one batched call on the slot's
    stream (a set of one takes the single-series call, which launches fewer
    kernels and gives the same indices), then copies the indices to the slot's
    pinned host buffer on that stream. Workspace and output of every step come
    from one device arena of `arena_bytes` allocated here. Launches, copies and
    completion events go through the C ABI and the HIP runtime with raw
    pointers, so a step costs the host a few calls."""

    def __init__(self, y, offsets, lengths, x=None, n_slots: int = 2, arena_bytes: int = 256 << 20,
                 host_capacity: int = 1 << 20):
        import torch

        self.torch = torch
        self.y, self.x = y, x
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.lengths = np.asarray(lengths, dtype=np.int64)
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.capacity = int(arena_bytes)
        self.arena = torch.empty(self.capacity, dtype=torch.uint8, device=y.device)
        self.blocks = Arena(self.capacity)
        self.host = [torch.empty(host_capacity, dtype=torch.int64, pin_memory=True) for _ in range(n_slots)]
        self.lib = _lib.load()
        self.hip = _HipRuntime()
        self.events = [self.hip.event() for _ in range(n_slots)]
        self.stream_ptrs = [s.cuda_stream for s in self.streams]
        self.arena_ptr = self.arena.data_ptr()
        self.y_ptr = y.data_ptr()
        self.x_ptr = x.data_ptr() if x is not None else None
        self.xk = _lib.X_INT64 if x is not None else _lib.X_IMPLICIT
        self._ws_cache = {}

    def __del__(self):
        try:
            for ev in getattr(self, "events", []):
                self.hip.h.hipEventDestroy(ev)
        except Exception:  # interpreter shutdown
            pass

    def series_len(self, s: int) -> int:
        return int(self.lengths[s])

    def _single_ws(self, n_out: int, r_ps: int) -> int:
        key = (n_out, r_ps)
        v = self._ws_cache.get(key)
        if v is None:
            v = int(_lib.load().mmlttb_workspace_size(1, n_out, r_ps))
            self._ws_cache[key] = v
        return v

    def request_ws(self, r: Request) -> int:
        """Device bytes of the request served alone (workspace and output)."""
        return Arena.round(self._single_ws(r.n_out, r.r_ps)) + Arena.round(8 * min(r.n, r.n_out))

    def _segs(self, reqs):
        return [(int(self.offsets[r.series]) + r.lo, r.n, r.n_out, r.r_ps) for r in reqs]

    def reserve(self, reqs):
        """The step's exact device memory (workspace sized by the library for
        this step, output indices) as one arena block, or None when it does
        not fit now."""
        table = None
        if len(reqs) == 1:
            ws = self._single_ws(reqs[0].n_out, reqs[0].r_ps)
        else:
            from .ops import segment_table

            table = segment_table(self._segs(reqs))
            ws = int(_lib.load().mmlttb_batched_workspace_size(table[0], len(table[0])))
        total_out = sum(min(r.n, r.n_out) for r in reqs)
        ws_r = Arena.round(ws)
        block = self.blocks.alloc(ws_r + Arena.round(8 * total_out))
        if block is None:
            return None
        return {"block": block, "ws": ws_r, "out": total_out, "table": table}

    @staticmethod
    def token_bytes(token) -> int:
        return token["block"][1]

    def release(self, token):
        if token is not None:
            self.blocks.release(token["block"])

    def _views(self, token):
        o, ln = token["block"]
        ws = self.arena[o: o + token["ws"]]
        out = self.arena[o + token["ws"]: o + token["ws"] + 8 * max(token["out"], 1)].view(self.torch.int64)
        return ws, out

    def _host(self, slot, count):
        torch = self.torch
        if self.host[slot].numel() < count:
            self.host[slot] = torch.empty(max(count, 2 * self.host[slot].numel()), dtype=torch.int64,
                                          pin_memory=True)
        return self.host[slot][:count]

    def _finish(self, slot, out_ptr, count):
        """Copy the step's indices to the slot's pinned buffer and record the
        slot's event, both on the slot's stream."""
        host = self._host(slot, count)
        if count:
            self.hip.copy_to_host(host.data_ptr(), out_ptr, 8 * count, self.stream_ptrs[slot])
        self.hip.record(self.events[slot], self.stream_ptrs[slot])
        return host

    def _launch_one(self, r, slot, ws_ptr, ws_bytes, out_ptr):
        o = int(self.offsets[r.series]) + r.lo
        xp = None if self.x_ptr is None else self.x_ptr + 8 * o
        _lib.check(self.lib.mmlttb_minmaxlttb(self.xk, xp, self.y_ptr + 4 * o, r.n, r.n_out, r.r_ps, out_ptr,
                                              ws_ptr, ws_bytes, self.stream_ptrs[slot]))

    def _launch_single(self, r, slot, token):
        """A step of one request: the single-series call into the step's block."""
        base = self.arena_ptr + token["block"][0]
        ws_bytes = token["ws_each"][0] if token.get("ws_each") else token["ws"]
        self._launch_one(r, slot, base, ws_bytes, base + token["ws"])
        k = min(r.n, r.n_out)
        return (self.events[slot], self._finish(slot, base + token["ws"], k), [0], [k])

    def launch(self, reqs, slot, token):
        if len(reqs) == 1:
            return self._launch_single(reqs[0], slot, token)
        from .ops import minmaxlttb_batched

        torch = self.torch
        ws, out = self._views(token)
        with torch.cuda.stream(self.streams[slot]):
            _, outoff = minmaxlttb_batched(self.y, None, x_base=self.x, out=out, ws=ws, table=token["table"])
        host = self._finish(slot, out.data_ptr(), token["out"])
        return (self.events[slot], host, outoff, [min(r.n, r.n_out) for r in reqs])

    def poll(self, handle) -> bool:
        return self.hip.done(handle[0])

    def collect(self, handle):
        _, host, outoff, counts = handle
        h = host.numpy()
        return [h[o: o + c].copy() for o, c in zip(outoff, counts)]


class PlainGpuExecutor(GpuExecutor):
    """Comparator: one single-series call per request, in arrival order, each
    with its own workspace region of the step's arena block."""

    def reserve(self, reqs):
        ws = [Arena.round(self._single_ws(r.n_out, r.r_ps)) for r in reqs]
        total_out = sum(min(r.n, r.n_out) for r in reqs)
        block = self.blocks.alloc(sum(ws) + Arena.round(8 * total_out))
        if block is None:
            return None
        return {"block": block, "ws": sum(ws), "ws_each": ws, "out": total_out, "table": None}

    def launch(self, reqs, slot, token):
        if len(reqs) == 1:
            return self._launch_single(reqs[0], slot, token)
        base = self.arena_ptr + token["block"][0]
        ws_each = token.get("ws_each") or [token["ws"]]
        out_ptr = base + token["ws"]
        counts = [min(r.n, r.n_out) for r in reqs]
        offs = [0] * len(reqs)
        w = o_out = 0
        for i, (r, k, wb) in enumerate(zip(reqs, counts, ws_each)):
            offs[i] = o_out
            self._launch_one(r, slot, base + w, wb, out_ptr + 8 * o_out)
            w += wb
            o_out += k
        host = self._finish(slot, out_ptr, token["out"])
        return (self.events[slot], host, offs, counts)
