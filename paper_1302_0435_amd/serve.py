"""Serving loop: a stream of query distributions scored against centroids
kept resident in HBM (the labelling step of Alg. 2, Step 2, one query at a
time as requests arrive).

Queries arrive on an open-loop Poisson schedule.  Each request carries its
support points and weights; its footprint on the device is its input bytes
plus its K distances, label, minimum and status.  The scheduler

  * admits requests in arrival order while their footprint fits the HBM
    budget still free and a stream slot is free (requests that do not fit
    wait; nothing is dropped).  The budget is one device buffer: each batch
    gets a contiguous range of it from a first-fit allocator and gives it
    back when it completes, so the requests' device memory is the budget,
    whatever the batch sizes,
  * packs every admitted request that has arrived into one batch
    (continuous batching: a slot that frees up takes whatever is waiting),
  * runs the batch on its own HIP stream -- host-to-device copy from pinned
    memory, d2_assign against the resident centroids, copy back -- so
    batches on different slots overlap on the device,
  * measures each request's latency from its scheduled arrival time to the
    device completion of its batch (no coordinated omission).  Device times
    are kept against a reference event; the host time at which that event is
    known to have passed is taken as its place on the host clock, so a
    latency can only be overstated by that bound, never understated.

The scheduler core is independent of the device: it drives an executor
object (GpuExecutor here; tests use a scripted one) through submit / poll.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Optional

import numpy as np

# ------------------------------------------------------------ query pool


@dataclasses.dataclass
class QueryPool:
    """Ragged host-side set of query distributions (FP64), reused cyclically."""
    offsets: np.ndarray
    points: np.ndarray
    weights: np.ndarray

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def d(self) -> int:
        return int(self.points.shape[1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)


def request_bytes(t: int, d: int, k: int) -> int:
    """Device footprint of one request: points, weights, offset, K distances,
    label, minimum, status."""
    return t * d * 8 + t * 8 + 8 + k * 8 + 4 + 8 + 4


@dataclasses.dataclass
class Batch:
    slot: int
    first: int          # first request index (arrival order)
    count: int
    nbytes: int
    submit_s: float = 0.0
    arena_off: int = 0  # start of the batch's range of the budget buffer
    arena_len: int = 0  # its length (the requests' bytes, the extra offset, alignment)


BATCH_EXTRA = 8         # a batch's offsets array has one entry more than requests


class Arena:
    """First-fit allocation of byte ranges of one buffer of ``size`` bytes;
    lengths are rounded up to ``align``, freed ranges merge with their free
    neighbours."""

    def __init__(self, size: int, align: int = 256):
        self.size, self.align = int(size), int(align)
        self.free = [(0, self.size)] if self.size > 0 else []   # sorted (start, length)

    def need(self, nbytes: int) -> int:
        return -(-(int(nbytes) + BATCH_EXTRA) // self.align) * self.align

    def largest(self) -> int:
        return max((n for _, n in self.free), default=0)

    def alloc(self, length: int) -> Optional[int]:
        for i, (a, n) in enumerate(self.free):
            if n >= length:
                if n == length:
                    del self.free[i]
                else:
                    self.free[i] = (a + length, n - length)
                return a
        return None

    def release(self, start: int, length: int):
        self.free.append((start, length))
        self.free.sort()
        merged = []
        for a, n in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + n)
            else:
                merged.append((a, n))
        self.free = merged


# ------------------------------------------------------------ scheduler


@dataclasses.dataclass
class ServeStats:
    arrivals: np.ndarray
    done_s: np.ndarray          # completion time per request (nan: not completed)
    batch_sizes: List[int]
    max_queue: int
    duration_s: float

    def latencies_ms(self) -> np.ndarray:
        ok = ~np.isnan(self.done_s)
        return (self.done_s[ok] - self.arrivals[ok]) * 1e3

    def summary(self, k: int) -> dict:
        lat = self.latencies_ms()
        done = int((~np.isnan(self.done_s)).sum())
        end = float(np.nanmax(self.done_s)) if done else self.duration_s
        span = max(end, self.duration_s)
        return {
            "requests": int(self.arrivals.size), "completed": done,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "max_ms": float(lat.max()) if lat.size else None,
            "distances_per_s": done * k / span,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "batches": len(self.batch_sizes), "max_queue": self.max_queue,
        }


class Scheduler:
    """Admission by HBM budget, slots, continuous batching, latency record."""

    def __init__(self, executor, sizes: np.ndarray, d: int, k: int, budget_bytes: int,
                 max_batch: int, slots: int, align: int = 256):
        self.ex = executor
        self.sizes = sizes          # support size of every request, in arrival order
        self.d, self.k = d, k
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.slots = int(slots)
        self.align = int(align)

    def run(self, arrivals: np.ndarray, clock=time.perf_counter, sleep=time.sleep,
            idle_sleep=50e-6) -> ServeStats:
        n = arrivals.size
        fp = np.array([request_bytes(int(t), self.d, self.k) for t in self.sizes[:n]], np.int64)
        done_s = np.full(n, np.nan)
        free_slots = collections.deque(range(self.slots))
        inflight: List[Batch] = []
        arena = Arena(self.budget, self.align)
        next_req = 0            # first request not yet admitted
        batch_sizes: List[int] = []
        max_queue = 0
        t0 = clock()
        # the executor reports completions against its own origin; `shift`
        # places that origin on this loop's clock (arrivals count from t0)
        shift = self.ex.start(clock) - t0
        while True:
            now = clock() - t0
            arrived = int(np.searchsorted(arrivals, now, side="right"))
            max_queue = max(max_queue, arrived - next_req)
            progressed = False
            # retire finished batches, freeing their slot and budget
            for b in list(inflight):
                t_done = self.ex.poll(b)
                if t_done is not None:
                    done_s[b.first:b.first + b.count] = t_done + shift
                    arena.release(b.arena_off, b.arena_len)
                    free_slots.append(b.slot)
                    inflight.remove(b)
                    progressed = True
            # admit and launch everything that has arrived, within the limits
            while free_slots and next_req < arrived:
                count, nbytes = 0, 0
                room = arena.largest()
                while (next_req + count < arrived and count < self.max_batch and
                       arena.need(nbytes + fp[next_req + count]) <= room):
                    nbytes += int(fp[next_req + count])
                    count += 1
                if count == 0:
                    break       # the head request does not fit yet: it waits
                length = arena.need(nbytes)
                b = Batch(free_slots.popleft(), next_req, count, nbytes, now,
                          arena.alloc(length), length)
                self.ex.submit(b)
                inflight.append(b)
                next_req += count
                batch_sizes.append(count)
                progressed = True
            if next_req >= n and not inflight:
                break
            if arrived == n and not inflight and arena.need(fp[next_req]) > self.budget:
                break           # budget below one request: it stays queued, unserved
            if not progressed:
                nxt = arrivals[arrived] - now if arrived < n else idle_sleep
                sleep(max(0.0, min(idle_sleep, nxt)))
        self.ex.stop()
        return ServeStats(arrivals, done_s, batch_sizes, max_queue,
                          float(arrivals[-1]) if n else 0.0)


def warm_up(sch: "Scheduler", arrivals: np.ndarray, burst: int = 512, seconds: float = 0.5,
            **run_kw):
    """Serve a burst of requests arriving together, then the first
    ``seconds`` of the schedule, before a measured run on the same scheduler.
    The first batches of each shape carry one-time costs (kernel code loaded
    on first launch, allocations): measured at 36 ms in one submit, which
    queued the requests behind it and set the p99 of a 2 s run.  The burst
    reaches the largest batch and every support class.  ``run_kw`` goes to
    ``Scheduler.run`` (clock, sleep)."""
    n = min(int(burst), int(arrivals.size))
    if n:
        sch.run(np.zeros(n), **run_kw)
        sch.run(arrivals[arrivals < seconds], **run_kw)


# ------------------------------------------------------------ executors


class GpuExecutor:
    """Runs batches on HIP streams: pinned-host copy in, d2_assign against the
    resident centroids, copy out.  Completion times come from HIP events.

    The requests' device data (points, weights, offsets, K distances, label,
    minimum, status) live in one buffer of ``budget_bytes``: a batch's arrays
    are views of the range the scheduler allocated to it (``Batch.arena_off``),
    so the scheduler's budget is the memory they use.  Each slot also holds
    the library workspace for ``max_batch`` requests, outside the budget."""

    def __init__(self, pool: QueryPool, req_pool_index: np.ndarray, Zd, k: int, slots: int,
                 max_batch: int, device: int = 0, keep_results: bool = False, init: int = 0,
                 budget_bytes: int = 256 << 20):
        import torch
        from . import api
        self.torch = torch
        self.api = api
        self.dev = torch.device("cuda", device)
        self.h = api.Handle(device)
        self.pool = pool
        self.idx = req_pool_index              # request -> pool entry (cyclic)
        self.Zd = Zd
        self.k = k
        self.d = pool.d
        self.opts = api.Opts(init=init, flags=1)   # eager: batch shapes vary
        tmax = int(pool.sizes().max())
        self.max_batch = max_batch
        # pinned host copies of the pool
        self.h_pts = torch.from_numpy(np.ascontiguousarray(pool.points)).pin_memory()
        self.h_w = torch.from_numpy(np.ascontiguousarray(pool.weights)).pin_memory()
        self.sizes = pool.sizes()
        self.keep = keep_results
        self.results = {}
        self.arena = torch.empty(max(int(budget_bytes), 1), dtype=torch.uint8, device=self.dev)
        self.slots = []
        for _ in range(slots):
            s = {
                "stream": torch.cuda.Stream(device=self.dev),
                "h_off": torch.empty(max_batch + 1, dtype=torch.int64).pin_memory(),
                "h_labels": torch.empty(max_batch, dtype=torch.int32).pin_memory(),
                "h_best": torch.empty(max_batch, dtype=torch.float64).pin_memory(),
                "h_all": torch.empty((max_batch, k), dtype=torch.float64).pin_memory(),
                "h_status": torch.empty(max_batch, dtype=torch.int32).pin_memory(),
                "ev": torch.cuda.Event(enable_timing=True),
            }
            self.slots.append(s)
        # workspace big enough for any batch of at most max_batch requests
        # (the size depends on the request count and the largest support)
        p_off = torch.zeros(max_batch + 1, dtype=torch.int64, device=self.dev)
        p_pts = torch.empty((1, self.d), dtype=torch.float64, device=self.dev)
        p_w = torch.empty(1, dtype=torch.float64, device=self.dev)
        ws_b = 0
        for nq in range(1, max_batch + 1):
            probe = api.DeviceSet(p_off[:nq + 1], p_pts, p_w, tmax)
            ws_b = max(ws_b, api.d2_workspace_bytes(self.h, 2, probe, Zd, 0, self.opts))
        del p_off, p_pts, p_w
        self.ws_bytes = ws_b
        for s in self.slots:
            s["ws"] = torch.empty(max(ws_b, 1), dtype=torch.uint8, device=self.dev)
        self.ref = torch.cuda.Event(enable_timing=True)

    def _views(self, b: Batch, atoms: int):
        """The batch's device arrays, carved in order from its arena range."""
        torch = self.torch
        c, d, k = b.count, self.d, self.k
        if b.arena_off < 0 or b.arena_off + b.arena_len > self.arena.numel():
            raise ValueError("batch range outside the budget buffer")
        o = b.arena_off
        out = []
        for nbytes, dtype in ((atoms * d * 8, torch.float64), (atoms * 8, torch.float64),
                              ((c + 1) * 8, torch.int64), (c * k * 8, torch.float64),
                              (c * 8, torch.float64), (c * 4, torch.int32), (c * 4, torch.int32)):
            out.append(self.arena[o:o + nbytes].view(dtype))
            o += nbytes
        if o - b.arena_off != b.nbytes + BATCH_EXTRA or o - b.arena_off > b.arena_len:
            raise ValueError("batch footprint does not match its requests")
        pts, w, off, allv, best, labels, status = out
        return pts.view(atoms, d), w, off, allv.view(c, k), best, labels, status

    def start(self, clock=time.perf_counter) -> float:
        """Record the reference event on an idle device; return the host time
        once it has completed (an upper bound on the event's own time)."""
        self.torch.cuda.synchronize(self.dev)
        self.ref.record(self.torch.cuda.current_stream(self.dev))
        self.ref.synchronize()
        return clock()

    def stop(self):
        self.torch.cuda.synchronize(self.dev)

    def submit(self, b: Batch):
        torch = self.torch
        s = self.slots[b.slot]
        ids = self.idx[b.first:b.first + b.count]
        sz = self.sizes[ids]
        off = np.zeros(b.count + 1, np.int64)
        np.cumsum(sz, out=off[1:])
        pts, w, d_off, allv, best, labels, status = self._views(b, int(off[-1]))
        s["h_off"][:b.count + 1].copy_(torch.from_numpy(off))
        with torch.cuda.stream(s["stream"]):
            d_off.copy_(s["h_off"][:b.count + 1], non_blocking=True)
            # requests are consecutive pool entries except across the wrap point
            pos = 0
            runs = np.split(ids, np.flatnonzero(np.diff(ids) != 1) + 1)
            for r in runs:
                a0, a1 = int(self.pool.offsets[r[0]]), int(self.pool.offsets[r[-1] + 1])
                pts[pos:pos + a1 - a0].copy_(self.h_pts[a0:a1], non_blocking=True)
                w[pos:pos + a1 - a0].copy_(self.h_w[a0:a1], non_blocking=True)
                pos += a1 - a0
            Xd = self.api.DeviceSet(d_off, pts, w, int(sz.max()))
            self.api.d2_assign_into(self.h, Xd, self.Zd, self.opts, labels, best, allv, status,
                                    s["ws"], self.ws_bytes)
            s["h_labels"][:b.count].copy_(labels, non_blocking=True)
            s["h_best"][:b.count].copy_(best, non_blocking=True)
            s["h_all"][:b.count].copy_(allv, non_blocking=True)
            s["h_status"][:b.count].copy_(status, non_blocking=True)
            s["ev"].record(s["stream"])
        s["batch"] = b

    def poll(self, b: Batch) -> Optional[float]:
        s = self.slots[b.slot]
        if not s["ev"].query():
            return None
        if self.keep:
            for q in range(b.count):
                self.results[b.first + q] = (int(s["h_labels"][q]), float(s["h_best"][q]),
                                             s["h_all"][q].numpy().copy(), int(s["h_status"][q]))
        return self.ref.elapsed_time(s["ev"]) / 1e3


class ScriptedExecutor:
    """Test double: a batch takes `duration(count)` seconds from submission
    (batches run concurrently, one per slot) and returns given results."""

    def __init__(self, duration, clock=time.perf_counter):
        self.duration = duration
        self.clock = clock
        self.t0 = None
        self.submitted = []

    def start(self, clock=None) -> float:
        self.t0 = self.clock()
        return self.t0

    def stop(self):
        pass

    def submit(self, b: Batch):
        b.submit_s = self.clock() - self.t0
        self.submitted.append((b.first, b.count, b.slot))

    def poll(self, b: Batch) -> Optional[float]:
        t_done = b.submit_s + self.duration(b.count)
        return t_done if self.clock() - self.t0 >= t_done else None
