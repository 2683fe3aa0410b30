"""Served form of the path: continuous batching of frames from several
simulated camera streams on one GPU.

* Requests arrive per stream (Poisson traces from datagen.poisson_arrivals).
* Each stream owns slots: resident device buffer sets (inputs, every
  intermediate of the path, the disparity outputs).  A slot is carved the
  first time the stream needs one and then reused for every later frame of
  that stream.  All slots live in one device arena of the HBM budget's size,
  allocated once: the budget is the memory the server holds, not a count.
  When a stream needs a slot that does not fit, idle slots of other streams
  are released back to the arena (least recently used first) -- no device
  allocation or free happens while serving.  HIP streams and the pinned
  output buffers are made once, so admitting a slot allocates nothing at
  all.  A frame is admitted as soon as one of its stream's slots is idle
  (or a new one fits the budget) and fewer than `hip_streams` frames are in
  flight, so frames that arrive while others run start at once and overlap
  with them on the device.  Per stream, frames are admitted in arrival
  order.  A run hands its slots back to the arena at the end.
* Per frame: pinned H2D copy of the pair, the streamlined path (census of
  both images, cost, aggregation fused with the selection), D2H copy of the
  disparity map, all on one HIP stream of the pool, taken in turn;
  completion is an event.
  Latency = time of the event (read against an event recorded at the start)
  minus the arrival time.
* The plain reference serves the same trace FIFO, one frame at a time on one
  stream.

The scheduling loop is independent of the device: GpuBackend runs it on the
GPU, FakeBackend simulates service times on a virtual clock for CPU tests.
"""
from __future__ import annotations

import collections
import gc
import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import datagen


@dataclass
class Request:
    stream: int
    seq: int
    arrival: float           # seconds from the start of the trace
    frame: int               # index into the stream's frame pool


@dataclass
class StreamSpec:
    width: int
    height: int
    ndisp: int
    seed: int


@dataclass
class Result:
    request: Request
    start: float             # admission time
    done: float              # completion time
    slot: int


@dataclass
class Stats:
    served: int = 0
    rejected: int = 0
    deferred: int = 0        # admissions that had to wait for a slot or budget
    evictions: int = 0       # idle slots released to admit another stream
    peak_bytes: int = 0
    results: List[Result] = field(default_factory=list)

    def latencies_ms(self):
        return np.array([(r.done - r.request.arrival) * 1e3 for r in self.results])

    def summary(self, specs) -> dict:
        lat = self.latencies_ms()
        span = max((r.done for r in self.results), default=0.0)
        des = sum(specs[r.request.stream].width * specs[r.request.stream].height *
                  specs[r.request.stream].ndisp for r in self.results)
        return {"frames": self.served, "rejected": self.rejected, "deferred": self.deferred,
                "evictions": self.evictions,
                "p50_ms": round(float(np.percentile(lat, 50)), 3) if len(lat) else None,
                "p99_ms": round(float(np.percentile(lat, 99)), 3) if len(lat) else None,
                "max_ms": round(float(lat.max()), 3) if len(lat) else None,
                "frames_per_s": round(self.served / span, 1) if span > 0 else None,
                "mdes": round(des / span / 1e6, 1) if span > 0 else None,
                "peak_gib": round(self.peak_bytes / 2 ** 30, 3)}


def make_trace(specs, rate_hz: float, duration_s: float, frames_per_stream: int, seed: int):
    """Merged, time-ordered Poisson arrivals of every stream."""
    reqs = []
    for s in range(len(specs)):
        for k, t in enumerate(datagen.poisson_arrivals(rate_hz, duration_s, seed * 100 + s)):
            reqs.append(Request(s, k, float(t), k % frames_per_stream))
    reqs.sort(key=lambda r: (r.arrival, r.stream))
    return reqs


def _a256(b: int) -> int:
    return (b + 255) // 256 * 256


class Arena:
    """First-fit allocator over [0, capacity) in 256-byte units, with
    coalescing of released ranges.  Host bookkeeping only; GpuBackend maps
    its offsets onto one device buffer."""

    ALIGN = 256

    def __init__(self, capacity: int):
        self.capacity = capacity // self.ALIGN * self.ALIGN
        self.free = [(0, self.capacity)]         # sorted, disjoint (offset, size)
        self.used = 0

    @classmethod
    def round(cls, nbytes: int) -> int:
        return (max(1, nbytes) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def alloc(self, nbytes: int) -> Optional[int]:
        need = self.round(nbytes)
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, size - need)
                self.used += need
                return off
        return None

    def release(self, off: int, nbytes: int):
        size = self.round(nbytes)
        self.used -= size
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, (off, size))
        # merge with the neighbours
        if i + 1 < len(self.free) and off + size == self.free[i + 1][0]:
            self.free[i] = (off, size + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def largest_free(self) -> int:
        return max((size for _, size in self.free), default=0)


def slot_bytes(spec: StreamSpec, npaths: int, p2: int) -> int:
    """Device bytes of one slot as the arena carves it, each buffer rounded up
    to 256 bytes: the two input images, both census maps, the cost volume,
    the two disparity maps, and the workspace of the streamlined aggregation
    (path slices, S_bar only where the fused selection does not apply, D^R
    keys, D^L); one path slice per pair of opposite directions, uint8 for
    P2 <= 127, else uint16."""
    n = spec.width * spec.height
    nd = spec.ndisp
    slices = npaths // 2 * _a256(n * nd) * (1 if p2 <= 127 else 2)
    fused = nd % 16 == 0 and nd <= 256
    work = _a256(slices) + (0 if fused else _a256(2 * n * nd)) + _a256(4 * n) + _a256(2 * n)
    return 2 * _a256(n) + 2 * _a256(8 * n) + _a256(n * nd) + 2 * _a256(2 * n) + _a256(work)


class Server:
    """Continuous-batching scheduler over a backend (see module docstring)."""

    def __init__(self, specs: List[StreamSpec], backend, budget_bytes: int, hip_streams: int = 8,
                 max_slots_per_stream: int = 2, npaths: int = 8, p2: int = 120):
        self.specs = specs
        self.backend = backend
        self.budget = budget_bytes
        self.hip_streams = hip_streams
        self.max_slots = max_slots_per_stream
        self.sizes = [slot_bytes(s, npaths, p2) for s in specs]
        self.slots: Dict[int, List[dict]] = collections.defaultdict(list)
        self.used_bytes = 0
        self.evictions = 0
        self._tick = 0

    def _evict_for(self, need: int) -> bool:
        """Releases idle slots, least recently used first, until `need` more
        bytes fit; False if the idle slots are not enough."""
        idle = sorted(((slot["last"], s, slot) for s, lst in self.slots.items() for slot in lst
                       if slot["job"] is None), key=lambda t: t[0])
        free = self.budget - self.used_bytes
        if free + sum(self.sizes[s] for _, s, _ in idle) < need:
            return False
        for _, s, slot in idle:
            if free >= need:
                break
            self.slots[s].remove(slot)
            self.backend.free_slot(slot["handle"])
            self.used_bytes -= self.sizes[s]
            free += self.sizes[s]
            self.evictions += 1
        return True

    def _evict_one(self, exclude: int) -> bool:
        idle = sorted(((slot["last"], t, slot) for t, lst in self.slots.items() for slot in lst
                       if slot["job"] is None and t != exclude), key=lambda v: v[0])
        if not idle:
            return False
        _, t, slot = idle[0]
        self.slots[t].remove(slot)
        self.backend.free_slot(slot["handle"])
        self.used_bytes -= self.sizes[t]
        self.evictions += 1
        return True

    def _free_slot(self, s: int) -> Optional[dict]:
        self._tick += 1
        for slot in self.slots[s]:
            if slot["job"] is None:
                slot["last"] = self._tick
                return slot
        if len(self.slots[s]) >= self.max_slots:
            return None
        if self.used_bytes + self.sizes[s] > self.budget:
            if self.slots[s] or not self._evict_for(self.sizes[s]):
                return None          # only a stream with no slot may evict others
        handle = self.backend.alloc_slot(s)
        while handle is None:
            # the arena has the bytes but not in one piece: release the least
            # recently used idle slot of another stream and try again
            if self.slots[s] or not self._evict_one(exclude=s):
                return None
            handle = self.backend.alloc_slot(s)
        slot = {"id": len(self.slots[s]), "handle": handle, "job": None, "last": self._tick}
        self.slots[s].append(slot)
        self.used_bytes += self.sizes[s]
        return slot

    def run(self, trace: List[Request], keep=None, release: bool = True) -> Stats:
        """Serves the trace; `keep(request)` says whether to copy a result to
        the host for checking (the backend keeps it in result_of).  With
        `release` the slots go back to the backend at the end, so that
        another server can use its memory; else they stay for the next run.
        Before the clock starts, every stream of the trace that has no slot
        gets one while the budget holds them without evictions (streams are
        known up front), and Python's garbage collector is paused for the
        run so that no collection lands inside a frame's latency."""
        stats = Stats()
        for s, size in enumerate(self.sizes):
            if size > self.budget:
                stats.rejected += sum(1 for r in trace if r.stream == s)
        trace = [r for r in trace if self.sizes[r.stream] <= self.budget]
        for s in dict.fromkeys(r.stream for r in trace):
            if not self.slots[s] and self.used_bytes + self.sizes[s] <= self.budget:
                handle = self.backend.alloc_slot(s)
                if handle is None:
                    continue
                self.slots[s].append({"id": 0, "handle": handle, "job": None, "last": self._tick})
                self.used_bytes += self.sizes[s]
        pending = collections.defaultdict(collections.deque)
        inflight = []
        waited = set()
        i = 0
        gc_enabled = gc.isenabled()
        gc.collect()
        gc.disable()
        try:
            return self._serve(trace, keep, release, stats, pending, inflight, waited, i)
        finally:
            if gc_enabled:
                gc.enable()

    def _serve(self, trace, keep, release, stats, pending, inflight, waited, i) -> Stats:
        self.backend.start()
        while i < len(trace) or inflight or any(pending.values()):
            now = self.backend.now()
            while i < len(trace) and trace[i].arrival <= now:
                pending[trace[i].stream].append(trace[i])
                i += 1
            # completions free their slot
            still = []
            for job in inflight:
                t_done = self.backend.done(job["handle"])
                if t_done is not None:
                    job["slot"]["job"] = None
                    stats.results.append(Result(job["req"], job["start"], t_done, job["slot"]["id"]))
                    stats.served += 1
                else:
                    still.append(job)
            inflight = still
            # admission: oldest waiting head first, per-stream FIFO
            heads = sorted((q[0].arrival, s) for s, q in pending.items() if q)
            admitted = False
            for _, s in heads:
                if len(inflight) >= self.hip_streams:
                    break
                slot = self._free_slot(s)
                req = pending[s][0]
                if slot is None:
                    if (req.stream, req.seq) not in waited:
                        waited.add((req.stream, req.seq))
                        stats.deferred += 1
                    continue
                pending[s].popleft()
                handle = self.backend.submit(s, slot["handle"], req, keep(req) if keep else False)
                slot["job"] = handle
                inflight.append({"req": req, "slot": slot, "handle": handle, "start": now})
                stats.peak_bytes = max(stats.peak_bytes, self.used_bytes)
                admitted = True
            if heads and not admitted and not inflight:
                # nothing runs and nothing could be admitted: every slot is
                # idle and eviction already failed, so no later pass can
                # succeed (the backend's memory is held by someone else);
                # reject the oldest waiting frame instead of waiting forever
                _, s = heads[0]
                pending[s].popleft()
                stats.rejected += 1
                continue
            next_arrival = trace[i].arrival if i < len(trace) else None
            if next_arrival is not None and not inflight and not any(pending.values()):
                self.backend.wait_until(next_arrival)
            else:
                self.backend.idle(next_arrival)
        stats.evictions = self.evictions
        if release:
            self.close()
        return stats

    def close(self):
        """Returns every slot of this server to the backend (all are idle
        once run() has drained its trace)."""
        for s in list(self.slots):
            for slot in self.slots[s]:
                self.backend.free_slot(slot["handle"])
                self.used_bytes -= self.sizes[s]
            self.slots[s] = []


class FakeBackend:
    """Virtual clock; a frame takes N*D / rate seconds, frames overlap
    freely (CPU tests of the scheduling logic)."""

    def __init__(self, specs, mdes_per_s: float = 1e5, arena_bytes: Optional[int] = None,
                 npaths: int = 8, p2: int = 120):
        self.specs = specs
        self.rate = mdes_per_s * 1e6
        self.t = 0.0
        self.live = {}
        self.result_of = {}
        self.submitted = []
        self.arena = Arena(arena_bytes) if arena_bytes else None
        self.sizes = [slot_bytes(sp, npaths, p2) for sp in specs]

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def alloc_slot(self, s):
        off = None
        if self.arena is not None:
            off = self.arena.alloc(self.sizes[s])
            if off is None:
                return None
        self.allocs = getattr(self, "allocs", 0) + 1
        return ("slot", s, off)

    def free_slot(self, handle):
        if self.arena is not None:
            self.arena.release(handle[2], self.sizes[handle[1]])
        self.frees = getattr(self, "frees", 0) + 1

    def submit(self, s, slot, req, keep):
        sp = self.specs[s]
        handle = object()
        self.live[handle] = self.t + sp.width * sp.height * sp.ndisp / self.rate
        self.submitted.append((self.t, req))
        return handle

    def done(self, handle):
        t = self.live[handle]
        return t if t <= self.t else None

    def idle(self, next_arrival=None):
        pending = [t for t in self.live.values() if t > self.t]
        if next_arrival is not None and next_arrival > self.t:
            pending.append(next_arrival)
        self.t = min(pending) if pending else self.t + 1e-4

    def wait_until(self, t):
        self.t = max(self.t, t)


class GpuBackend:
    """Slots are StereoSGM buffer sets, with their own device inputs, carved
    out of one device arena; frames run on a fixed pool of HIP streams
    (default priority).  Everything a slot needs besides its arena range --
    its stream and its pinned output buffer -- is made once, up front, and
    reused, so admitting a slot (also after an eviction) allocates nothing."""

    def __init__(self, specs, params, frames_per_stream: int = 4, device="cuda", occlusion=0.05,
                 arena_bytes: int = 8 << 30, hip_streams: int = 8, slots_per_stream: int = 2):
        import torch

        from . import sgm
        self.torch, self.sgm = torch, sgm
        self.specs, self.params, self.device = specs, params, torch.device(device)
        self.pool = []      # pinned host frames per stream
        for s in specs:
            frames = []
            for k in range(frames_per_stream):
                pair = datagen.make_pair(s.width, s.height, s.ndisp, s.seed * 10 + k, (8, 16), occlusion)
                frames.append((torch.from_numpy(pair["left"]).pin_memory(),
                               torch.from_numpy(pair["right"]).pin_memory()))
            self.pool.append(frames)
        self.sizes = [slot_bytes(sp, params.npaths, params.p2) for sp in specs]
        self.arena = Arena(arena_bytes)
        # the one device allocation of the server: every slot lives in it
        self.memory = torch.empty(self.arena.capacity + Arena.ALIGN, dtype=torch.uint8,
                                  device=self.device)
        self.base = (-self.memory.data_ptr()) % Arena.ALIGN
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(hip_streams)]
        self._next_stream = 0
        # pinned host buffers for D, per stream spec, one per possible slot
        self.out_pool = [[torch.empty((sp.height, sp.width), dtype=torch.uint16).pin_memory()
                          for _ in range(slots_per_stream)] for sp in specs]
        self.result_of = {}
        self.t0_event = None
        self.t0 = 0.0

    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record()
        # the host clock starts once the event's timestamp is taken, so that
        # device completion times and host arrival times share one origin
        self.t0_event.synchronize()
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def alloc_slot(self, s):
        """A slot's buffers carved from the arena, or None if they do not fit
        in one free range."""
        torch, sgm = self.torch, self.sgm
        sp = self.specs[s]
        if not self.out_pool[s]:
            return None
        off = self.arena.alloc(self.sizes[s])
        if off is None:
            return None
        cursor = [self.base + off]

        def take(nbytes):
            start = cursor[0]
            cursor[0] += _a256(nbytes)
            return self.memory[start: start + nbytes]

        n = sp.width * sp.height
        prm = sgm.Params(**{**self.params.__dict__, "ndisp": sp.ndisp})
        left = take(n).view(sp.height, sp.width)
        right = take(n).view(sp.height, sp.width)
        eng = sgm.StereoSGM(sp.width, sp.height, prm, device=self.device, alloc=take)
        assert cursor[0] - self.base - off <= self.sizes[s], "slot layout exceeds slot_bytes"
        return {"eng": eng, "left": left, "right": right, "off": off, "stream_index": s,
                "out": self.out_pool[s].pop()}

    def submit(self, s, slot, req, keep):
        torch = self.torch
        hl, hr = self.pool[s][req.frame]
        # streams in turn: with fewer frames in flight than streams, two
        # frames in flight never share one
        st = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        with torch.cuda.stream(st):
            slot["left"].copy_(hl, non_blocking=True)
            slot["right"].copy_(hr, non_blocking=True)
            slot["eng"].run(slot["left"], slot["right"], stream=st)
            slot["out"].copy_(slot["eng"].disp, non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        return {"event": ev, "slot": slot, "req": req, "keep": keep}

    def done(self, handle):
        ev = handle["event"]
        if not ev.query():
            return None
        if handle["keep"]:
            r = handle["req"]
            self.result_of[(r.stream, r.seq)] = handle["slot"]["out"].numpy().copy()
        return self.t0_event.elapsed_time(ev) * 1e-3

    def free_slot(self, handle):
        # only idle slots are released: their last frame has completed
        self.arena.release(handle["off"], self.sizes[handle["stream_index"]])
        self.out_pool[handle["stream_index"]].append(handle["out"])
        handle.clear()

    def idle(self, next_arrival=None):
        time.sleep(5e-5)

    def wait_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.01))


def serve_plain(trace, specs, backend) -> Stats:
    """FIFO reference: one frame at a time, in arrival order, one stream, one
    slot per stream (within the backend's arena)."""
    srv = Server(specs, backend, budget_bytes=backend.arena.capacity if getattr(
        backend, "arena", None) is not None else 1 << 62, hip_streams=1, max_slots_per_stream=1)
    return srv.run(trace)
