"""Continuous batching of fit requests over device-resident slot pools.

Each spectral shape (pixel count, grid, basis, arms) has a ``Pool`` of fit
slots on its own HIP stream.  A request (a group of spectra of one shape) is
admitted when its memory footprint (spectra x bytes per slot) fits in a
contiguous free slot range, loaded into those slots (per-slot Adam state
starts at step 0), and then advances together with every other resident fit
each tick (k Adam steps per tick, one launch sequence per shape, the shapes'
streams overlapping on the device).  When a request has taken its n_steps,
its slots are evaluated, the results are copied to pinned host memory and,
once that copy has completed, the slots are freed for queued requests.  With
the stopping rules on (a pool created with stop_window > 0) a request also
finishes as soon as every one of its fits has stopped: each tick enqueues a
copy of the pool's per-slot stopped flags to pinned memory and a later tick
reads it.

All arithmetic runs in the library's kernels; this module is bookkeeping:
slot allocation, queues, tick pacing and latency timestamps.
"""

from __future__ import annotations

import bisect
import dataclasses
import time
from collections import deque

import torch

from .lasp import N_PAR, Pool


class SlotAllocator:
    """First-fit allocator of contiguous slot ranges in [0, capacity)."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free = [(0, capacity)]          # sorted, disjoint (start, length)
        self.used = {}                       # start -> length

    def alloc(self, n: int):
        for i, (s, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, l - n)
                self.used[s] = n
                return s
        return None

    def release(self, start: int):
        n = self.used.pop(start)
        i = bisect.bisect_left(self.free, (start, 0))
        self.free.insert(i, (start, n))
        merged = []
        for s, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((s, l))
        self.free = merged

    def high_water(self) -> int:
        return max((s + l for s, l in self.used.items()), default=0)

    def used_slots(self) -> int:
        return sum(self.used.values())


@dataclasses.dataclass
class Request:
    rid: int
    lane: str
    obs: torch.Tensor          # [n, P] device
    ivar: torch.Tensor
    init: torch.Tensor         # [n, 5] device
    t_arrival: float
    slot0: int = -1
    steps: int = 0
    t_admit: float = 0.0
    t_done: float = 0.0
    admit_tick: int = -1
    params: torch.Tensor | None = None   # pinned host results
    status: torch.Tensor | None = None
    chi2: torch.Tensor | None = None
    cov: torch.Tensor | None = None
    event: torch.cuda.Event | None = None

    @property
    def n(self) -> int:
        return self.obs.shape[0]


class Lane:
    """One shape: its pool, allocator, queue and resident requests."""

    def __init__(self, name: str, pool: Pool):
        self.name = name
        self.pool = pool
        self.alloc = SlotAllocator(pool.capacity)
        self.queue: deque[Request] = deque()
        self.active: list[Request] = []
        self.finishing: list[Request] = []
        self.tick_event: torch.cuda.Event | None = None
        # stopped flags of the slots (stopping rules): device copy, pinned
        # host copy, the event that marks the host copy complete and the
        # tick at which the flags were taken
        self.done_dev = self.done_host = self.snap_event = None
        self.snap_tick = -1
        if pool.stop_window > 0:
            self.done_dev = torch.zeros(pool.capacity, dtype=torch.int32, device=pool.device)
            self.done_host = torch.zeros(pool.capacity, dtype=torch.int32, pin_memory=True)

    @property
    def footprint_bytes(self) -> int:
        return self.alloc.used_slots() * self.pool.slot_bytes


class Server:
    def __init__(self, lanes: dict[str, Pool], n_steps: int = 500, steps_per_tick: int = 25,
                 want_cov: bool = False):
        self.lanes = {k: Lane(k, p) for k, p in lanes.items()}
        self.n_steps = n_steps
        self.k = steps_per_tick
        self.want_cov = want_cov
        self.done: list[Request] = []
        self.ticks = 0

    def submit(self, req: Request):
        self.lanes[req.lane].queue.append(req)

    def _admit(self, lane: Lane, now: float):
        while lane.queue:
            req = lane.queue[0]
            if req.n > lane.pool.capacity:
                raise ValueError(f"request of {req.n} spectra exceeds the pool capacity")
            slot0 = lane.alloc.alloc(req.n)
            if slot0 is None:
                return                         # wait for memory to free up
            lane.queue.popleft()
            req.slot0 = slot0
            req.t_admit = now
            req.admit_tick = self.ticks
            with torch.cuda.stream(lane.pool.stream):
                lane.pool.load(slot0, req.obs, req.ivar, req.init, self.n_steps)
            lane.active.append(req)

    def _finish(self, lane: Lane, req: Request):
        dev = lane.pool.device
        n = req.n
        with torch.cuda.stream(lane.pool.stream):
            p = torch.empty((n, N_PAR), dtype=torch.float32, device=dev)
            st = torch.empty(n, dtype=torch.int32, device=dev)
            c2 = torch.empty(n, dtype=torch.float64, device=dev)
            cv = (torch.empty((n, N_PAR, N_PAR), dtype=torch.float64, device=dev)
                  if self.want_cov else None)
            lane.pool.finish(req.slot0, p, cv, st, c2)
            req.params = torch.empty((n, N_PAR), dtype=torch.float32, pin_memory=True)
            req.status = torch.empty(n, dtype=torch.int32, pin_memory=True)
            req.chi2 = torch.empty(n, dtype=torch.float64, pin_memory=True)
            req.params.copy_(p, non_blocking=True)
            req.status.copy_(st, non_blocking=True)
            req.chi2.copy_(c2, non_blocking=True)
            if cv is not None:
                req.cov = torch.empty((n, N_PAR, N_PAR), dtype=torch.float64, pin_memory=True)
                req.cov.copy_(cv, non_blocking=True)
            req.event = torch.cuda.Event()
            req.event.record(lane.pool.stream)
        lane.finishing.append(req)

    def tick(self, now: float):
        """Admit, advance every resident fit by k steps, start finished ones."""
        for lane in self.lanes.values():
            self._admit(lane, now)
        for lane in self.lanes.values():
            if not lane.active:
                continue
            prev = lane.tick_event
            with torch.cuda.stream(lane.pool.stream):
                k = min(self.k, max(self.n_steps - r.steps for r in lane.active))
                lane.pool.step(lane.alloc.high_water(), k)
                for r in lane.active:
                    r.steps += k
                fin = [r for r in lane.active if r.steps >= self.n_steps]
                if lane.snap_event is not None and lane.snap_event.query():
                    flags = lane.done_host.numpy()
                    for r in lane.active:
                        # flags taken before r was loaded belong to older fits
                        if (r not in fin and r.admit_tick <= lane.snap_tick
                                and flags[r.slot0:r.slot0 + r.n].all()):
                            fin.append(r)
                    lane.snap_event = None
                for r in fin:
                    lane.active.remove(r)
                    self._finish(lane, r)
                if lane.done_dev is not None and lane.snap_event is None and lane.active:
                    hw = lane.alloc.high_water()
                    lane.pool.progress(0, done=lane.done_dev[:hw])
                    lane.done_host[:hw].copy_(lane.done_dev[:hw], non_blocking=True)
                    lane.snap_event = torch.cuda.Event()
                    lane.snap_event.record(lane.pool.stream)
                    lane.snap_tick = self.ticks
                lane.tick_event = torch.cuda.Event()
                lane.tick_event.record(lane.pool.stream)
            if prev is not None:
                prev.synchronize()             # keep at most two ticks in flight
        self.ticks += 1

    def poll(self, now: float) -> int:
        """Collect finished requests whose results reached the host."""
        n = 0
        for lane in self.lanes.values():
            for r in list(lane.finishing):
                if r.event.query():
                    r.t_done = now
                    lane.finishing.remove(r)
                    lane.alloc.release(r.slot0)
                    self.done.append(r)
                    n += 1
        return n

    def busy(self) -> bool:
        return any(l.queue or l.active or l.finishing for l in self.lanes.values())

    def run(self, arrivals, clock=time.perf_counter, t_end: float | None = None):
        """Serve ``arrivals`` (sorted list of (t_offset, Request factory))."""
        t0 = clock()
        i = 0
        while i < len(arrivals) or self.busy():
            now = clock() - t0
            while i < len(arrivals) and arrivals[i][0] <= now:
                req = arrivals[i][1]()
                req.t_arrival = t0 + arrivals[i][0]
                self.submit(req)
                i += 1
            if any(l.queue or l.active for l in self.lanes.values()):
                self.tick(clock())
            elif i < len(arrivals):
                time.sleep(min(0.002, max(0.0, arrivals[i][0] - now)))
            self.poll(clock())
            if t_end is not None and now > t_end:
                break
        return self.done
