"""Binding of the library's fit server (lasp_server_*): argument marshalling
and request bookkeeping only.

The server itself is native (csrc/lasp_server.hip): a worker thread admits
requests by HBM footprint against one device-wide budget, grows and shrinks
one slot pool per spectral shape inside that budget, advances every
resident fit of a shape with one launch sequence per tick (the shapes on
streams of their own, overlapping on the device), and evaluates finished
requests into the caller's output tensors.  This module allocates those
output tensors, keeps each request's tensors alive until the server reports
it done, and converts the server's timestamps into latencies.
"""

from __future__ import annotations

import ctypes
import dataclasses
import time

import numpy as np
import torch

from .lasp import (N_BASIS, N_PAR, Arms, RequestInfo, ServerCounters, ServerOpts, _check, _dev,
                   _grid, _ptr, load, make_opts)


@dataclasses.dataclass
class Request:
    rid: int
    shape: int
    obs: torch.Tensor              # [n, P] device (kept alive until done)
    ivar: torch.Tensor
    init: torch.Tensor             # [n, 5] device
    params: torch.Tensor           # [n, 5] float32 device output
    status: torch.Tensor           # [n] int32 device output
    chi2: torch.Tensor             # [n] float64 device output
    cov: torch.Tensor | None = None
    t_arrival: float | None = None  # scheduled arrival, server clock (s)
    info: RequestInfo | None = None

    @property
    def n(self) -> int:
        return self.obs.shape[0]

    @property
    def latency_s(self) -> float:
        """Arrival (or submit) to results complete in device memory."""
        t0 = self.info.t_submit if self.t_arrival is None else min(self.t_arrival,
                                                                  self.info.t_submit)
        return self.info.t_done - t0


class Server:
    """lasp_server_* on the current device."""

    def __init__(self, *, hbm_budget: int = 0, n_steps: int = 500, steps_per_tick: int = 25,
                 want_cov: bool = False, capacity_quantum: int = 1024, device=None):
        lib = load()
        o = ServerOpts()
        lib.lasp_server_default_opts(ctypes.byref(o))
        o.hbm_budget = int(hbm_budget)
        o.n_steps, o.steps_per_tick = int(n_steps), int(steps_per_tick)
        o.want_cov, o.capacity_quantum = int(bool(want_cov)), int(capacity_quantum)
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.want_cov = bool(want_cov)
        self.n_steps = int(n_steps)
        self._s = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.lasp_server_create(ctypes.byref(o), ctypes.byref(self._s)))
        self._t0 = time.perf_counter()        # the server clock's origin, this process's clock
        self._pending: dict[int, Request] = {}
        self._shapes: list[int] = []           # pixels per shape
        self._keep = []                        # host grids of the shapes

    def clock(self) -> float:
        """Seconds on the server's clock (approximately)."""
        return time.perf_counter() - self._t0

    def add_shape(self, wave_grid, basis, *, margin=64, degree=10, precision="fp32", lr=1e-2,
                  betas=(0.9, 0.999), eps=1e-8, weight_quantile=0.5, arms: Arms | None = None,
                  box=None, stop_window=0, stop_tol=1e-5, n_classes=1, class_edges=None) -> int:
        P = int(np.asarray(wave_grid).shape[0])
        _dev(basis, "basis", torch.float32, (N_BASIS * n_classes, P + 2 * margin))
        grid = _grid(wave_grid, P)
        opts = make_opts(1, P, margin=margin, degree=degree, precision=precision, lr=lr,
                         betas=betas, eps=eps, weight_quantile=weight_quantile, arms=arms,
                         box=box, stream=torch.cuda.current_stream(self.device),
                         stop_window=stop_window, stop_tol=stop_tol, n_classes=n_classes,
                         class_edges=class_edges)
        sid = ctypes.c_int32()
        torch.cuda.current_stream(self.device).synchronize()   # basis ready
        with torch.cuda.device(self.device):
            _check(load().lasp_server_add_shape(self._s, grid.ctypes.data_as(ctypes.c_void_p),
                                                _ptr(basis), ctypes.byref(opts),
                                                ctypes.byref(sid)))
        self._shapes.append(P)
        self._keep.append(grid)
        return int(sid.value)

    def submit(self, shape: int, obs, ivar, init_params, t_arrival: float | None = None) -> Request:
        """Queue a group of spectra (device tensors whose producing work has
        finished).  t_arrival: scheduled arrival on the server clock, for the
        latency (defaults to the submit time)."""
        n, P = obs.shape
        if shape < 0 or shape >= len(self._shapes) or P != self._shapes[shape]:
            raise ValueError("obs does not match the shape's pixel count")
        _dev(obs, "obs", torch.float32, (n, P))
        _dev(ivar, "ivar", torch.float32, (n, P))
        _dev(init_params, "init_params", torch.float32, (n, N_PAR))
        dev = obs.device
        req = Request(-1, shape, obs, ivar, init_params,
                      torch.empty((n, N_PAR), dtype=torch.float32, device=dev),
                      torch.empty(n, dtype=torch.int32, device=dev),
                      torch.empty(n, dtype=torch.float64, device=dev),
                      torch.empty((n, N_PAR, N_PAR), dtype=torch.float64, device=dev)
                      if self.want_cov else None, t_arrival)
        # the server's stream must not overtake work on this stream that
        # produced the inputs or last used the outputs' memory
        torch.cuda.current_stream(dev).synchronize()
        rid = ctypes.c_int64()
        _check(load().lasp_server_submit(self._s, int(shape), int(n), _ptr(obs), _ptr(ivar),
                                         _ptr(init_params), _ptr(req.params), _ptr(req.cov),
                                         _ptr(req.status), _ptr(req.chi2), ctypes.byref(rid)))
        req.rid = int(rid.value)
        self._pending[req.rid] = req
        return req

    def poll(self, timeout_ms: int = 0, max_done: int = 256) -> list[Request]:
        """Requests finished since the last poll (their outputs are complete)."""
        buf = (RequestInfo * max_done)()
        n = ctypes.c_int32()
        _check(load().lasp_server_poll(self._s, buf, int(max_done), int(timeout_ms),
                                       ctypes.byref(n)))
        out = []
        for i in range(n.value):
            info = RequestInfo.from_buffer_copy(buf[i])
            req = self._pending.pop(int(info.id))
            req.info = info
            out.append(req)
        return out

    def stats(self) -> dict:
        c = ServerCounters()
        _check(load().lasp_server_stats(self._s, ctypes.byref(c)))
        d = {f: getattr(c, f) for f, _ in ServerCounters._fields_}
        d["capacity"] = list(c.capacity)[:c.n_shapes]
        d["used_slots"] = list(c.used_slots)[:c.n_shapes]
        return d

    def busy(self) -> bool:
        return bool(self._pending)

    def run(self, arrivals, t_end: float | None = None, stall_s: float = 60.0) -> list[Request]:
        """Serve a schedule: ``arrivals`` is a sorted list of (offset s,
        factory) where factory() returns (shape, obs, ivar, init).  Each
        request is submitted once its offset has passed on the server clock
        (counted from this call) and carries that offset as its arrival.
        Returns the finished requests; raises if nothing finishes for
        stall_s seconds while requests are pending."""
        done = []
        start = self.clock()
        last = start
        i = 0
        while i < len(arrivals) or self._pending:
            now = self.clock() - start
            if self._pending and self.clock() - last > stall_s:
                raise RuntimeError(f"no request finished in {stall_s} s: {self.stats()}")
            while i < len(arrivals) and arrivals[i][0] <= now:
                shape, obs, ivar, init = arrivals[i][1]()
                self.submit(shape, obs, ivar, init, t_arrival=start + arrivals[i][0])
                i += 1
            wait = 2
            if i < len(arrivals):
                wait = int(max(0.0, min(0.002, arrivals[i][0] - now)) * 1e3)
            got = self.poll(timeout_ms=wait)
            if got:
                last = self.clock()
                done.extend(got)
            if t_end is not None and now > t_end:
                break
        return done

    def close(self):
        if self._s:
            load().lasp_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
