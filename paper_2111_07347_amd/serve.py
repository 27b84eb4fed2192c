"""Serving loop: continuous batching of streamed scan rows against resident
template libraries (the real-time, on-line indexing use of the method that
the paper's discussion anticipates: one pattern in a few to tens of
milliseconds, comparable to a detector's acquisition time).

A detector releases scan rows (requests) over time, each to be indexed
against one of several libraries kept resident on the GPU. The scheduler:

* queues requests first in, first out;
* admits work whenever a stream slot is free and the HBM footprint of all
  work in flight plus the new batch stays within a budget (a request larger
  than the whole budget is rejected);
* batches continuously: when a slot frees up it takes the oldest queued
  request and, behind it, further queued requests for the same library (up to
  a row limit), so rows that arrived while others were on the GPU join the
  next launch;
* runs each batch on its own HIP stream (polar transform and match kernels of
  different batches overlap on the device) and timestamps completion.

Every pattern's result is independent of what it is batched with (the
kernels compute each pattern alone, in a fixed order), so a row's result is
identical alone and in the mix.

`Scheduler` is pure bookkeeping (testable without a GPU); `GpuExecutor` does
the device work through the libtm binding; `Server` joins them.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable

import numpy as np


class BudgetError(ValueError):
    """A request whose footprint exceeds the whole HBM budget."""


@dataclasses.dataclass
class Request:
    req_id: int
    lib_id: int
    n_patterns: int
    t_arrival: float
    payload: object = None       # host rows [n, H, W] (pinned torch tensor) or test data
    nbytes: int = 0              # device footprint of this request alone


@dataclasses.dataclass
class Result:
    req_id: int
    lib_id: int
    top_template: np.ndarray
    top_angle: np.ndarray
    top_score: np.ndarray
    t_arrival: float
    t_admit: float
    t_done: float
    batch_id: int
    batch_rows: int
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclasses.dataclass
class Batch:
    batch_id: int
    slot: int
    lib_id: int
    requests: list
    nbytes: int
    t_admit: float
    timed_out: bool = False


class Scheduler:
    """FIFO queue, slot and HBM-budget admission, same-library batching."""

    def __init__(self, budget_bytes: int, slots: int, max_batch_rows: int = 4):
        if slots < 1 or max_batch_rows < 1 or budget_bytes <= 0:
            raise ValueError("need slots >= 1, max_batch_rows >= 1, budget_bytes > 0")
        self.budget = int(budget_bytes)
        self.slots = slots
        self.max_batch_rows = max_batch_rows
        self.queue: collections.deque = collections.deque()
        self.free_slots = list(range(slots))
        self.inflight: dict = {}
        self.used = 0
        self._next_batch = 0

    def push(self, req: Request):
        if req.nbytes > self.budget:
            raise BudgetError(f"request {req.req_id} needs {req.nbytes} bytes, budget {self.budget}")
        self.queue.append(req)

    def cancel(self, req_id: int) -> bool:
        """Drop a queued (not yet admitted) request."""
        for r in self.queue:
            if r.req_id == req_id:
                self.queue.remove(r)
                return True
        return False

    def admit(self, now: float) -> Batch | None:
        """Next batch to launch, or None (no free slot, empty queue, or the
        head request does not fit the remaining budget)."""
        if not self.free_slots or not self.queue:
            return None
        head = self.queue[0]
        if self.used + head.nbytes > self.budget:
            return None
        picked = [head]
        nbytes = head.nbytes
        for r in list(self.queue)[1:]:
            if len(picked) >= self.max_batch_rows:
                break
            if r.lib_id == head.lib_id and self.used + nbytes + r.nbytes <= self.budget:
                picked.append(r)
                nbytes += r.nbytes
        for r in picked:
            self.queue.remove(r)
        slot = self.free_slots.pop(0)
        b = Batch(self._next_batch, slot, head.lib_id, picked, nbytes, now)
        self._next_batch += 1
        self.inflight[slot] = b
        self.used += nbytes
        return b

    def complete(self, slot: int) -> Batch:
        b = self.inflight.pop(slot)
        self.used -= b.nbytes
        self.free_slots.append(slot)
        self.free_slots.sort()
        return b

    @property
    def idle(self) -> bool:
        return not self.queue and not self.inflight


class GpuExecutor:
    """Device work of a batch on the slot's stream: host-to-device copy of the
    rows, polar transform, match (plain; or, for the libraries listed in
    `bound`, the exact search with window upper bounds, or, for those in
    `fourier`, the Fourier route with certified rescoring, both of which give
    the plain path's top-N; or pre-filtered in reduced precision with exact
    rescoring), device-to-host copy of the top-N, completion event."""

    def __init__(self, libraries: dict, grid, N: int, slots: int, gamma: float = 1.0,
                 subtract: float = 0.0, prefilter_keep: float = 0.0, precision: str = "bf16",
                 fourier=(), bound=()):
        import torch

        import paper_2111_07347_amd as tm
        self.tm = tm
        self.torch = torch
        self.libraries = libraries
        self.grid = grid
        self.N = N
        self.gamma = gamma
        self.subtract = subtract
        self.keep = prefilter_keep
        self.precision = precision
        self.fourier = set(fourier)     # library ids loaded with spectra (Library(fft=True))
        self.bound = set(bound)         # library ids searched with window bounds
        self.streams = [torch.cuda.Stream() for _ in range(slots)]   # default priority
        self.events = [None] * slots
        self.outputs = [None] * slots

    def footprint(self, n_patterns: int, H: int, W: int, itemsize: int, lib_id: int) -> int:
        """Device bytes one request of n_patterns holds while in flight."""
        R, nt = self.grid.R, self.grid.n_theta
        rows = self.libraries[lib_id].rows()[0] or R       # compact polar: touched rows
        b = n_patterns * (H * W * itemsize + rows * nt * 4 + 8 + R * 4 + self.N * 12)
        if lib_id in self.bound:
            # bounds in chunk-slot order, candidate lists (at most 10 % of
            # T') and the split launches' partial lists
            Tp = self.libraries[lib_id].n_total
            b += n_patterns * (Tp + 64) * 4 + n_patterns * (Tp // 10 + 1) * 4 + (16384 * self.N * 12)
        elif lib_id in self.fourier:
            # stored C(k) (float16 re/im per frequency and template, chunked
            # to 2 GiB), approximate scores and the certified candidate lists
            lib = self.libraries[lib_id]
            Tp, Fp = lib.n_total, nt // 2 + 1
            b += min(n_patterns * Fp * Tp * 4, 2 << 30) + n_patterns * Tp * 8
        elif self.keep > 0.0:
            T = self.libraries[lib_id].T
            n_keep = int(np.ceil(self.keep * T))
            b += n_patterns * (T * 4 + 2 * n_keep * 4)
        return int(b)

    def launch(self, batch: Batch):
        torch, tm = self.torch, self.tm
        s = self.streams[batch.slot]
        lib = self.libraries[batch.lib_id]
        rows = [r.payload for r in batch.requests]
        n = sum(h.shape[0] for h in rows)
        with torch.cuda.stream(s):
            x = torch.empty((n,) + tuple(rows[0].shape[1:]), dtype=rows[0].dtype, device="cuda")
            o = 0
            for h in rows:
                x[o:o + h.shape[0]].copy_(h, non_blocking=True)
                o += h.shape[0]
            polar, norms, prof = tm.polar_transform(x, self.grid, self.gamma, self.subtract,
                                                    want_profile=self.keep > 0.0, lib=lib)
            if batch.lib_id in self.bound:
                tt, ts, tq = tm.match_batch(lib, polar, norms, self.N, coarse="bound")
            elif batch.lib_id in self.fourier:
                tt, ts, tq = tm.match_batch(lib, polar, norms, self.N, coarse="fft")
            elif self.keep > 0.0:
                tt, ts, tq = tm.match_batch(lib, polar, norms, self.N, profiles=prof,
                                            prefilter_keep=self.keep, prefilter_prec=self.precision)
            else:
                tt, ts, tq = tm.match_batch(lib, polar, norms, self.N)
            host = [torch.empty(o.shape, dtype=o.dtype, pin_memory=True) for o in (tt, ts, tq)]
            for h, o in zip(host, (tt, ts, tq)):
                h.copy_(o, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # keep device tensors alive until the stream has finished with them
        self.outputs[batch.slot] = (host, (x, polar, norms, prof, tt, ts, tq))
        self.events[batch.slot] = ev

    def done(self, slot: int) -> bool:
        ev = self.events[slot]
        return ev is not None and ev.query()

    def collect(self, batch: Batch):
        host, _ = self.outputs[batch.slot]
        self.outputs[batch.slot] = None
        self.events[batch.slot] = None
        tt, ts, tq = (h.numpy() for h in host)
        out, o = [], 0
        for r in batch.requests:
            out.append((tt[o:o + r.n_patterns].copy(), ts[o:o + r.n_patterns].copy(),
                        tq[o:o + r.n_patterns].copy()))
            o += r.n_patterns
        return out


class Server:
    """Event loop joining a Scheduler and an executor (GpuExecutor or any
    object with launch/done/collect)."""

    def __init__(self, executor, budget_bytes: int, slots: int, max_batch_rows: int = 4,
                 clock: Callable[[], float] = time.perf_counter, timeout_s: float | None = None):
        self.ex = executor
        self.sched = Scheduler(budget_bytes, slots, max_batch_rows)
        self.clock = clock
        self.timeout_s = timeout_s
        self._next_id = 0
        self.results: list = []

    def submit(self, payload, lib_id: int, n_patterns: int, nbytes: int,
               t_arrival: float | None = None) -> int:
        rid = self._next_id
        self._next_id += 1
        t = self.clock() if t_arrival is None else t_arrival
        self.sched.push(Request(rid, lib_id, n_patterns, t, payload, nbytes))
        return rid

    def _fail(self, b: Batch, msg: str, now: float) -> list:
        empty = np.zeros((0,), dtype=np.int32)
        return [Result(r.req_id, r.lib_id, empty, empty, empty.astype(np.float32), r.t_arrival,
                       b.t_admit, now, b.batch_id, len(b.requests), msg) for r in b.requests]

    def step(self) -> list:
        """Collect finished batches, report overdue ones (watchdog), then admit
        as many as fit. Returns the results finished in this step."""
        finished = []
        for slot in list(self.sched.inflight):
            b = self.sched.inflight[slot]
            if self.ex.done(slot):
                self.sched.complete(slot)
                t_done = self.clock()
                outs = self.ex.collect(b)
                if b.timed_out:
                    continue          # already reported; the slot is free again now
                for r, (tt, ts, tq) in zip(b.requests, outs):
                    finished.append(Result(r.req_id, r.lib_id, tt, ts, tq, r.t_arrival,
                                           b.t_admit, t_done, b.batch_id, len(b.requests)))
            elif (self.timeout_s is not None and not b.timed_out
                  and self.clock() - b.t_admit > self.timeout_s):
                # device work cannot be recalled: report the requests as failed
                # and keep the slot (and its budget) until the work finishes
                b.timed_out = True
                finished += self._fail(b, "timeout", self.clock())
        while True:
            b = self.sched.admit(self.clock())
            if b is None:
                break
            try:
                self.ex.launch(b)
            except Exception as e:     # a failed launch frees its slot at once
                self.sched.complete(b.slot)
                finished += self._fail(b, f"launch failed: {e}", self.clock())
        self.results.extend(finished)
        return finished

    def drain(self, poll_s: float = 2e-4, sleep: Callable[[float], None] = time.sleep) -> list:
        out = []
        while not self.sched.idle:
            out += self.step()
            if not self.sched.idle:
                sleep(poll_s)
        return out


def latency_report(results: list) -> dict:
    results = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in results]) * 1e3
    n = sum(len(r.top_template) for r in results)
    if len(lat) == 0:
        return {}
    span = max(r.t_done for r in results) - min(r.t_arrival for r in results)
    return {"rows": len(results), "patterns": int(n),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "sustained_patterns_per_s": round(float(n / span), 1) if span > 0 else None,
            "mean_batch_rows": round(float(np.mean([r.batch_rows for r in results])), 3)}


def run_stream(server: Server, rows: list, lib_ids, arrivals, poll_s: float = 2e-4) -> list:
    """Replay a detector stream: request i (host rows[i], library lib_ids[i])
    is submitted at t0 + arrivals[i]; the server is stepped in between. All
    arrivals equal to 0 is burst mode. Returns every result."""
    t0 = server.clock()
    i = 0
    n = len(rows)
    while i < n or not server.sched.idle:
        now = server.clock()
        while i < n and now >= t0 + arrivals[i]:
            h = rows[i]
            server.submit(h, int(lib_ids[i]), h.shape[0],
                          server.ex.footprint(h.shape[0], h.shape[1], h.shape[2],
                                              h.element_size(), int(lib_ids[i])),
                          t_arrival=t0 + arrivals[i])
            i += 1
        server.step()
        if i < n or not server.sched.idle:
            time.sleep(poll_s)
    return server.results


class PinnedIndexer:
    """End-to-end indexing of a pattern stack held in pinned host memory
    (the paper's GPU timing counts the transfer of the images to the device
    and of the results back).

    The stack is cut into chunks. Chunk i + 1 is copied to the device on a
    copy stream while chunk i is transformed and matched on the compute
    stream, from two alternating device buffers; each chunk's top-N rows go
    back to pinned host memory on the compute stream. Both streams have the
    default priority. Device buffers are allocated once, at construction,
    and reused by every call."""

    def __init__(self, lib, grid, N: int, chunk: int, H: int, W: int, dtype,
                 gamma: float = 1.0, subtract: float = 0.0, **match_kw):
        import torch

        import paper_2111_07347_amd as tm
        self.tm, self.torch = tm, torch
        self.lib, self.grid, self.N, self.chunk = lib, grid, N, chunk
        self.gamma, self.subtract, self.match_kw = gamma, subtract, match_kw
        dev = torch.device("cuda")
        self.want_profile = match_kw.get("prefilter_keep", 0.0) > 0.0
        n_rows = lib.rows()[0] or grid.R
        self.xbuf = [torch.empty((chunk, H, W), dtype=dtype, device=dev) for _ in range(2)]
        self.polar = torch.empty((chunk, n_rows, grid.n_theta), dtype=torch.float32, device=dev)
        self.norms = torch.empty((chunk,), dtype=torch.float64, device=dev)
        self.prof = (torch.empty((grid.R, chunk), dtype=torch.float32, device=dev)
                     if self.want_profile else None)
        self.out = (torch.empty((chunk, N), dtype=torch.int32, device=dev),
                    torch.empty((chunk, N), dtype=torch.int32, device=dev),
                    torch.empty((chunk, N), dtype=torch.float32, device=dev))
        self.copy_s = torch.cuda.Stream()
        self.comp_s = torch.cuda.Stream()

    def __call__(self, host, results=None):
        """Index host [B, H, W] (pinned); returns pinned host (template,
        angle, score) [B, N] after the work has finished."""
        torch, tm = self.torch, self.tm
        B = host.shape[0]
        if results is None:
            results = tuple(torch.empty((B, self.N), dtype=d, pin_memory=True)
                            for d in (torch.int32, torch.int32, torch.float32))
        n_chunks = -(-B // self.chunk)
        x_free = [None, None]               # compute done reading buffer i
        for c in range(n_chunks):
            lo, hi = c * self.chunk, min(B, (c + 1) * self.chunk)
            n = hi - lo
            k = c % 2
            xb = self.xbuf[k][:n]
            with torch.cuda.stream(self.copy_s):
                if x_free[k] is not None:
                    self.copy_s.wait_event(x_free[k])
                xb.copy_(host[lo:hi], non_blocking=True)
                copied = torch.cuda.Event()
                copied.record(self.copy_s)
            with torch.cuda.stream(self.comp_s):
                self.comp_s.wait_event(copied)
                polar, norms = self.polar[:n], self.norms[:n]
                prof = None
                if self.want_profile:
                    prof = self.prof if n == self.chunk else torch.empty(
                        (self.grid.R, n), dtype=torch.float32, device=xb.device)
                tm.polar_transform(xb, self.grid, self.gamma, self.subtract, polar_out=polar,
                                   norm_out=norms, profile_out=prof,
                                   want_profile=self.want_profile, lib=self.lib)
                ev = torch.cuda.Event()
                ev.record(self.comp_s)
                x_free[k] = ev
                out = tuple(o[:n] for o in self.out)
                kw = dict(self.match_kw)
                if self.want_profile:
                    kw["profiles"] = prof
                tm.match_batch(self.lib, polar, norms, self.N, out=out, **kw)
                for h, o in zip(results, out):
                    h[lo:hi].copy_(o, non_blocking=True)
        self.comp_s.synchronize()
        self.copy_s.synchronize()
        return results
