"""Continuous-batching APSP service on one GPU.

Requests (one graph each, of any size) arrive over time.  The server:

* admits a request when its matrix fits the HBM budget next to the matrices
  already resident and a slot (a HIP stream) is free: first fit in arrival
  order, except that a request passed over ``max_bypass`` times blocks the
  ones behind it, so large requests cannot starve;
* keeps each admitted matrix in device memory from ingestion to completion;
* solves in slices of ``slice_rounds`` rounds of the blocked method
  (``apsp_solve_rounds``), at most ``inflight`` slices per request enqueued
  ahead, round-robin over the active requests; the slot streams run
  concurrently, so work of different requests overlaps on the device and a
  small request that arrives behind a large one does not wait for it;
* records, per request, arrival / admission / completion times, and reports
  p50 / p99 latency and cell updates per second.

A solve split into round slices produces exactly the bits of an unsplit one
(every slice runs the same phases on the same data), so a request's result is
the same alone and in any mix.

The scheduling logic talks to a small backend interface, so it can be tested
without a GPU (``SimBackend``); ``GpuBackend`` drives the C ABI through the
package binding.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, Optional


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    arrival: float                      # seconds on the server clock
    payload: Any = None                 # what the backend ingests (edge list ...)
    # filled in by the server
    status: str = "pending"             # pending|running|done|rejected|cancelled|failed
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Any = None
    error: Optional[str] = None
    bypassed: int = 0
    # scheduler state
    handle: Any = None
    slot: Optional[int] = None
    next_round: int = 0
    rounds: int = 0
    inflight: list = dataclasses.field(default_factory=list)   # (token, round_end)
    retries: int = 0
    slice_failed: bool = False

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class SimBackend:
    """Backend without a device: each slice takes a modelled time.

    ``rate`` is cell updates per second of one slot; a slice of rounds r0..r1
    of an n-vertex problem does (r1 - r0) * b * n^2 updates.  ``fail`` may
    name request ids whose first slice reports a device failure.
    """

    def __init__(self, rate: float = 1e12, b: int = 128, clock: Callable[[], float] = None,
                 fail: tuple = ()):
        self.rate = rate
        self.b = b
        self.clock = clock or time.perf_counter
        self.busy_until = {}
        self.fail = set(fail)
        self.allocated = 0
        self.freed = 0

    def bytes_needed(self, n: int) -> int:
        return 4 * n * n

    def num_rounds(self, n: int) -> int:
        return -(-n // self.b) if n else 0

    def alloc(self, req: Request, slot: int):
        self.allocated += 1
        return {"n": req.n}

    def free(self, handle):
        self.freed += 1

    def load(self, handle, req: Request, slot: int):
        pass

    def enqueue(self, handle, req: Request, slot: int, r0: int, r1: int):
        start = max(self.clock(), self.busy_until.get(slot, 0.0))
        kb = min(r1 * self.b, req.n) - r0 * self.b
        end = start + kb * req.n * req.n / self.rate
        self.busy_until[slot] = end
        failed = req.rid in self.fail and r0 == 0 and req.retries == 0
        return ("sim", end, failed)

    def query(self, token) -> bool:
        return self.clock() >= token[1]

    def failed(self, token) -> bool:
        return bool(token[2])

    def finish(self, handle, req: Request):
        return None


class GpuBackend:
    """Device backend: torch memory and streams, the C ABI for every solve step.

    ``payload`` of a request is an edge list (u, v, w) (undirected, one entry
    per edge) or a host matrix; it is turned into the dense device matrix on
    the request's slot stream.  With ``keep_results`` the solved matrix is
    handed to the caller in ``Request.result``; that memory is then the
    caller's and no longer counted against the server's budget.
    """

    def __init__(self, device=None, slots: int = 4, dtype: str = "f32", keep_results=True):
        import torch

        import paper_1902_04446_amd as apsp

        self.torch = torch
        self.apsp = apsp
        self.device = torch.device(device or "cuda:0")
        with torch.cuda.device(self.device):
            self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.dtype = dtype
        self.keep_results = keep_results

    def bytes_needed(self, n: int) -> int:
        return 4 * n * n

    def num_rounds(self, n: int) -> int:
        return self.apsp.num_rounds(n)

    def alloc(self, req: Request, slot: int):
        # allocated on the slot stream, where every later use of it is ordered:
        # the caching allocator then only hands out a block whose earlier uses
        # on that stream precede this request's work
        tdt = self.torch.float32 if self.dtype == "f32" else self.torch.int32
        with self.torch.cuda.stream(self.streams[slot]):
            return self.torch.empty((req.n, req.n), dtype=tdt, device=self.device)

    def free(self, handle):
        pass  # dropped with the last reference (torch's caching allocator reuses it)

    def load(self, handle, req: Request, slot: int):
        import numpy as np

        torch = self.torch
        s = self.streams[slot]
        # the matrix is used on the slot stream: the caching allocator must not
        # hand its memory out again before that stream's work is done
        handle.record_stream(s)
        with torch.cuda.stream(s):
            p = req.payload
            if isinstance(p, np.ndarray):
                handle.copy_(torch.from_numpy(p).to(self.device, non_blocking=False))
            else:
                u, v, w = p
                fill = float("inf") if handle.dtype == torch.float32 else float(self.apsp.INF_I32)
                handle.fill_(fill)
                if len(u):
                    tu = torch.as_tensor(np.asarray(u, np.int64), device=self.device)
                    tv = torch.as_tensor(np.asarray(v, np.int64), device=self.device)
                    tw = torch.as_tensor(np.asarray(w).astype(
                        np.float32 if handle.dtype == torch.float32 else np.int32),
                        device=self.device)
                    handle[tu, tv] = tw
                    handle[tv, tu] = tw
        # the solve normalises the diagonal itself (round 0)

    def enqueue(self, handle, req: Request, slot: int, r0: int, r1: int):
        s = self.streams[slot]
        self.apsp.solve_rounds(handle, r0, r1, stream=s)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return ev

    def query(self, token) -> bool:
        return token.query()

    def failed(self, token) -> bool:
        return False

    def finish(self, handle, req: Request):
        return handle if self.keep_results else None


class ApspServer:
    def __init__(self, backend, hbm_budget: int, slots: int = 4, slice_rounds: int = 8,
                 inflight: int = 2, max_bypass: int = 8, max_retries: int = 1,
                 clock: Callable[[], float] = None):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.slots = slots
        self.slice_rounds = max(1, slice_rounds)
        self.inflight = max(1, inflight)
        self.max_bypass = max_bypass
        self.max_retries = max_retries
        self.clock = clock or time.perf_counter
        self.pending: collections.deque = collections.deque()
        self.active: list = []
        self.finished: list = []
        self.used = 0
        self.free_slots = list(range(slots))

    # ---------------------------------------------------------------- API
    def submit(self, req: Request):
        if self.backend.bytes_needed(req.n) > self.budget:
            req.status = "rejected"
            req.error = "matrix larger than the HBM budget"
            self.finished.append(req)
            return req
        self.pending.append(req)
        return req

    def cancel(self, rid: int) -> bool:
        for q in (self.pending,):
            for r in list(q):
                if r.rid == rid:
                    q.remove(r)
                    r.status = "cancelled"
                    self.finished.append(r)
                    return True
        for r in self.active:
            if r.rid == rid:
                r.status = "cancelled"  # released once its enqueued slices drain
                return True
        return False

    def idle(self) -> bool:
        return not self.pending and not self.active

    # ------------------------------------------------------------ one tick
    def step(self, now: Optional[float] = None) -> list:
        now = self.clock() if now is None else now
        done_now = self._poll(now)
        self._admit(now)
        self._issue()
        return done_now

    def _release(self, req: Request):
        self.used -= self.backend.bytes_needed(req.n)
        self.free_slots.append(req.slot)
        self.backend.free(req.handle)
        req.slot = None
        req.handle = None

    def _poll(self, now: float) -> list:
        out = []
        for req in list(self.active):
            while req.inflight and self.backend.query(req.inflight[0][0]):
                token, _ = req.inflight.pop(0)
                if self.backend.failed(token):
                    req.slice_failed = True
            if req.slice_failed and not req.inflight and req.status == "running":
                # a failed slice: once the request's queue has drained, retry it
                # from round 0 (its input is ingested again) or give up
                req.slice_failed = False
                req.retries += 1
                if req.retries > self.max_retries:
                    req.status = "failed"
                    req.error = "device reported a failed slice"
                else:
                    req.next_round = 0
                    self.backend.load(req.handle, req, req.slot)
            if req.status == "cancelled" and not req.inflight:
                self.active.remove(req)
                self._release(req)
                self.finished.append(req)
                continue
            if req.status == "failed" and not req.inflight:
                self.active.remove(req)
                self._release(req)
                self.finished.append(req)
                continue
            if (req.next_round >= req.rounds and not req.inflight and not req.slice_failed
                    and req.status == "running"):
                req.done = now
                req.status = "done"
                req.result = self.backend.finish(req.handle, req)
                self.active.remove(req)
                self._release(req)
                self.finished.append(req)
                out.append(req)
        return out

    def _admit(self, now: float):
        blocked = False
        for req in list(self.pending):
            if req.arrival > now or not self.free_slots:
                break
            need = self.backend.bytes_needed(req.n)
            if self.used + need <= self.budget and not blocked:
                self.pending.remove(req)
                req.slot = self.free_slots.pop(0)
                req.handle = self.backend.alloc(req, req.slot)
                self.used += need
                req.rounds = self.backend.num_rounds(req.n)
                req.next_round = 0
                req.admitted = now
                req.status = "running"
                self.backend.load(req.handle, req, req.slot)
                self.active.append(req)
            else:
                req.bypassed += 1
                if req.bypassed > self.max_bypass:
                    blocked = True  # nothing behind it may overtake it any more

    def _issue(self):
        progressed = True
        while progressed:  # round-robin, one slice per request per pass
            progressed = False
            for req in self.active:
                if req.status != "running" or req.next_round >= req.rounds or req.slice_failed:
                    continue
                if len(req.inflight) >= self.inflight:
                    continue
                r0 = req.next_round
                r1 = min(r0 + self.slice_rounds, req.rounds)
                token = self.backend.enqueue(req.handle, req, req.slot, r0, r1)
                req.inflight.append((token, r1))
                req.next_round = r1
                progressed = True

    # ------------------------------------------------------------ run loop
    def run(self, requests, realtime: bool = True, spin: float = 2e-5) -> dict:
        """Serve a whole request stream (arrival times relative to the start)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival += t0
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.clock()
            while i < len(reqs) and (reqs[i].arrival <= now or not realtime):
                self.submit(reqs[i])
                i += 1
            self.step(now)
            if realtime and spin > 0:
                time.sleep(spin)
        t1 = self.clock()
        for r in reqs:
            r.arrival -= t0
            if r.done is not None:
                r.done -= t0
            if r.admitted is not None:
                r.admitted -= t0
        return summarize(reqs, t1 - t0)


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, math.ceil(q / 100.0 * len(v)) - 1))
    return v[k]


def summarize(reqs, makespan: float) -> dict:
    done = [r for r in reqs if r.status == "done"]
    lat = [r.latency for r in done]
    work = float(sum(float(r.n) ** 3 for r in done))
    return {
        "requests": len(reqs),
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "failed": sum(r.status == "failed" for r in reqs),
        "cancelled": sum(r.status == "cancelled" for r in reqs),
        "p50_ms": percentile(lat, 50) * 1e3 if lat else None,
        "p99_ms": percentile(lat, 99) * 1e3 if lat else None,
        "mean_ms": (sum(lat) / len(lat)) * 1e3 if lat else None,
        "makespan_s": makespan,
        "cell_updates_per_s": work / makespan if makespan > 0 else None,
    }
