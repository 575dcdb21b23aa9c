"""Continuous-batching APSP service on one GPU.

Requests (one graph each, of any size) arrive over time.  The server:

* admits a request when its matrix (and checkpoint buffers) fit the HBM
  budget next to what is already resident and a slot (a HIP stream) is free:
  first fit in arrival order, except that a request passed over
  ``max_bypass`` times blocks the ones behind it, so large requests cannot
  starve.  The solver state a slot's stream keeps (helper streams' word and
  panel copies, which grow with the largest request the slot solved and
  outlive each request) is counted too, as it grows;
* keeps each admitted matrix in device memory from ingestion to completion;
* solves in slices of ``slice_rounds`` rounds of the blocked method
  (``apsp_solve_rounds``), at most ``inflight`` slices per request enqueued
  ahead; the slot streams run concurrently, so work of different requests
  overlaps on the device and a small request that arrives behind a large one
  does not wait for it.  ``policy`` orders the requests that get slices:
  ``"rr"`` round-robin in admission order, ``"fifo"`` by arrival, ``"srpt"``
  by least remaining work (rounds left x n^2) first; at most ``max_running``
  requests have slices in flight at once (default: every slot), and at most
  ``max_large`` of those with n >= ``large_n`` (when set);
* with ``checkpoint_rounds`` > 0, copies a request's matrix aside (on its
  slot stream) whenever a slice ends on a multiple of that many rounds, and
  retries a failed slice from the last checkpoint whose slice completed,
  instead of from round 0 (which re-ingests the input);
* records, per request, arrival / admission / completion times, and reports
  p50 / p99 latency, overall and per request size, and cell updates per
  second; the first ``warmup`` requests (in arrival order) are served but
  left out of the latency figures.

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
    # checkpoints: (round, buffer) of the last one whose slice completed, and
    # the one enqueued behind a slice still in flight (its token)
    ckpt: Any = None
    ckpt_pending: Any = None
    spare: Any = None                   # checkpoint buffer not holding either

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class SimBackend:
    """Backend without a device: each slice takes a modelled time.

    ``rate`` is cell updates per second of one slot; a slice of rounds r0..r1
    of an n-vertex problem does (r1 - r0) * b * n^2 updates.  ``fail`` may
    name request ids whose first slice reports a device failure, ``fail_at``
    maps request ids to a round whose slice fails once.  The handle records
    the rounds applied to it, so tests can check that a retried request
    ends with every round applied once, in order.
    """

    def __init__(self, rate: float = 1e12, b: int = 128, clock: Callable[[], float] = None,
                 fail: tuple = (), fail_at: dict = None):
        self.rate = rate
        self.b = b
        self.clock = clock or time.perf_counter
        self.busy_until = {}
        self.fail = set(fail)
        self.fail_at = dict(fail_at or {})
        self.allocated = 0
        self.freed = 0
        self.loads = 0
        self.restores = 0

    def bytes_needed(self, n: int, checkpoints: int = 0) -> int:
        return 4 * n * n * (1 + checkpoints)

    def state_bytes(self, n: int) -> int:
        return 0

    def num_rounds(self, n: int) -> int:
        return -(-n // self.b) if n else 0

    def work(self, n: int, rounds: int) -> float:
        return float(rounds) * self.b * n * n

    def alloc(self, req: Request, slot: int):
        self.allocated += 1
        return {"n": req.n, "rounds": []}

    def alloc_checkpoint(self, req: Request, slot: int):
        return {"rounds": []}

    def free(self, handle, req: Request, slot: int):
        self.freed += 1

    def load(self, handle, req: Request, slot: int):
        self.loads += 1
        handle["rounds"] = []

    def checkpoint(self, handle, buf, req: Request, slot: int):
        buf["rounds"] = list(handle["rounds"])

    def restore(self, handle, buf, req: Request, slot: int):
        self.restores += 1
        handle["rounds"] = list(buf["rounds"])

    def enqueue(self, handle, req: Request, slot: int, r0: int, r1: int):
        start = max(self.clock(), self.busy_until.get(slot, 0.0))
        kb = min(r1 * self.b, req.n) - r0 * self.b
        end = start + kb * req.n * req.n / self.rate
        self.busy_until[slot] = end
        failed = req.rid in self.fail and r0 == 0 and req.retries == 0
        at = self.fail_at.get(req.rid)
        if at is not None and r0 <= at < r1:
            failed = True
            del self.fail_at[req.rid]
        # a failed slice leaves the matrix in an unknown state
        handle["rounds"].extend(["?"] if failed else range(r0, r1))
        return ("sim", end, failed)

    def query(self, token) -> bool:
        return self.clock() >= token[1]

    def failed(self, token) -> bool:
        return bool(token[2])

    def finish(self, handle, req: Request):
        return list(handle["rounds"])  # the rounds applied, in order


class GpuBackend:
    """Device backend: torch memory and streams, the C ABI for every solve step.

    ``payload`` of a request is an edge list (u, v, w) (undirected, one entry
    per edge) or a host matrix; it is turned into the dense device matrix on
    the request's slot stream.  With ``keep_results`` the solved matrix is
    handed to the caller in ``Request.result``; that memory is then the
    caller's and no longer counted against the server's budget.
    """

    def __init__(self, device=None, slots: int = 4, dtype: str = "f32", keep_results=True,
                 fail_at: dict = None):
        import torch

        import paper_1902_04446_amd as apsp

        self.torch = torch
        self.apsp = apsp
        self.device = torch.device(device or "cuda:0")
        with torch.cuda.device(self.device):
            self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        self.dtype = dtype
        self.code = apsp.APSP_F32 if dtype == "f32" else apsp.APSP_I32
        self.keep_results = keep_results
        # request id -> round: the slice holding that round is reported failed
        # once and the matrix overwritten (a failure forced from the host, to
        # exercise the retry path)
        self.fail_at = dict(fail_at or {})
        # per-slot pinned staging buffers of the inputs, grown on demand.  A
        # copy from pageable memory would block the host until the device is
        # idle (every slot's work); from pinned memory it is queued on the
        # slot stream and the host goes on.  Before a buffer is refilled the
        # host waits for the event recorded after its last copy (in the
        # server a slot is handed out again only once its stream has
        # drained, so that wait is already over).
        self._staging = [dict() for _ in range(slots)]

    @staticmethod
    def _ld(n: int) -> int:
        # rows padded to 16 bytes: the library then solves every slice in
        # place (rows off 16 bytes would be copied into an aligned working
        # copy for each slice)
        return (n + 3) // 4 * 4

    def bytes_needed(self, n: int, checkpoints: int = 0) -> int:
        """Device bytes a request holds while admitted: its matrix and its
        checkpoint buffers (rows padded to a multiple of 4 elements)."""
        return 4 * n * self._ld(n) * (1 + checkpoints)

    def state_bytes(self, n: int) -> int:
        """Device bytes of the solver's state that a slot stream keeps once it
        has solved an n-vertex request (kept with the slot, grown, not shrunk)."""
        return self.apsp.stream_state_bytes(n, self.code)

    def num_rounds(self, n: int) -> int:
        return self.apsp.num_rounds(n, self.code)

    def work(self, n: int, rounds: int) -> float:
        return float(rounds) * self.apsp.round_width(n, self.code) * n * n

    def _empty(self, n: int, slot: int):
        # allocated on the slot stream, where every later use of it is ordered:
        # the caching allocator then only hands out a block whose earlier uses
        # on that stream precede this request's work
        tdt = self.torch.float32 if self.dtype == "f32" else self.torch.int32
        with self.torch.cuda.stream(self.streams[slot]):
            return self.torch.empty((n, self._ld(n)), dtype=tdt, device=self.device)[:, :n]

    def alloc(self, req: Request, slot: int):
        return self._empty(req.n, slot)

    def alloc_checkpoint(self, req: Request, slot: int):
        return self._empty(req.n, slot)

    def free(self, handle, req: Request, slot: int):
        pass  # dropped with the last reference (torch's caching allocator reuses it)

    def close(self):
        """Release the solver state of every slot stream (waits for them)."""
        for s in self.streams:
            self.apsp.release_stream_state(s)

    def checkpoint(self, handle, buf, req: Request, slot: int):
        with self.torch.cuda.stream(self.streams[slot]):
            buf.copy_(handle)

    def restore(self, handle, buf, req: Request, slot: int):
        with self.torch.cuda.stream(self.streams[slot]):
            handle.copy_(buf)

    def _stage(self, slot: int, key: str, arr):
        """Device copy of host array `arr`, copied through slot's pinned
        buffer `key` (asynchronous on the current stream, the slot's)."""
        torch = self.torch
        src = torch.from_numpy(arr.reshape(-1))
        buf, ev = self._staging[slot].get(key, (None, None))
        if ev is not None:
            ev.synchronize()  # the previous copy out of this buffer is done
        if buf is None or buf.dtype != src.dtype or buf.numel() < src.numel():
            buf = torch.empty(max(src.numel(), 1 << 16), dtype=src.dtype, pin_memory=True)
        host = buf[:src.numel()]
        host.copy_(src)
        dev = host.to(self.device, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        self._staging[slot][key] = (buf, ev)
        return dev.view(arr.shape)

    def load(self, handle, req: Request, slot: int):
        import numpy as np

        torch = self.torch
        s = self.streams[slot]
        # the matrix is used on the slot stream: the caching allocator must not
        # hand its memory out again before that stream's work is done
        handle.record_stream(s)
        ddt = np.float32 if handle.dtype == torch.float32 else np.int32
        with torch.cuda.stream(s):
            p = req.payload
            if isinstance(p, np.ndarray):
                handle.copy_(self._stage(slot, "dense", np.ascontiguousarray(p, ddt)))
            else:
                u, v, w = p
                fill = float("inf") if handle.dtype == torch.float32 else float(self.apsp.INF_I32)
                handle.fill_(fill)
                if len(u):
                    uv = self._stage(slot, "uv", np.stack([np.asarray(u, np.int64),
                                                           np.asarray(v, np.int64)]))
                    tw = self._stage(slot, "w", np.asarray(w).astype(ddt))
                    handle[uv[0], uv[1]] = tw
                    handle[uv[1], uv[0]] = tw
        # the solve normalises the diagonal itself (round 0)

    def enqueue(self, handle, req: Request, slot: int, r0: int, r1: int):
        s = self.streams[slot]
        failed = False
        try:
            self.apsp.solve_rounds(handle, r0, r1, stream=s)
        except self.apsp.ApspError:
            failed = True
        at = self.fail_at.get(req.rid)
        if at is not None and r0 <= at < r1:
            del self.fail_at[req.rid]
            failed = True
            with self.torch.cuda.stream(s):
                handle.fill_(-1.0)  # what the failed slice left is unusable
        ev = self.torch.cuda.Event()
        ev.record(s)
        return (ev, failed)

    def query(self, token) -> bool:
        return token[0].query()

    def failed(self, token) -> bool:
        return token[1]

    def finish(self, handle, req: Request):
        return handle if self.keep_results else None


class ApspServer:
    POLICIES = ("rr", "fifo", "srpt")

    def __init__(self, backend, hbm_budget: int, slots: int = 4, slice_rounds: int = 8,
                 inflight: int = 2, max_bypass: int = 8, max_retries: int = 1,
                 clock: Callable[[], float] = None, policy: str = "rr",
                 max_running: Optional[int] = None, checkpoint_rounds: int = 0,
                 warmup: int = 0, large_n: Optional[int] = None, max_large: int = 1):
        if policy not in self.POLICIES:
            raise ValueError(f"policy must be one of {self.POLICIES}")
        self.backend = backend
        self.budget = int(hbm_budget)
        self.slots = slots
        self.slice_rounds = max(1, slice_rounds)
        self.inflight = max(1, inflight)
        self.max_bypass = max_bypass
        self.max_retries = max_retries
        self.clock = clock or time.perf_counter
        self.policy = policy
        self.max_running = max(1, max_running or slots)
        self.checkpoint_rounds = max(0, checkpoint_rounds)
        self.warmup = max(0, warmup)
        # requests of at least large_n vertices fill the whole device on
        # their own: at most max_large of them have slices in flight at once
        # (in policy order), so they do not split the device among themselves
        # while smaller requests still run beside them
        self.large_n = large_n
        self.max_large = max(1, max_large)
        self.pending: collections.deque = collections.deque()
        self.active: list = []
        self.finished: list = []
        self.used = 0
        # the solver state each slot's stream keeps (counted in `used` while
        # the server lives: it outlasts the requests that grew it)
        self.slot_state = [0] * slots
        self.free_slots = list(range(slots))

    # ---------------------------------------------------------------- API
    def need(self, n: int) -> int:
        """Bytes a request of n vertices holds while admitted."""
        return self.backend.bytes_needed(n, 2 if self.checkpoint_rounds else 0)

    def submit(self, req: Request):
        if self.need(req.n) + self.backend.state_bytes(req.n) > self.budget:
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
        self.used -= self.need(req.n)
        self.free_slots.append(req.slot)
        self.backend.free(req.handle, req, req.slot)
        req.slot = None
        req.handle = None
        req.ckpt = req.ckpt_pending = req.spare = None

    def _poll(self, now: float) -> list:
        out = []
        for req in list(self.active):
            while req.inflight and self.backend.query(req.inflight[0][0]):
                token, _ = req.inflight.pop(0)
                if self.backend.failed(token):
                    req.slice_failed = True
                elif (req.ckpt_pending is not None and req.ckpt_pending[2] is token
                      and not req.slice_failed):
                    # the slice before the copy completed: the copy holds good
                    # data (it is ordered after the slice on the slot stream)
                    if req.ckpt is not None:
                        req.spare = req.ckpt[1]
                    req.ckpt = req.ckpt_pending[:2]
                    req.ckpt_pending = None
            if req.slice_failed and not req.inflight and req.status == "running":
                # a failed slice: once the request's queue has drained, retry it
                # from the last good checkpoint, else from round 0 (its input
                # ingested again), or give up
                req.slice_failed = False
                req.retries += 1
                if req.ckpt_pending is not None:  # taken behind a failed slice
                    req.spare = req.ckpt_pending[1]
                    req.ckpt_pending = None
                if req.retries > self.max_retries:
                    req.status = "failed"
                    req.error = "device reported a failed slice"
                elif req.ckpt is not None:
                    req.next_round = req.ckpt[0]
                    self.backend.restore(req.handle, req.ckpt[1], req, req.slot)
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
            need = self.need(req.n)
            slot = self.free_slots[0]
            grow = max(0, self.backend.state_bytes(req.n) - self.slot_state[slot])
            if self.used + need + grow <= self.budget and not blocked:
                self.pending.remove(req)
                req.slot = self.free_slots.pop(0)
                self.slot_state[slot] += grow
                self.used += grow
                req.handle = self.backend.alloc(req, req.slot)
                self.used += need
                req.rounds = self.backend.num_rounds(req.n)
                req.next_round = 0
                req.admitted = now
                req.status = "running"
                if self.checkpoint_rounds:
                    req.spare = self.backend.alloc_checkpoint(req, req.slot)
                    req.ckpt = (0, self.backend.alloc_checkpoint(req, req.slot))
                self.backend.load(req.handle, req, req.slot)
                if self.checkpoint_rounds:  # round 0: the ingested input
                    self.backend.checkpoint(req.handle, req.ckpt[1], req, req.slot)
                self.active.append(req)
            else:
                req.bypassed += 1
                if req.bypassed > self.max_bypass:
                    blocked = True  # nothing behind it may overtake it any more

    def _order(self) -> list:
        """Running requests in the order the policy serves them."""
        live = [r for r in self.active if r.status == "running"]
        if self.policy == "fifo":
            live.sort(key=lambda r: (r.arrival, r.rid))
        elif self.policy == "srpt":
            live.sort(key=lambda r: (self.backend.work(r.n, r.rounds - r.next_round),
                                     r.arrival, r.rid))
        return live

    def _issue(self):
        # the first max_running requests in policy order may have slices in
        # flight; requests outside them that still have slices in flight keep
        # a place (their slices cannot be recalled)
        order = self._order()
        busy = [r for r in order if r.inflight]
        large = (lambda r: self.large_n is not None and r.n >= self.large_n)
        n_large = sum(1 for r in busy if large(r))
        chosen = []
        for r in order:
            if len(chosen) >= self.max_running:
                break
            if r.next_round < r.rounds and not r.slice_failed:
                if large(r) and not r.inflight:
                    if n_large >= self.max_large:
                        continue
                    n_large += 1
                chosen.append(r)
        room = self.max_running - len([r for r in busy if r not in chosen])
        chosen = chosen[:max(0, room)]
        progressed = True
        while progressed:  # one slice per chosen request per pass
            progressed = False
            for req in chosen:
                if req.next_round >= req.rounds or req.slice_failed:
                    continue
                if len(req.inflight) >= self.inflight:
                    continue
                r0 = req.next_round
                r1 = min(r0 + self.slice_rounds, req.rounds)
                token = self.backend.enqueue(req.handle, req, req.slot, r0, r1)
                req.inflight.append((token, r1))
                req.next_round = r1
                progressed = True
                k = self.checkpoint_rounds
                if (k and r1 < req.rounds and r1 // k > r0 // k and req.ckpt_pending is None
                        and req.spare is not None):
                    buf, req.spare = req.spare, None
                    self.backend.checkpoint(req.handle, buf, req, req.slot)
                    req.ckpt_pending = (r1, buf, token)

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
        return summarize(reqs, t1 - t0, warmup=self.warmup)


def percentile(values, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(0, min(len(v) - 1, math.ceil(q / 100.0 * len(v)) - 1))
    return v[k]


def summarize(reqs, makespan: float, warmup: int = 0) -> dict:
    """Counts over every request; latencies over the completed requests after
    the first ``warmup`` arrivals, overall and per size; throughput (n^3 per
    second) over every completed request and the whole makespan."""
    done = [r for r in reqs if r.status == "done"]
    measured = [r for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))[warmup:]
                if r.status == "done"]
    lat = [r.latency for r in measured]
    work = float(sum(float(r.n) ** 3 for r in done))
    per_size = {}
    for n in sorted({r.n for r in measured}):
        ls = [r.latency for r in measured if r.n == n]
        per_size[str(n)] = {"count": len(ls), "p50_ms": percentile(ls, 50) * 1e3,
                            "p99_ms": percentile(ls, 99) * 1e3,
                            "max_ms": max(ls) * 1e3}
    return {
        "requests": len(reqs),
        "done": len(done),
        "warmup_excluded": min(warmup, len(reqs)),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "failed": sum(r.status == "failed" for r in reqs),
        "cancelled": sum(r.status == "cancelled" for r in reqs),
        "p50_ms": percentile(lat, 50) * 1e3 if lat else None,
        "p99_ms": percentile(lat, 99) * 1e3 if lat else None,
        "mean_ms": (sum(lat) / len(lat)) * 1e3 if lat else None,
        "per_size": per_size,
        "makespan_s": makespan,
        "cell_updates_per_s": work / makespan if makespan > 0 else None,
    }
