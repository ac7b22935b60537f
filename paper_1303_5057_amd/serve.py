"""Continuous-batching request loop for camera requests (image renders).

Requests (a camera each: spin, inclination, image size) arrive over time.
All admitted requests share one resident photon pool in HBM and are advanced
together by ONE persistent integrate launch per iteration (slot mode of the C
ABI: the camera table is a slot table, one slot per in-flight request). The
launch works through a list of live photon ids and writes the list of those
still running (work-list mode), so an iteration costs what the live photons
cost, not what the pool holds.
Between iterations the loop

  * retires requests whose photons have all stopped (per-slot counts of
    stopped photons kept by the integrator, read back with one small
    device-to-host copy),
  * admits waiting requests in arrival order while a slot is free and their
    photons fit the pool (admission by HBM footprint; no bypass, so large
    requests are not starved),
  * sizes the next iteration's step budget (call_steps) so that an iteration
    takes about `slice_ms`, and gives a request whose last photons are
    running (at most 1/64 of them, or 256) `tail_boost` times that budget:
    those few photons then need fewer iterations to finish, while an
    iteration's length is set by the pool's total work, not by the steps of
    a few photons,
  * cancels requests on demand: a waiting one leaves the queue; an admitted
    one has its photons set to a terminal status behind the launch in flight
    (the next launch drops them from the work list when it reads their
    status), and its pool range is reused only after that launch, so no
    stale list entry can reach a new request's photons.

A photon's step is a function of its stored state alone, so a request's
result does not depend on what else is in the pool or on how its steps are
split into iterations.

The loop is host code (scheduling); every step of the hot path runs in the
HIP kernels of libgray.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import gray as G
from .workloads import Camera, Params, Request

ALIGN = 64


class RangeAllocator:
    """First-fit allocator of photon ranges in [0, capacity), 64-aligned."""

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free: List[List[int]] = [[0, capacity]]   # sorted [start, end)

    def alloc(self, n: int) -> Optional[int]:
        need = (n + ALIGN - 1) // ALIGN * ALIGN
        for k, (s, e) in enumerate(self.free):
            if e - s >= need:
                if e - s == need:
                    self.free.pop(k)
                else:
                    self.free[k][0] = s + need
                return s
        return None

    def release(self, start: int, n: int) -> None:
        need = (n + ALIGN - 1) // ALIGN * ALIGN
        k = bisect.bisect_left(self.free, [start, start + need])
        self.free.insert(k, [start, start + need])
        merged: List[List[int]] = []
        for s, e in self.free:
            if merged and merged[-1][1] == s:
                merged[-1][1] = e
            else:
                merged.append([s, e])
        self.free = merged

    def used(self) -> int:
        return self.capacity - sum(e - s for s, e in self.free)


@dataclass
class RequestResult:
    rid: int
    arrival_s: float
    admit_s: float = 0.0
    done_s: float = 0.0
    photons: int = 0
    photon_steps: int = 0
    status: Optional[np.ndarray] = None
    x: Optional[np.ndarray] = None      # (8, n) final state (double; FP32C: hi + lo)
    steps: Optional[np.ndarray] = None
    cancelled: bool = False             # cancelled before it finished (no results)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def bytes_per_photon(precision: str) -> int:
    """HBM footprint of one resident photon: state (FP64 64 B, FP32C 32 B hi +
    32 B lo), status/steps/camera (12 B), counters (12 B), classify flag (1 B)."""
    return 64 + 12 + 12 + 1


@dataclass
class Server:
    """Resident pool + slot table + iteration loop."""
    budget_bytes: int
    params: Params = field(default_factory=lambda: Params(precision="fp32c"))
    max_slots: int = 64
    slice_ms: float = 40.0
    keep_results: bool = False
    device: str = "cuda"
    tail_boost: int = 8

    def __post_init__(self):
        import torch
        self.torch = torch
        cap = self.budget_bytes // bytes_per_photon(self.params.precision)
        self.capacity = max(ALIGN, cap // ALIGN * ALIGN)
        S = self.capacity
        fp64 = self.params.precision == "fp64"
        dt = torch.float64 if fp64 else torch.float32
        dev = self.device
        self.x = torch.zeros(8 * S, dtype=dt, device=dev)
        self.lo = None if fp64 else torch.zeros(8 * S, dtype=torch.float32, device=dev)
        # Photons outside every slot stay in a terminal status (ignored).
        self.status = torch.full((S,), G.UNFINISHED, dtype=torch.int32, device=dev)
        self.steps = torch.zeros(S, dtype=torch.int32, device=dev)
        self.cam = torch.zeros(S, dtype=torch.int32, device=dev)
        self.counters = torch.zeros(3 * S, dtype=torch.int32, device=dev)
        self.flag = torch.zeros(S, dtype=torch.int8, device=dev)
        self.counts = torch.zeros(5 * self.max_slots, dtype=torch.int32, device=dev)
        self.counts_host = torch.zeros(5 * self.max_slots, dtype=torch.int32, pin_memory=True)
        # Work lists of live photon ids (double-buffered) and their lengths.
        self.work = [torch.zeros(S + G.GRAY_WORKLIST_SLACK, dtype=torch.int32, device=dev)
                     for _ in range(2)]
        self.work_count = torch.zeros(2, dtype=torch.int32, device=dev)
        # photons of each slot that have stopped (updated by the integrator),
        # copied to one of two host buffers after each iteration: the loop
        # reads iteration k's copy while iteration k + 1 runs
        self.cam_done = torch.zeros(self.max_slots, dtype=torch.int32, device=dev)
        self.done_host = [torch.zeros(self.max_slots, dtype=torch.int32, pin_memory=True) for _ in range(2)]
        self.done_event = [torch.cuda.Event() for _ in range(2)]
        self.state = G.gray_state(self.x.data_ptr(), None if fp64 else self.lo.data_ptr(),
                                  self.status.data_ptr(), self.steps.data_ptr(), self.cam.data_ptr(),
                                  self.counters.data_ptr(), None, None, S, S)
        self.state.cam_done = self.cam_done.data_ptr()
        self._cur = 0
        self._bind_work()
        self.p = G.params_struct(self.params)
        self.p.flags |= G.GRAY_SLOTS | G.GRAY_WORKLIST
        self.slots = (G.gray_camera * self.max_slots)()
        for k in range(self.max_slots):
            self.slots[k] = G.gray_camera(0.0, 1000.0, 0.0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0.0)
        ws = G.gray_workspace_size(S, self.max_slots, self.p)
        self._ws = torch.zeros(ws + 256, dtype=torch.uint8, device=dev)
        self.ws_ptr = self._ws.data_ptr() + (-self._ws.data_ptr()) % 256
        self.ws_bytes = ws
        self.result_struct = G.gray_result(self.flag.data_ptr(), None, None, self.counts.data_ptr())
        self.alloc = RangeAllocator(S)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.active: Dict[int, tuple] = {}     # slot -> (Request, first, n, RequestResult)
        self._done_seen: Dict[int, int] = {}   # slot -> stopped photons in the last counts read
        self.call_steps = 64
        self.iterations = 0
        self.max_active = 0
        self.max_used = 0
        self.admit_order: List[int] = []
        self._gather: List[tuple] = []
        # ranges of cancelled requests: (first, n, the launch that drops their
        # photons from the work list); freed once that launch is enqueued
        self._release_after: List[tuple] = []

    def _bind_work(self) -> None:
        """work_in = list `_cur` (read by the next integrate, appended to by
        admissions), work_out = the other list."""
        a, b = self._cur, 1 - self._cur
        cp = self.work_count.data_ptr()
        self.state.work_in = self.work[a].data_ptr()
        self.state.work_out = self.work[b].data_ptr()
        self.state.work_in_count = cp + 4 * a
        self.state.work_out_count = cp + 4 * b

    # ------------------------------------------------------------ pool ops
    def _admit(self, req: Request, now: float) -> bool:
        c = req.camera
        n = c.nx * c.ny
        if n > self.capacity:
            raise ValueError(f"request {req.rid} ({n} photons) exceeds the pool")
        free_slots = [k for k in range(self.max_slots) if k not in self.active]
        if not free_slots:
            return False
        first = self.alloc.alloc(n)
        if first is None:
            return False
        k = free_slots[0]
        self.slots[k] = G.camera_struct(c, first)
        G.gray_camera_init_slot(self.slots, self.max_slots, k, self.p, self.state, self.stream)
        res = RequestResult(req.rid, req.arrival_s, admit_s=now, photons=n)
        # the first launch that includes the request
        self.active[k] = (req, first, n, res, self.iterations)
        self._done_seen[k] = 0
        self.admit_order.append(req.rid)
        self.max_active = max(self.max_active, len(self.active))
        self.max_used = max(self.max_used, self.alloc.used())
        return True

    def _retire(self, k: int, now: float) -> RequestResult:
        """Free slot k; the request's results are gathered on the device in
        stream order (behind the launch still running) and read back once
        the loop ends, so retiring never waits for the GPU."""
        req, first, n, res, _ = self.active.pop(k)
        self._done_seen.pop(k, None)
        torch = self.torch
        st = self.steps[first:first + n]
        dev = {"photon_steps": st.to(torch.int64).sum()}
        if self.keep_results:
            dev["status"] = self.status[first:first + n].clone()
            dev["steps"] = st.clone()
            rows = self.x.view(8, self.capacity)[:, first:first + n].double()
            if self.lo is not None:
                rows = rows + self.lo.view(8, self.capacity)[:, first:first + n].double()
            dev["x"] = rows.clone()   # FP64: .double() is the pool itself
        self._gather.append((res, dev))
        # free the range: its photons stay terminal (status is not RUNNING)
        self.alloc.release(first, n)
        self.slots[k] = G.gray_camera(0.0, 1000.0, 0.0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0.0)
        res.done_s = now
        return res

    def _cancel(self, k: int, now: float) -> RequestResult:
        """Cancel the request in slot k. Its photons are set to a terminal
        status in stream order, behind the launch in flight; the next launch
        reads that status for the ids still listed and drops them. The slot
        is free at once (a photon that is not running is never counted);
        the range only after that next launch."""
        req, first, n, res, _ = self.active.pop(k)
        self._done_seen.pop(k, None)
        self.status[first:first + n].fill_(G.UNFINISHED)
        self.slots[k] = G.gray_camera(0.0, 1000.0, 0.0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0, 0, 0.0)
        self._release_after.append((first, n, self.iterations))
        res.cancelled = True
        res.done_s = now
        return res

    def _release_cancelled(self, idle: bool = False) -> None:
        """Free the ranges whose photons no later launch can still list: those
        of requests cancelled before the last enqueued launch, or every one
        when the loop is idle (the input list is then emptied instead)."""
        if idle and self._release_after:
            self.work_count[self._cur].zero_()
        keep = []
        for first, n, launch in self._release_after:
            if idle or launch < self.iterations:
                self.alloc.release(first, n)
            else:
                keep.append((first, n, launch))
        self._release_after = keep

    def _read_back(self) -> None:
        """Host copies of the retired requests' device results."""
        for res, dev in self._gather:
            res.photon_steps = int(dev["photon_steps"].item())
            if "x" in dev:
                res.status = dev["status"].cpu().numpy()
                res.steps = dev["steps"].cpu().numpy()
                res.x = dev["x"].cpu().numpy()
        self._gather = []

    def _launch(self) -> int:
        """Enqueue one integrate launch over every in-flight request and the
        copy of the per-slot stop counts behind it; returns the buffer index
        of that copy. Nothing waits here."""
        b = self.iterations % 2
        self.p.call_steps = int(self.call_steps)
        # tail budget, capped so that one photon's steps at about 2 us each
        # take at most half a slice
        tail = int(min(self.call_steps * self.tail_boost, self.slice_ms * 250.0))
        for k, a in self.active.items():
            n = a[2]
            left = n - self._done_seen.get(k, 0)
            self.slots[k].call_steps = tail if left <= max(256, n // 64) else 0
        G.gray_integrate(self.slots, self.max_slots, self.p, self.state, self.ws_ptr, self.ws_bytes,
                         self.stream)
        self._cur = 1 - self._cur          # the ids still running are the next input
        self._bind_work()
        self.iterations += 1
        self.done_host[b].copy_(self.cam_done, non_blocking=True)
        self.done_event[b].record()
        self._release_cancelled()
        return b

    def _wait(self, b: int, prev_done: Optional[float]) -> tuple:
        """Wait for the launch whose counts went to buffer b; adapt the step
        budget to the time since the previous launch was seen to end (the
        iteration time, the loop keeping the GPU busy). Returns the counts
        and the time this launch was seen to end."""
        self.done_event[b].synchronize()
        t = time.perf_counter()
        if prev_done is not None:
            dt = (t - prev_done) * 1e3
            scale = self.slice_ms / max(dt, 1e-3)
            self.call_steps = int(min(4096, max(32, self.call_steps * min(4.0, max(0.25, scale)))))
        return self.done_host[b].numpy().copy(), t

    # -------------------------------------------------------------- driver
    def run(self, requests: Sequence[Request], realtime: bool = True,
            on_done=None, cancel: Optional[Dict[int, int]] = None) -> List[RequestResult]:
        """Serve `requests` (sorted by arrival). With realtime=False every
        request is available at once (closed loop, for saturation). `cancel`
        maps request ids to a launch count: once that many launches have
        been enqueued, the request is cancelled wherever it is (waiting or in
        flight; a request already finished is not affected). Cancelled
        requests are returned with `cancelled` set."""
        pending = list(requests)
        waiting: List[Request] = []
        done: List[RequestResult] = []
        cancel = dict(cancel or {})
        t_start = time.perf_counter()
        i = 0
        # (count buffer, launch index) of the launch not yet read back
        inflight: Optional[tuple] = None
        last_done: Optional[float] = None
        while i < len(pending) or waiting or self.active:
            now = time.perf_counter() - t_start
            while i < len(pending) and (not realtime or pending[i].arrival_s <= now):
                waiting.append(pending[i])
                i += 1
            for rid in [r for r, at in cancel.items() if at <= self.iterations]:
                slot = next((k for k, a in self.active.items() if a[0].rid == rid), None)
                w = next((r for r in waiting if r.rid == rid), None)
                if slot is not None:
                    done.append(self._cancel(slot, now))
                elif w is not None:
                    waiting.remove(w)
                    done.append(RequestResult(w.rid, w.arrival_s, done_s=now, photons=w.camera.n,
                                              cancelled=True))
                elif any(r.rid == rid for r in pending[i:]):
                    continue            # not arrived yet: cancelled on arrival
                del cancel[rid]
            while waiting and self._admit(waiting[0], now):
                waiting.pop(0)
            if not self.active:
                self._release_cancelled(idle=True)
                if i < len(pending):
                    time.sleep(max(0.0, pending[i].arrival_s - (time.perf_counter() - t_start)))
                continue
            # Launch the next iteration before reading the previous one's
            # counts, so the GPU runs while the host retires and admits
            # (stream order keeps every admission behind the running launch).
            b = self._launch()
            prev, inflight = inflight, (b, self.iterations - 1)
            if prev is None:
                continue
            counts, last_done = self._wait(prev[0], last_done)
            now = time.perf_counter() - t_start
            # a slot's count in that copy is its request's only if the
            # request was in that launch (a reused slot still shows the
            # previous request's count until its own init runs)
            for k in list(self.active.keys()):
                if self.active[k][4] <= prev[1]:
                    self._done_seen[k] = int(counts[k])
                if self.active[k][4] <= prev[1] and counts[k] == self.active[k][2]:
                    r = self._retire(k, now)
                    done.append(r)
                    if on_done:
                        on_done(r)
            if not self.active:
                # nothing left to run: the launch behind is empty for us
                self.torch.cuda.current_stream().synchronize()
                inflight = None
                last_done = None
        self.torch.cuda.current_stream().synchronize()
        self._read_back()
        return done


# request-size classes for latency breakdowns: photons <= 128^2, <= 512^2, more
SIZE_CLASSES = (("small", 0, 128 * 128), ("medium", 128 * 128, 512 * 512), ("large", 512 * 512, 1 << 62))


def size_class(photons: int) -> str:
    for name, lo, hi in SIZE_CLASSES:
        if lo < photons <= hi:
            return name
    return SIZE_CLASSES[0][0]


def latency_stats(results: Sequence[RequestResult], skip: int = 0) -> dict:
    rs = [r for r in sorted(results, key=lambda r: r.rid)[skip:] if not r.cancelled]
    lat = np.array([r.latency_s for r in rs]) * 1e3
    steps = sum(r.photon_steps for r in rs)
    span = max(r.done_s for r in rs) - min(r.arrival_s for r in rs)
    out = {"requests": len(rs), "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
           "photon_steps_per_s": steps / span, "span_s": span,
           "photons": int(sum(r.photons for r in rs))}
    by = {}
    for name, _, _ in SIZE_CLASSES:
        sel = np.array([size_class(r.photons) == name for r in rs])
        if sel.any():
            w = np.array([(r.admit_s - r.arrival_s) for r in rs])[sel] * 1e3
            by[name] = {"requests": int(sel.sum()), "p50_ms": float(np.percentile(lat[sel], 50)),
                        "p99_ms": float(np.percentile(lat[sel], 99)),
                        "queue_wait_p50_ms": float(np.percentile(w, 50)),
                        "queue_wait_p99_ms": float(np.percentile(w, 99))}
    out["by_size"] = by
    return out
