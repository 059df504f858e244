"""Continuous-batching server for QUAPI propagation requests on one GPU.

Requests (different M, L, bath, kT, step counts and precisions) arrive over
time.  The server:

* admits a waiting request whenever a slot is free and the request's device
  footprint (the library's ``footprint``) fits in the remaining HBM budget --
  the paper's "did not fit on the GPU" becomes "wait for memory".  Policy
  ``"fifo"`` admits in arrival order; ``"sjf"`` admits the waiting request
  with the least estimated device work first (non-preemptive);
* keeps every admitted request's tensor resident in its own workspace (a
  torch uint8 tensor) and runs it on its own HIP stream, so the work of
  different requests overlaps on the device;
* batches the requests small enough for the library's persistent path
  (N^L <= 2^14: one workgroup per request runs all of its steps): every
  loop iteration, the newly admitted ones of the same M and precision go to
  the GPU together in one ``propagate_batch`` call, which advances each of
  them through all of its steps in one launch;
* enqueues every other request's steps in chunks through
  ``propagate_async``, round-robin over the active requests, at most two
  chunks in flight per request.  A chunk is sized to about ``chunk_ms`` of
  estimated device time, so the streams that share a hardware queue
  interleave finely and a long request's steps do not hold a short one's
  for long;
* records arrival, admission and completion times and reports p50/p99
  latency (arrival -> rho on the host) and aggregate throughput.

The work estimate is the HBM traffic of the steps at a nominal rate:
2 N^min(n+1, L) sizeof(complex) bytes per step n at 4 TB/s, and at least
10 microseconds per step (launch-bound small tensors).

A request returns rho(t_k) for k = 0..n_steps ('allPoints', Sec. IV of the
paper), or with ``meta['final_only']`` just rho(t_0) and rho(t_n_steps)
('justFinalPoint'), which skips the rho reduction of every other step.  A
request with a Hamiltonian per interval (``H_t``, a driven system) runs one
step per launch, like any driven context.  The kernels are deterministic and each request has its own
context, so a request's result does not depend on what else is running.
"""
from __future__ import annotations

import sys
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import quapi as Q

__all__ = ["Server", "RequestResult", "work_entries", "est_step_s", "est_work_s", "summarize"]


def work_entries(N: int, L: int, n_steps: int) -> int:
    """Tensor entries written over a run: step n writes N^min(n+1, L) entries."""
    return int(sum(N ** min(n + 1, L) for n in range(1, n_steps + 1)))


_NOMINAL_BYTES_PER_S = 4.0e12
_MIN_STEP_S = 1.0e-5


def est_step_s(w) -> float:
    """Estimated device time of one full-window step of request w."""
    cs = 16 if w.dtype == "c128" else 8
    return max(2.0 * w.N ** w.L * cs / _NOMINAL_BYTES_PER_S, _MIN_STEP_S)


def est_work_s(w) -> float:
    """Estimated device time of the whole request."""
    cs = 16 if w.dtype == "c128" else 8
    return max(2.0 * work_entries(w.N, w.L, w.n_steps) * cs / _NOMINAL_BYTES_PER_S, _MIN_STEP_S * w.n_steps)


@dataclass
class RequestResult:
    index: int
    name: str
    M: int
    L: int
    dtype: str
    n_steps: int
    arrival_s: float
    admit_s: float
    finish_s: float
    rho: np.ndarray
    entries: int

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s


@dataclass
class _Active:
    w: object
    index: int
    ctx: Q.Context
    stream: object
    rho_dev: object
    slot: int
    fp: int
    admit_s: float
    fuse: int = 1
    final_only: bool = False
    persistent: bool = False       # batched through propagate_batch
    enqueued: int = 0
    events: deque = field(default_factory=deque)


class Server:
    """Admission by footprint, one stream and context per active request."""

    def __init__(self, max_active: int = 8, hbm_budget: Optional[int] = None, chunk_steps: int = 32,
                 device: str = "cuda:0", progress: bool = False, policy: str = "fifo",
                 chunk_ms: Optional[float] = None):
        """chunk_steps: steps per chunk; with chunk_ms set, the chunk is instead
        sized to about chunk_ms of estimated device time (2 to 256 steps)."""
        import torch
        if policy not in ("fifo", "sjf"):
            raise ValueError(f"unknown policy {policy!r}")
        self.torch = torch
        self.device = device
        self.max_active = max_active
        self.chunk = max(2, chunk_steps)
        self.chunk_ms = chunk_ms
        self.policy = policy
        self.progress = progress
        self.streams = [torch.cuda.Stream(device) for _ in range(max_active)]
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget = int(free * 0.85)
        self.budget = int(hbm_budget)
        self.batched = 0               # requests run through propagate_batch
        self.batch_calls = 0

    def _admit(self, w, index: int, slot: int, now: float) -> _Active:
        torch = self.torch
        p = Q.params_from(w)
        stream = self.streams[slot]
        ctx = Q.create_in_torch(p, stream=stream, device=self.device)
        final_only = bool(w.meta.get("final_only", False))
        rows = 2 if final_only else w.n_steps + 1
        rho_dev = torch.empty((rows, w.N, 2), dtype=torch.float64, device=self.device)
        ctx.propagate_async(0, [0], rho_dev.data_ptr())          # rho(t_0)
        return _Active(w=w, index=index, ctx=ctx, stream=stream, rho_dev=rho_dev, slot=slot,
                       fp=Q.footprint(p), admit_s=now, fuse=ctx.fused_steps(), final_only=final_only,
                       persistent=ctx.persistent() != 0)

    def _launch_batches(self, active) -> int:
        """One propagate_batch call per (M, precision) over the admitted
        persistent-path requests that have not started: each runs all of its
        steps.  Returns the number of requests launched."""
        torch = self.torch
        groups: dict = {}
        for a in active.values():
            if a.persistent and a.enqueued == 0 and a.w.n_steps > 0:
                groups.setdefault((a.w.M, a.w.dtype), []).append(a)
        launched = 0
        for grp in groups.values():
            n = [a.w.n_steps for a in grp]
            modes = [2 if a.final_only else 1 for a in grp]
            outs = [a.rho_dev.data_ptr() + a.w.N * 16 for a in grp]
            Q.propagate_batch([a.ctx for a in grp], n, modes, outs)
            ev = torch.cuda.Event()
            ev.record(grp[0].stream)                # the batch runs on its first request's stream
            for a in grp:
                a.enqueued = a.w.n_steps
                a.events.append(ev)
            self.batch_calls += 1
            launched += len(grp)
        self.batched += launched
        return launched

    def run(self, requests, realtime: bool = True) -> list[RequestResult]:
        """Serve the requests (each with meta['arrival_s']); returns results in index order."""
        torch = self.torch
        order = sorted(range(len(requests)), key=lambda i: requests[i].meta.get("arrival_s", 0.0))
        pending = deque(order)
        waiting: deque = deque()
        active: dict[int, _Active] = {}
        free_slots = list(range(self.max_active))[::-1]
        used = 0
        fps = {}
        results: list[RequestResult] = []
        t0 = time.perf_counter()

        def now() -> float:
            return time.perf_counter() - t0

        while pending or waiting or active:
            progressed = False
            t = now()
            while pending and (not realtime or requests[pending[0]].meta.get("arrival_s", 0.0) <= t):
                waiting.append(pending.popleft())
            # admission by slot and HBM footprint: the head of the queue (fifo), or
            # the waiting request with the least estimated work that fits (sjf)
            while waiting and free_slots:
                for i in waiting:
                    if i not in fps:
                        fps[i] = Q.footprint(Q.params_from(requests[i]))
                        if fps[i] > self.budget:
                            raise Q.QuapiError(Q.ERR_NOMEM,
                                               f"request {i} needs {fps[i]} bytes, more than the budget")
                if self.policy == "fifo":
                    i = waiting[0]
                    if used + fps[i] > self.budget:
                        break
                else:
                    fit = [j for j in waiting if used + fps[j] <= self.budget]
                    if not fit:
                        break
                    i = min(fit, key=lambda j: (est_work_s(requests[j]), j))
                waiting.remove(i)
                slot = free_slots.pop()
                a = self._admit(requests[i], i, slot, now())
                used += a.fp
                active[slot] = a
                progressed = True
            # the newly admitted small requests, batched
            if self._launch_batches(active):
                progressed = True
            # enqueue the next chunk of every other active request (two chunks in flight at most)
            for a in active.values():
                while a.events and a.events[0].query():
                    a.events.popleft()
                if not a.persistent and a.enqueued < a.w.n_steps and len(a.events) < 2:
                    chunk = self.chunk
                    if self.chunk_ms is not None:
                        chunk = int(min(256, max(2, self.chunk_ms * 1e-3 / est_step_s(a.w))))
                    end = min(a.enqueued + chunk, a.w.n_steps)
                    # never end a chunk inside a fused step group (L+1 .. L+F), ...:
                    # the run then has the same bits as one call of all steps
                    if end < a.w.n_steps and end > a.w.L and (end - a.w.L) % a.fuse:
                        end -= (end - a.w.L) % a.fuse
                        if end <= a.enqueued:
                            end = min(a.enqueued + a.fuse, a.w.n_steps)
                    k = end - a.enqueued
                    if a.final_only:                             # rho only at the last step
                        sel = [a.w.n_steps] if end == a.w.n_steps else []
                        a.ctx.propagate_async(k, sel, a.rho_dev.data_ptr() + a.w.N * 16)
                    else:
                        off = (a.enqueued + 1) * a.w.N * 16
                        a.ctx.propagate_async(k, None, a.rho_dev.data_ptr() + off)
                    a.enqueued += k
                    ev = torch.cuda.Event()
                    ev.record(a.stream)
                    a.events.append(ev)
                    progressed = True
            # completions
            for slot in list(active):
                a = active[slot]
                if a.enqueued == a.w.n_steps and all(e.query() for e in a.events):
                    with torch.cuda.stream(a.stream):
                        rho = a.rho_dev.cpu().numpy()
                    finish = now()
                    a.ctx.destroy()
                    used -= a.fp
                    free_slots.append(slot)
                    del active[slot]
                    w = a.w
                    results.append(RequestResult(
                        index=a.index, name=w.name, M=w.M, L=w.L, dtype=w.dtype, n_steps=w.n_steps,
                        arrival_s=(w.meta.get("arrival_s", 0.0) if realtime else 0.0), admit_s=a.admit_s,
                        finish_s=finish, rho=rho.view(np.complex128).reshape(-1, w.M, w.M),
                        entries=work_entries(w.N, w.L, w.n_steps)))
                    progressed = True
                    if self.progress and len(results) % 16 == 0:
                        print(f"serve: {len(results)} done at {finish:.1f} s, {len(active)} active, "
                              f"{len(waiting)} waiting", file=sys.stderr, flush=True)
            if not progressed:
                if not active and pending and realtime:
                    time.sleep(max(0.0, min(0.01, requests[pending[0]].meta.get("arrival_s", 0.0) - now())))
                else:
                    time.sleep(0.0002)
        results.sort(key=lambda r: r.index)
        return results


def summarize(results: list[RequestResult]) -> dict:
    lat = np.array([r.latency_s for r in results])
    makespan = max(r.finish_s for r in results) - min(r.arrival_s for r in results)
    total = sum(r.entries for r in results)
    return {
        "requests": len(results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()),
        "makespan_s": float(makespan),
        "gelem_s": total / makespan / 1e9,
        "entries": int(total),
    }
