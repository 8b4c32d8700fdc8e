"""Serving RSM decompositions on one GPU with continuous batching.

Requests arrive over time (each names a device-resident input of a pool and carries its
own RSM seed).  The server admits waiting requests while their HBM footprint (workspace
with N and the solver's matrices, plus the factors U-hat and V-hat) fits the budget, and
launches every admitted group as one batched library call on one of several streams.
Requests that arrive while batches run are admitted as soon as memory and a stream free
up, so their work overlaps on the device with the batches still running.  Inputs (Y, W)
stay resident for the whole run; each request's factors stay on the device in its result.
Each stream owns one workspace arena, grown to the largest group it has run and reused by
every later group on that stream, so the caching allocator does not accumulate one
workspace per batch (memory that the runtime may need itself, e.g. for kernel scratch).
A group admitted while other groups run asks the library to keep its steps' launch groups
in order on its own stream (SERIAL_STEPS): the overlap then comes from the server's
streams, which the library's own side-by-side lanes would otherwise queue behind each
other.  A group admitted onto an idle device may spread its steps over those lanes.

`batching=False, max_inflight=1` serves the same trace first-in first-out one request at
a time through the single-problem call: the plain baseline.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field, replace

import numpy as np

from . import Request, _lib, _problem, decompose, decompose_batched, workspace_bytes


@dataclass
class Job:
    """One request of a trace."""
    rid: int
    arrival: float          # seconds from the start of the trace
    item: int               # index into the server's input pool
    seed: int               # this request's RSM seed
    start: float = math.nan
    done: float = math.nan
    result: object = None
    kept: object = None     # (V-hat, sampled rows of U-hat, info bytes) when sampled


def poisson_trace(n_items: int, qps: float, seconds: float, seed: int) -> list[Job]:
    """Arrivals of a Poisson process of rate qps over `seconds`, uniform over the pool, with
    a per-request seed."""
    rng = np.random.default_rng(seed)
    jobs, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / qps)
        if t >= seconds:
            break
        jobs.append(Job(rid=len(jobs), arrival=t, item=int(rng.integers(n_items)),
                        seed=int(rng.integers(0, 2**62))))
    return jobs


@dataclass
class PoolItem:
    """A device-resident input and its decomposition parameters."""
    Y: object
    W: object
    r: int
    num_submatrices: int
    l: int = 0
    gram: str = "f32"
    flags: int = 0                      # library flags, e.g. DETERMINISTIC
    footprint: int = field(default=0)   # bytes per request (filled by the server)


def footprint(it: PoolItem) -> int:
    """HBM bytes one request on `it` holds while in flight: the library's workspace for
    exactly the problem the server will run (its flags included: rows-first sampling
    carves extra buffers), the factors U-hat (m x r) and V-hat (n x r) in FP64, and the
    small info record."""
    req = Request(Y=it.Y, W=it.W, r=it.r, num_submatrices=it.num_submatrices, seed=0,
                  l=it.l, gram=it.gram, flags=it.flags)
    m, n = it.Y.shape
    return _lib.workspace_bytes([_problem(req)]) + 8 * it.r * (m + n) + 4096


class Server:
    def __init__(self, pool: list[PoolItem], *, budget_bytes: int = 16 << 30,
                 max_batch: int = 256, max_inflight: int = 3, batching: bool = True,
                 keep_results: bool = False):
        import torch
        self.torch = torch
        self.pool = pool
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch) if batching else 1
        self.max_inflight = int(max_inflight)
        self.batching = batching
        self.keep = keep_results
        self.device = pool[0].Y.device
        self.streams = [torch.cuda.Stream(self.device) for _ in range(self.max_inflight)]
        self.arenas = [None] * self.max_inflight   # per stream: uint8 tensor, 256-aligned
        for it in pool:
            it.footprint = self._footprint(it)
            if it.footprint > self.budget:
                raise ValueError("a pool item does not fit the memory budget alone")

    def _request(self, job: Job) -> Request:
        it = self.pool[job.item]
        return Request(Y=it.Y, W=it.W, r=it.r, num_submatrices=it.num_submatrices,
                       seed=job.seed, l=it.l, gram=it.gram, flags=it.flags)

    def _footprint(self, it: PoolItem) -> int:
        return footprint(it)

    def _arena(self, si: int, nbytes: int):
        """The stream's workspace arena, grown (by a quarter beyond the need) when a group
        needs more; allocated on that stream, and only replaced between its groups."""
        torch = self.torch
        a = self.arenas[si]
        if a is None or a.numel() < nbytes:
            self.arenas[si] = None
            with torch.cuda.stream(self.streams[si]):
                buf = torch.empty(nbytes + nbytes // 4 + 256, dtype=torch.uint8,
                                  device=self.device)
            off = (-buf.data_ptr()) % 256
            a = buf[off:]
            self.arenas[si] = a
        return a

    def run(self, jobs: list[Job], time_limit: float | None = None,
            sample: dict | None = None) -> dict:
        """Serve `jobs` (sorted by arrival) in real time; returns latency / throughput
        statistics.  Stops admitting new work after time_limit seconds (if given).
        `sample` maps request ids to a device index tensor of rows: for those requests the
        result's V-hat, those rows of U-hat and the raw info record are kept in `job.kept`
        (the rest of the result, its workspace included, is released as for every other
        request)."""
        torch = self.torch
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        waiting: deque[Job] = deque()
        inflight = []            # [event, jobs, bytes, stream index]
        free_streams = list(range(self.max_inflight))
        used = 0
        batches = 0
        batch_sizes = []
        peak_used = 0
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit and not inflight:
                break
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            for entry in list(inflight):
                ev, group, nbytes, si = entry
                if ev.query():
                    t = time.perf_counter() - t0
                    for j in group:
                        j.done = t
                        if sample is not None and j.rid in sample:
                            # on the request's stream: U-hat's memory returns to that
                            # stream's pool when the result is dropped below, and the next
                            # work there is ordered after this copy
                            with torch.cuda.stream(self.streams[si]):
                                j.kept = (j.result.V, j.result.U[sample[j.rid]],
                                          j.result.info_raw)
                        if not self.keep:
                            j.result = None
                    used -= nbytes
                    free_streams.append(si)
                    inflight.remove(entry)
                    progressed = True
            admit = time_limit is None or now <= time_limit
            while admit and waiting and free_streams:
                group, nbytes = [], 0
                while waiting and len(group) < self.max_batch:
                    f = self.pool[waiting[0].item].footprint
                    if used + nbytes + f > self.budget:
                        break
                    group.append(waiting.popleft())
                    nbytes += f
                if not group:
                    break
                si = free_streams.pop()
                st = self.streams[si]
                with torch.cuda.stream(st):
                    reqs = [self._request(j) for j in group]
                    if inflight:
                        reqs[0] = replace(reqs[0], flags=reqs[0].flags | _lib.SERIAL_STEPS)
                    if self.batching:
                        ws = self._arena(si, workspace_bytes(reqs))
                        results = decompose_batched(reqs, stream=st, workspace=ws)
                    else:
                        ws = self._arena(si, max(workspace_bytes([q]) for q in reqs))
                        results = [decompose(q.Y, q.W, q.r, q.num_submatrices, q.seed, l=q.l,
                                             gram=q.gram, flags=q.flags, stream=st,
                                             workspace=ws)
                                   for q in reqs]
                    ev = torch.cuda.Event()
                    ev.record(st)
                t = time.perf_counter() - t0
                for j, res in zip(group, results):
                    j.start = t
                    j.result = res
                used += nbytes
                peak_used = max(peak_used, used)
                inflight.append([ev, group, nbytes, si])
                batches += 1
                batch_sizes.append(len(group))
                progressed = True
            if not progressed:
                # nothing to do until the next arrival or completion
                time.sleep(20e-6)
        t_stop = time.perf_counter() - t0
        stats = latency_stats(jobs, t_stop)
        stats.update({
            "batches": batches,
            "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
            "peak_bytes": int(peak_used),
            "budget_bytes": self.budget,
        })
        return stats


def latency_stats(jobs: list[Job], t_stop: float) -> dict:
    """Completion counts, throughput and latency percentiles of a served trace.  Requests
    never completed (admission stopped at a time limit) have waited at least until the
    stop, so `latency_all_ms` counts them at t_stop: exact when nothing was left unserved,
    otherwise lower bounds of the percentiles over every request."""
    done = [j for j in jobs if not math.isnan(j.done)]
    lat = np.array([j.done - j.arrival for j in done]) if done else np.zeros(1)
    span = (max(j.done for j in done) - min(j.arrival for j in done)) if done else 0.0
    unserved = [j for j in jobs if math.isnan(j.done)]
    lat_all = np.concatenate([lat if done else np.zeros(0),
                              np.array([max(0.0, t_stop - j.arrival) for j in unserved])])
    if lat_all.size == 0:
        lat_all = np.zeros(1)
    return {
        "requests": len(jobs),
        "completed": len(done),
        "unserved": len(unserved),
        "throughput_per_s": len(done) / span if span > 0 else 0.0,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(lat.mean() * 1e3)},
        "latency_all_ms": {"p50": float(np.percentile(lat_all, 50) * 1e3),
                           "p99": float(np.percentile(lat_all, 99) * 1e3),
                           "lower_bound": bool(unserved)},
    }
