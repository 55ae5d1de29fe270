"""Serving loop: segmentation requests as they arrive, continuously batched.

A request is one image (already in device memory) plus its S, m and
iteration count.  The server

  * admits requests in arrival order while their HBM footprint (image,
    labels, centres, counts and their share of the batch workspace) fits the
    budget and a slot is free; admitted requests keep their outputs resident
    until they complete;
  * packs the admitted requests that are not yet running into one
    ``sslic_run_batch`` call on a free lane (a context with its own workspace
    and its own stream); lanes run concurrently, so requests that arrive while
    others are on the GPU start as soon as a lane and memory free up, and
    their work overlaps with the running batches;
  * records arrival, start and completion time of every request.

``fifo`` is the one-at-a-time baseline: each request in arrival order, alone
(``sslic_run``), after the previous one has finished.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

from . import sslic

_BYTES = {torch.uint8: 1, torch.uint16: 2, torch.float32: 4}


@dataclass
class Request:
    index: int
    arrival: float                 # seconds from the start of the run
    image: torch.Tensor            # device, (*reversed(dims), C)
    S: tuple
    m: float
    iterations: int
    start: float = float("nan")
    done: float = float("nan")
    out: dict = field(default_factory=dict)

    @property
    def voxels(self) -> int:
        return int(self.image.numel() // self.image.shape[-1])


def footprint(req: Request) -> int:
    """HBM bytes a request holds while admitted: its image, labels, centres
    and counts, and its share of the batch tables (centre records, bins,
    accumulators and tile slots, about 600 bytes per cluster in 3D grey)."""
    nd = req.image.dim() - 1
    C = int(req.image.shape[-1])
    dims = tuple(int(d) for d in reversed(req.image.shape[:-1]))
    K = sslic.num_clusters(dims, req.S)
    N = req.voxels
    img = N * C * _BYTES[req.image.dtype]
    F = 1 + nd + C
    per_cluster = (C + nd) * 8 + 8 + 2 * 4 * ((C + 3 * nd + 4) // 4 * 4) + \
        F * 8 + (F + 1) * 8 * (1 << nd) + 13
    return img + 4 * N + K * per_cluster + 4096


@dataclass
class Stats:
    latencies_ms: np.ndarray
    wall_s: float
    voxel_iters: float

    @property
    def p50(self) -> float:
        return float(np.percentile(self.latencies_ms, 50))

    @property
    def p99(self) -> float:
        return float(np.percentile(self.latencies_ms, 99))

    @property
    def mvoxel_iter_s(self) -> float:
        return self.voxel_iters / self.wall_s / 1e6

    def as_dict(self) -> dict:
        return {"p50_ms": round(self.p50, 3), "p99_ms": round(self.p99, 3),
                "mean_ms": round(float(self.latencies_ms.mean()), 3),
                "wall_s": round(self.wall_s, 3), "Mvoxel_iter_s": round(self.mvoxel_iter_s, 1),
                "requests": int(len(self.latencies_ms))}


def _stats(reqs: list, t_end: float) -> Stats:
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    work = float(sum(r.voxels * r.iterations for r in reqs))
    t0 = min(r.arrival for r in reqs)
    return Stats(lat, t_end - t0, work)


class Server:
    """Continuous batching over ``lanes`` concurrent batches."""

    def __init__(self, device: int = 0, hbm_budget: int = 64 << 30, max_slots: int = 256,
                 lanes: int = 3, max_batch: int = 64, tol: float = 0.0):
        self.device = torch.device("cuda", device)
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.tol = float(tol)
        self.ctxs = [sslic.Context(device) for _ in range(lanes)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(lanes)]
        self.busy: list = [None] * lanes  # per lane: (event, [requests]) or None
        self.peak_used = 0                # largest admitted footprint seen (bytes)
        self.peak_running = 0             # most requests on the GPU at once

    def warm(self, reqs: list) -> None:
        """Tile tuning for every (ndim, channels, dtype, S) in ``reqs`` on every
        lane, on the largest request of each kind (the tuner waits); then each
        lane's batch workspace is grown once to what its largest batch can
        need (as many copies of the request with the largest footprint as the
        budget admits, up to ``max_batch``), so that no batch while serving
        grows it: growing frees the old workspace, which waits for the device."""
        kinds = {}
        for r in reqs:
            k = (r.image.dim(), int(r.image.shape[-1]), r.image.dtype, tuple(r.S))
            if k not in kinds or r.voxels > kinds[k].voxels:
                kinds[k] = r
        big = max(reqs, key=footprint)
        nb = max(1, min(self.max_batch, self.max_slots, len(reqs), self.budget // footprint(big)))
        for ctx, st in zip(self.ctxs, self.streams):
            with torch.cuda.stream(st):
                ctx.run_batch([dict(image=r.image, S=r.S, m=r.m, iterations=1)
                               for r in kinds.values()], tol=self.tol, graph=False)
                if nb > 1:
                    ctx.run_batch([dict(image=big.image, S=big.S, m=big.m, iterations=1)] * nb,
                                  tol=self.tol, graph=False)
        torch.cuda.synchronize()

    def _launch(self, lane: int, batch: list) -> None:
        st = self.streams[lane]
        with torch.cuda.stream(st):
            items = [dict(image=r.image, S=r.S, m=r.m, iterations=r.iterations) for r in batch]
            outs = self.ctxs[lane].run_batch(items, tol=self.tol, sync=False, graph=False)
            ev = torch.cuda.Event()
            ev.record(st)
        for r, o in zip(batch, outs):
            r.out = o
        self.busy[lane] = (ev, batch)

    def serve(self, requests: list, clock: Callable[[], float] = time.perf_counter,
              closed_loop: bool = False) -> Stats:
        """Run ``requests`` (sorted by arrival).  Arrival times are honoured
        against ``clock`` unless ``closed_loop`` (all queued at time 0)."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        if closed_loop:
            for r in reqs:
                r.arrival = 0.0
        fp = {r.index: footprint(r) for r in reqs}
        for r in reqs:
            if fp[r.index] > self.budget:
                raise ValueError(f"request {r.index} needs {fp[r.index]} bytes, above the budget")
        arriving = collections.deque(reqs)
        waiting: collections.deque = collections.deque()   # arrived, not admitted
        admitted: collections.deque = collections.deque()  # admitted, not started
        used = 0
        slots = 0
        n_done = 0
        t0 = clock()
        while n_done < len(reqs):
            now = clock() - t0
            while arriving and arriving[0].arrival <= now:
                waiting.append(arriving.popleft())
            for lane, b in enumerate(self.busy):  # completions
                if b is not None and b[0].query():
                    t = clock() - t0
                    for r in b[1]:
                        r.done = t
                        used -= fp[r.index]
                        slots -= 1
                    n_done += len(b[1])
                    self.busy[lane] = None
            while waiting and slots < self.max_slots and used + fp[waiting[0].index] <= self.budget:
                r = waiting.popleft()  # admission in arrival order
                used += fp[r.index]
                slots += 1
                admitted.append(r)
                self.peak_used = max(self.peak_used, used)
            for lane in range(len(self.busy)):
                if not admitted:
                    break
                if self.busy[lane] is None:
                    batch = [admitted.popleft() for _ in range(min(self.max_batch, len(admitted)))]
                    t = clock() - t0
                    for r in batch:
                        r.start = t
                    self._launch(lane, batch)
            running = sum(len(b[1]) for b in self.busy if b is not None)
            self.peak_running = max(self.peak_running, running)
            if not admitted and not any(self.busy) and arriving and not waiting:
                gap = arriving[0].arrival - (clock() - t0)
                if gap > 2e-3:
                    time.sleep(gap - 1e-3)
        return _stats(reqs, max(r.done for r in reqs))


def fifo(requests: list, device: int = 0, clock: Callable[[], float] = time.perf_counter,
         closed_loop: bool = False, tol: float = 0.0) -> Stats:
    """One request at a time in arrival order, each alone (``sslic_run``)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    if closed_loop:
        for r in reqs:
            r.arrival = 0.0
    ctx = sslic.Context(device)
    t0 = clock()
    for r in reqs:
        while clock() - t0 < r.arrival:
            gap = r.arrival - (clock() - t0)
            if gap > 2e-3:
                time.sleep(gap - 1e-3)
        r.start = clock() - t0
        r.out = ctx.run(r.image, r.S, r.m, r.iterations, tol=tol, connectivity=False, sync=True)
        r.done = clock() - t0
    return _stats(reqs, max(r.done for r in reqs))


def make_requests(trace: list, image_of: Callable, device) -> list:
    """Requests of a synthetic trace [(arrival_s, ImageSpec)] with their images
    generated on ``device`` (standing in for images the caller has uploaded)."""
    out = []
    for t, sp in trace:
        out.append(Request(sp.index, float(t), image_of(sp, device), tuple(sp.S), float(sp.m),
                           int(sp.iterations)))
    return out
