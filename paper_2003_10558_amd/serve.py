"""Continuous-batching view server over resident scenes.

Requests (scene, view) arrive over time.  The server keeps every scene's
setup resident on the GPU and runs a loop that

* moves requests whose arrival time has passed into the admission queue,
* retires finished batches (event queries; no blocking synchronisation),
  releasing their device memory from the budget,
* admits queued requests into a new batch whenever one of its in-flight
  slots (one HIP stream each) is free and the batch fits the HBM budget,
  and submits it with one vsr_submit call on that slot's stream,

so requests that arrive while others are on the GPU join the next batch as
soon as a slot and memory free up, and batches on different streams overlap
on the device.  Latency is completion time minus scheduled arrival time.

Nothing here computes any part of the method; the batches run in the HIP
library.  Each request's images are bit-identical whether rendered alone or
inside any batch (the batched kernels run the single-view per-tile code).
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import pipeline, vsr


@dataclass
class Request:
    rid: int
    scene: int
    view: object
    arrival: float            # scheduled arrival, seconds from the start of the run
    admitted: float = math.nan
    done: float = math.nan
    dropped: bool = False
    result: Optional[tuple] = None  # (ids uint32 [H,W], depth float32 [H,W]) when kept


@dataclass
class ServeStats:
    offered: int = 0
    completed: int = 0
    dropped: int = 0
    wall_s: float = 0.0
    views_per_s: float = 0.0
    p50_ms: float = math.nan
    p99_ms: float = math.nan
    mean_ms: float = math.nan
    queue_p50_ms: float = math.nan
    queue_p99_ms: float = math.nan
    batches: int = 0
    mean_batch: float = 0.0
    max_inflight_bytes: int = 0
    budget_bytes: int = 0
    pixels: int = 0
    batch_size_hist: dict = field(default_factory=dict)    # batch size -> batches
    queue_depth_hist: dict = field(default_factory=dict)   # requests waiting at an admission -> admissions
    queue_wait_hist_ms: dict = field(default_factory=dict)  # upper edge of the wait bin (ms) -> requests
    overlapped_batches: int = 0   # batches whose device interval intersects another batch's
    max_concurrent_batches: int = 0
    extra: dict = field(default_factory=dict)

    def as_dict(self) -> dict:
        d = dict(self.__dict__)
        d.update(d.pop("extra"))
        return d


def request_bytes(view, fmt: int, mode: int, bin_depth: int) -> int:
    """Device bytes one request holds while in flight: its outputs and its
    share of the batch workspace."""
    w, h = int(view.width), int(view.height)
    out = w * h * 8
    ws = vsr.vsr_map_bytes(w, h, fmt)
    ws += vsr.vsr_render_bytes(w, h) if mode == vsr.VSR_SUBMIT_FUSED else vsr.vsr_bin_bytes(w, h, bin_depth)
    return out + ws + 1024


class Server:
    """Continuous batching over `scenes` (pipeline.Scene) on one GPU."""

    def __init__(self, scenes: Sequence[pipeline.Scene], streams: int = 2, max_batch: int = 32,
                 hbm_budget_bytes: int = 32 << 30, fmt: int = vsr.VSR_MAP_F32,
                 mode_for_scene: Optional[Callable[[int], tuple]] = None, max_queue_s: float = 5.0,
                 poll_s: float = 50e-6):
        self.scenes = list(scenes)
        self.fmt = fmt
        self.max_batch = max_batch
        self.budget = int(hbm_budget_bytes)
        self.max_queue_s = max_queue_s
        self.poll_s = poll_s
        self.streams = [torch.cuda.Stream(device=self.scenes[0].device) for _ in range(streams)]
        # (mode, bin_depth) per scene, e.g. from the autotuner
        self.mode_for_scene = mode_for_scene or (lambda s: (vsr.VSR_SUBMIT_FUSED, 1024))

    def run(self, requests: Sequence[Request], keep: Optional[set] = None) -> ServeStats:
        """Serve `requests` (sorted by arrival).  Request ids in `keep` get
        their images copied back into Request.result."""
        keep = keep or set()
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        free_slots = list(range(len(self.streams)))
        inflight: List[tuple] = []   # (end event, slot, reqs, bytes, batch, start event)
        used = 0
        st = ServeStats(offered=len(requests), budget_bytes=self.budget)
        batch_sizes, queue_depths = [], []
        intervals = []  # (start, end) in ms after ref_ev per batch: its device interval
        ref_ev = torch.cuda.Event(enable_timing=True)
        ref_ev.record(self.streams[0])
        t0 = time.perf_counter()
        while pending or queue or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # retire finished batches
            still = []
            for item in inflight:
                ev, slot, reqs, nbytes, batch, ev0 = item
                if ev.query():
                    # device interval of the batch (the events are released here)
                    intervals.append((ref_ev.elapsed_time(ev0), ref_ev.elapsed_time(ev)))
                    tdone = time.perf_counter() - t0
                    for q, r in enumerate(reqs):
                        r.done = tdone
                        if r.rid in keep:
                            ids, dep = batch.outputs[q]
                            r.result = (ids.cpu().numpy().view(np.uint32).copy(), dep.cpu().numpy().copy())
                    used -= nbytes
                    free_slots.append(slot)
                else:
                    still.append(item)
            inflight = still
            # drop requests that waited too long
            while queue and now - queue[0].arrival > self.max_queue_s:
                r = queue.popleft()
                r.dropped = True
            # admit
            admitted_any = False
            while free_slots and queue:
                queue_depths.append(len(queue))
                mode, depth = self.mode_for_scene(queue[0].scene)
                reqs, nbytes = [], 0
                rest = collections.deque()
                while queue and len(reqs) < self.max_batch:
                    r = queue.popleft()
                    if self.mode_for_scene(r.scene) != (mode, depth):
                        rest.append(r)
                        continue
                    b = request_bytes(r.view, self.fmt, mode, depth)
                    if used + nbytes + b > self.budget and reqs:
                        rest.append(r)
                        break
                    reqs.append(r)
                    nbytes += b
                queue.extendleft(reversed(rest))
                if not reqs:
                    break
                if used + nbytes > self.budget and inflight:
                    queue.extendleft(reversed(reqs))
                    break
                slot = free_slots.pop()
                stream = self.streams[slot]
                tadm = time.perf_counter() - t0
                with torch.cuda.stream(stream):
                    batch = pipeline.Batch([(self.scenes[r.scene], r.view) for r in reqs], fmt=self.fmt,
                                           mode=mode, bin_depth=depth)
                    ev0 = torch.cuda.Event(enable_timing=True)
                    ev0.record(stream)
                    batch.submit(stream)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(stream)

                for r in reqs:
                    r.admitted = tadm
                used += nbytes
                st.max_inflight_bytes = max(st.max_inflight_bytes, used)
                inflight.append((ev, slot, reqs, nbytes, batch, ev0))
                batch_sizes.append(len(reqs))
                admitted_any = True
            if not admitted_any:
                if inflight or (pending and pending[0].arrival - (time.perf_counter() - t0) < 1e-3):
                    time.sleep(self.poll_s)
                elif pending:
                    time.sleep(min(1e-3, max(0.0, pending[0].arrival - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        torch.cuda.synchronize()
        # device intervals of the batches (ms after the reference event); a
        # batch overlaps when another batch's interval intersects its own
        iv = np.array(intervals, dtype=np.float64).reshape(-1, 2)
        if len(iv):
            order = np.argsort(iv[:, 0])
            iv = iv[order]
            over = np.zeros(len(iv), bool)
            end_max, end_arg = -np.inf, -1
            for k in range(len(iv)):
                if iv[k, 0] < end_max:
                    over[k] = True
                    over[end_arg] = True
                if iv[k, 1] > end_max:
                    end_max, end_arg = iv[k, 1], k
            st.overlapped_batches = int(over.sum())
            ev_t = np.concatenate([np.stack([iv[:, 0], np.ones(len(iv))], 1), np.stack([iv[:, 1], -np.ones(len(iv))], 1)])
            ev_t = ev_t[np.lexsort((ev_t[:, 1], ev_t[:, 0]))]
            st.max_concurrent_batches = int(np.max(np.cumsum(ev_t[:, 1])))
        st.batch_size_hist = {int(k): int(v) for k, v in zip(*np.unique(batch_sizes, return_counts=True))} \
            if batch_sizes else {}
        qd_edges = [0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 1 << 30]
        qd = np.histogram(queue_depths, bins=qd_edges)[0] if queue_depths else np.zeros(len(qd_edges) - 1, int)
        st.queue_depth_hist = {f"{qd_edges[k]}-{qd_edges[k + 1] - 1}" if k + 2 < len(qd_edges) else
                               f">={qd_edges[k]}": int(qd[k]) for k in range(len(qd))}
        done = [r for r in requests if not r.dropped and not math.isnan(r.done)]
        st.completed = len(done)
        st.dropped = sum(1 for r in requests if r.dropped)
        st.wall_s = wall
        st.batches = len(batch_sizes)
        st.mean_batch = float(np.mean(batch_sizes)) if batch_sizes else 0.0
        st.pixels = int(sum(int(r.view.width) * int(r.view.height) for r in done))
        if done:
            lat = np.array([(r.done - r.arrival) * 1e3 for r in done])
            qd = np.array([(r.admitted - r.arrival) * 1e3 for r in done])
            st.p50_ms, st.p99_ms, st.mean_ms = (float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                                                float(lat.mean()))
            st.queue_p50_ms, st.queue_p99_ms = float(np.percentile(qd, 50)), float(np.percentile(qd, 99))
            w_edges = [0.0, 0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, np.inf]
            wh = np.histogram(qd, bins=w_edges)[0]
            st.queue_wait_hist_ms = {(f"<{w_edges[k + 1]:g}" if np.isfinite(w_edges[k + 1]) else f">={w_edges[k]:g}"):
                                     int(wh[k]) for k in range(len(wh))}
            last = max(r.done for r in done)
            first = min(r.arrival for r in requests)
            st.views_per_s = st.completed / max(1e-9, last - first)
        return st


def make_requests(n_scenes: int, rate_hz: float, duration_s: float, seed: int, view_seed: int,
                  resolutions) -> List[Request]:
    """Poisson arrivals; each request picks a scene and a random view."""
    import synth
    times = synth.poisson_arrivals(rate_hz, duration_s, seed)
    views = synth.random_views(len(times), view_seed, resolutions=resolutions)
    rng = np.random.default_rng(seed + 1000)
    scenes = rng.integers(0, n_scenes, size=len(times))
    return [Request(i, int(scenes[i]), views[i], float(times[i])) for i in range(len(times))]
