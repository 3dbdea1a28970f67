"""Novel-view serving: a resident map answering render requests batched on arrival.

Requests (a camera each; RGB + depth wanted) arrive over time. Whenever the GPU is free the
server takes every request that has arrived, in arrival order, up to 16 views and up to a
memory budget, and renders them with one batched forward (one launch per stage). The map
stays on the device between batches. Latency is arrival -> completion; throughput is output
megapixels per second. `simulate` replays an arrival schedule against the real GPU so the
batched policy and one-at-a-time FIFO can be compared on the same stream of requests.

Admission by memory: a request's estimated device bytes are its output planes (28 B per
pixel: colour, depth, opacity, transmittance, last) plus its share of tile pairs, estimated
from the pairs-per-pixel ratio of recent renders with a safety factor; if a batch still
overflows its pair capacity it is re-run with a larger plan.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import raster as R
from .batch import BatchPlan, ViewSlot

PIXEL_BYTES = 28
PAIR_BYTES = 4 * 6  # vals + two key/value ping-pong buffers per pair during the sort


@dataclasses.dataclass
class Request:
    rid: int
    camera: object
    arrival: float          # seconds since the start of the run
    done: float = math.nan  # completion time
    frame: R.Frame | None = None

    @property
    def pixels(self) -> int:
        return int(self.camera.w) * int(self.camera.h)


class RenderServer:
    def __init__(self, gm: R.GaussianMap, max_batch: int = 16, memory_budget: int = 4 << 30, tile: int = 8,
                 blend_depth: int = 256, device="cuda"):
        self.gm, self.max_batch, self.budget = gm, max_batch, memory_budget
        self.tile, self.bd, self.device = tile, blend_depth, device
        self.pairs_per_pixel = 4.0   # running estimate, refined from completed batches
        self.plans: dict[str, BatchPlan] = {}

    def estimate_bytes(self, req: Request) -> int:
        return int(req.pixels * (PIXEL_BYTES + 1.5 * self.pairs_per_pixel * PAIR_BYTES))

    def admit(self, queue: list[Request]) -> list[Request]:
        """Arrival-order prefix of the queue that fits the batch size and the memory budget."""
        batch, used = [], 0
        for r in queue:
            b = self.estimate_bytes(r)
            if batch and (len(batch) >= self.max_batch or used + b > self.budget):
                break
            batch.append(r)
            used += b
        return batch

    def _plan(self, views: int, pixels: int, pairs: int) -> BatchPlan:
        # one plan sized for max_batch views, grown (re-created) only when a batch needs more
        # pixels or pairs than it holds: its buffers scale with views x map size, so a plan per
        # batch shape would multiply the device memory
        pix_b = 1 << max(16, math.ceil(math.log2(max(pixels, 1))))
        cap = max(1 << 20, int(pairs * 1.5))
        p = self.plans.get("main")
        if p is None or p.capacity < cap or p.max_total_pixels < pixels:
            if p is not None:
                pix_b = max(pix_b, p.max_total_pixels)
                cap = max(cap, p.capacity)
                p.close()
            p = BatchPlan(self.gm.n, self.gm.sh_degree, self.max_batch, pix_b, self.tile, self.bd, cap, self.device)
            self.plans["main"] = p
        return p

    def render(self, batch: list[Request]) -> None:
        pixels = sum(r.pixels for r in batch)
        est_pairs = int(pixels * self.pairs_per_pixel * 1.5) + 4096
        while True:
            plan = self._plan(len(batch), pixels, est_pairs)
            slots = [ViewSlot.make(r.camera, self.device) for r in batch]
            plan.run(self.gm, slots, fwd=True)
            need = plan.num_pairs()  # synchronises the stream
            if need <= plan.capacity:
                break
            est_pairs = int(need * 1.25)
        self.pairs_per_pixel = 0.8 * self.pairs_per_pixel + 0.2 * (need / max(pixels, 1))
        for r, s in zip(batch, slots):
            r.frame = s.frame

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def simulate(server: RenderServer, cams, arrivals, batched: bool = True, keep_frames: bool = False) -> dict:
    """Replay requests arriving at `arrivals` (seconds) against the GPU; return latency stats."""
    reqs = [Request(i, c, float(a)) for i, (c, a) in enumerate(zip(cams, arrivals))]
    pending = list(reqs)
    queue: list[Request] = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    busy = 0.0
    while pending or queue:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.pop(0))
        if not queue:
            wait = pending[0].arrival - now
            if wait > 0:
                time.sleep(wait)
            continue
        batch = server.admit(queue) if batched else queue[:1]
        queue = queue[len(batch):]
        tb = time.perf_counter()
        server.render(batch)  # returns after the batch completed (pair count read back)
        te = time.perf_counter()
        busy += te - tb
        for r in batch:
            r.done = te - t0
            if not keep_frames:
                r.frame = None
    total = time.perf_counter() - t0
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    mpix = sum(r.pixels for r in reqs) / 1e6
    out = {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "mpix_per_s": mpix / total, "busy_frac": busy / total, "wall_s": total}
    if keep_frames:
        out["frames"] = [r.frame for r in reqs]
    return out
