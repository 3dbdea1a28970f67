"""Novel-view serving: a resident map answering render requests batched on arrival.

Requests (a camera each; RGB + depth wanted) arrive over time. Whenever the GPU is free the
server takes every request that has arrived, in arrival order, up to 16 views and up to a
memory budget, and renders them with one batched forward (one launch per stage). The map
stays on the device between batches. Latency is arrival -> completion; throughput is output
megapixels per second. `simulate` replays an arrival schedule against the real GPU so the
batched policy and one-at-a-time FIFO can be compared on the same stream of requests.

Admission by memory: the device bytes of a batch are those of a forward-only batch plan sized
for it (splat records of every view, tile lists, sort and compositing scratch; the pair
capacity from the pairs-per-pixel ratio of recent renders with a safety factor) plus each
request's output planes (28 B per pixel: colour, depth, opacity, transmittance, last). Requests
are admitted in arrival order while that total stays within the budget (a single request
larger than the budget is served alone). The server keeps one plan and re-creates it when a
batch needs more views, pixels or pairs than it holds; if a batch still overflows its pair
capacity it is re-run with a larger plan.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np
import torch

from . import raster as R
from .batch import BatchPlan, ViewSlot, plan_bytes

PIXEL_BYTES = 28


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
        self.plan: BatchPlan | None = None

    def _sizes(self, reqs: list[Request]) -> tuple[int, int, int]:
        """Plan arguments for a batch: views, total pixels, pair capacity."""
        pixels = sum(r.pixels for r in reqs)
        return len(reqs), pixels, max(1 << 16, int(pixels * self.pairs_per_pixel * 1.5) + 4096)

    def _plan_bytes(self, views: int, pixels: int, cap: int) -> int:
        return plan_bytes(self.gm.n, self.gm.sh_degree, views, pixels, self.tile, self.bd, cap, fwd_only=True)

    def batch_bytes(self, reqs: list[Request]) -> int:
        """Device bytes of a batch: its forward-only plan and the requests' output planes."""
        return self._plan_bytes(*self._sizes(reqs)) + sum(r.pixels for r in reqs) * PIXEL_BYTES

    def estimate_bytes(self, req: Request) -> int:
        return self.batch_bytes([req])

    def admit(self, queue: list[Request]) -> list[Request]:
        """Arrival-order prefix of the queue that fits the batch size and the memory budget."""
        batch: list[Request] = []
        for r in queue:
            if len(batch) >= self.max_batch or (batch and self.batch_bytes(batch + [r]) > self.budget):
                break
            batch.append(r)
        return batch

    def _plan_for(self, views: int, pixels: int, cap: int) -> BatchPlan:
        p = self.plan
        if p is not None and p.max_views >= views and p.max_total_pixels >= pixels and p.capacity >= cap:
            return p
        if p is not None:
            # grow to cover both shapes when that still fits the budget, else fit this batch
            both = (max(views, p.max_views), max(pixels, p.max_total_pixels), max(cap, p.capacity))
            if self._plan_bytes(*both) + pixels * PIXEL_BYTES <= self.budget:
                views, pixels, cap = both
            p.close()
            self.plan = None
        self.plan = BatchPlan(self.gm.n, self.gm.sh_degree, views, pixels, self.tile, self.bd, cap, self.device,
                              fwd_only=True)
        return self.plan

    def render(self, batch: list[Request]) -> None:
        views, pixels, cap = self._sizes(batch)
        while True:
            plan = self._plan_for(views, pixels, cap)
            slots = [ViewSlot.make(r.camera, self.device) for r in batch]
            plan.run(self.gm, slots, fwd=True)
            need = plan.num_pairs()  # synchronises the stream
            if need <= plan.capacity:
                break
            cap = int(need * 1.25)
        self.pairs_per_pixel = 0.8 * self.pairs_per_pixel + 0.2 * (need / max(pixels, 1))
        for r, s in zip(batch, slots):
            r.frame = s.frame

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None


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
