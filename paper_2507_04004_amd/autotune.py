"""Tile-size / blend-depth autotuner for the batched rasterizer.

Times each candidate (tile size in {8, 16, 32}, LDS batch depth in {64, 128, 256}) on the
real workload (the same map and views, graph-captured, fwd or fwd+bwd) and keeps the fastest.
The image does not depend on the choice (every pixel composites the same records in the same
order), so the tuner may pick freely. Results are cached in a JSON file keyed by the workload
shape.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import raster as R
from .batch import BatchPlan, ViewSlot

DEFAULT_CANDIDATES = [(8, 128), (8, 256), (16, 128), (16, 256), (32, 256)]


def workload_key(gm: R.GaussianMap, cams, backward: bool) -> str:
    shapes = ",".join(f"{c.w}x{c.h}@{round(float(c.fx))}" for c in cams)
    return f"n={gm.n};deg={gm.sh_degree};bwd={int(backward)};views={shapes}"


def _time_candidate(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets):
    plan = BatchPlan(gm.n, gm.sh_degree, len(cams), sum(c.w * c.h for c in cams), tile=tile, blend_depth=bd,
                     capacity=capacity, device=device)
    try:
        slots = [ViewSlot.make(c, device, backward=backward, target=targets[i] if targets else None)
                 for i, c in enumerate(cams)]
        if backward and not targets:
            for s, c in zip(slots, cams):  # a fixed upstream gradient stands in for the loss
                s.dL_dC = torch.full((3, c.h, c.w), 1.0 / (3 * c.w * c.h), device=device)
        grads = R.ParamGrads.zeros(gm) if backward else None
        run = lambda: plan.run(gm, slots, fwd=True, bwd=backward, grads=grads, graph=True)
        run()
        if plan.num_pairs() > plan.capacity:
            return float("inf"), plan.num_pairs()
        for _ in range(warmup):
            run()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            run()
            b.record()
        torch.cuda.synchronize()
        return statistics.median(a.elapsed_time(b) for a, b in ev), plan.num_pairs()
    finally:
        plan.close()


def autotune(gm: R.GaussianMap, cams, backward: bool = True, candidates=None, capacity: int | None = None,
             reps: int = 5, warmup: int = 2, device="cuda", cache_path: str | None = None, targets=None,
             verbose: bool = False):
    """Returns (tile, blend_depth, timings) for this workload; consults / updates the cache."""
    key = workload_key(gm, cams, backward)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            e = cache[key]
            return e["tile"], e["blend_depth"], e.get("timings", {})
    timings = {}
    best = None
    for tile, bd in (candidates or DEFAULT_CANDIDATES):
        ms, pairs = _time_candidate(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets)
        timings[f"{tile}x{tile}/{bd}"] = ms
        if verbose:
            print(f"[autotune] tile={tile} depth={bd}: {ms:.3f} ms (pairs {pairs})", flush=True)
        if best is None or ms < best[0]:
            best = (ms, tile, bd)
    _, tile, bd = best
    if cache_path:
        cache[key] = {"tile": tile, "blend_depth": bd, "timings": timings}
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return tile, bd, timings
