"""Tile-size / blend-depth / backward-schedule autotuner for the batched rasterizer.

Times each candidate (tile sides in {8, 16, 32}, square or not; LDS batch depth in {32, 64, 128,
256}; and for a backward the compositing-backward schedule: pixel-parallel chunks or
per-Gaussian buckets) on
the real workload (the same map and views, graph-captured, fwd or fwd+bwd) and keeps the
fastest. The image does not depend on the choice (every pixel composites the same records in
the same order) and the gradients only through float32 summation order, so the tuner may pick
freely. Results are cached in a JSON file keyed by the workload shape.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import _native as N
from . import raster as R
from .batch import BatchPlan, ViewSlot

# (tile, chunk length[, backward schedule]): every tile of sides 8, 16, 32 (square sides as one
# number) with every chunk length 32-256 under the pixel-parallel backward, and the bucketed
# backward (tiles of at most 256 pixels) at the two square shapes it runs on
SIDES = (8, 16, 32)
DEPTHS = (32, 64, 128, 256)
DEFAULT_CANDIDATES = [((tw if tw == th else (tw, th)), bd) for tw in SIDES for th in SIDES for bd in DEPTHS] + \
    [(8, 128, N.GS_BWD_BUCKETS), (16, 128, N.GS_BWD_BUCKETS)]
SCHEDULE_NAMES = {N.GS_BWD_CHUNKS: "chunks", N.GS_BWD_BUCKETS: "buckets"}


def _split(c):
    return (c[0], c[1], c[2]) if len(c) > 2 else (c[0], c[1], N.GS_BWD_CHUNKS)


def candidate_key(tile, bd, schedule=N.GS_BWD_CHUNKS) -> str:
    tw, th = R.tile_wh(tile)
    k = f"{tw}x{th}/{bd}"
    return k if schedule == N.GS_BWD_CHUNKS else f"{k}/{SCHEDULE_NAMES[schedule]}"


def workload_key(gm: R.GaussianMap, cams, backward: bool, candidates=None) -> str:
    """Cache key: the workload's shape and the candidate set it was tuned over."""
    shapes = ",".join(f"{c.w}x{c.h}@{round(float(c.fx))}" for c in cams)
    cands = ",".join(sorted({candidate_key(*_split(c)) for c in (candidates or DEFAULT_CANDIDATES)}))
    return f"n={gm.n};deg={gm.sh_degree};bwd={int(backward)};views={shapes};candidates={cands}"


def _time_candidate(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets, schedule):
    plan = BatchPlan(gm.n, gm.sh_degree, len(cams), sum(c.w * c.h for c in cams), tile=tile, blend_depth=bd,
                     capacity=capacity, device=device)
    try:
        slots = [ViewSlot.make(c, device, backward=backward, target=targets[i] if targets else None)
                 for i, c in enumerate(cams)]
        if backward and not targets:
            for s, c in zip(slots, cams):  # a fixed upstream gradient stands in for the loss
                s.dL_dC = torch.full((3, c.h, c.w), 1.0 / (3 * c.w * c.h), device=device)
        grads = R.ParamGrads.zeros(gm) if backward else None
        run = lambda: plan.run(gm, slots, fwd=True, bwd=backward, grads=grads, graph=True, schedule=schedule)
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


def autotune_config(gm: R.GaussianMap, cams, backward: bool = True, candidates=None, capacity: int | None = None,
                    reps: int = 5, warmup: int = 2, device="cuda", cache_path: str | None = None, targets=None,
                    verbose: bool = False) -> dict:
    """{"tile", "blend_depth", "schedule", "timings"} of the fastest candidate for this workload;
    consults / updates the cache. Without a backward the schedule plays no part."""
    key = workload_key(gm, cams, backward, candidates)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            e = cache[key]
            return {"tile": e["tile"], "blend_depth": e["blend_depth"],
                    "schedule": e.get("schedule", N.GS_BWD_CHUNKS), "timings": e.get("timings", {})}
    timings = {}
    best = None
    seen = set()
    for c in (candidates or DEFAULT_CANDIDATES):
        tile, bd, sched = _split(c)
        if not backward:
            sched = N.GS_BWD_CHUNKS
        tw, th = R.tile_wh(tile)
        tile = tw if tw == th else (tw, th)
        if (tile, bd, sched) in seen or (sched == N.GS_BWD_BUCKETS and tw * th > 256):
            continue
        seen.add((tile, bd, sched))
        ms, pairs = _time_candidate(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets, sched)
        timings[candidate_key(tile, bd, sched)] = ms
        if verbose:
            print(f"[autotune] tile={tile} depth={bd} schedule={SCHEDULE_NAMES[sched]}: {ms:.3f} ms "
                  f"(pairs {pairs})", flush=True)
        if best is None or ms < best[0]:
            best = (ms, tile, bd, sched)
    _, tile, bd, sched = best
    out = {"tile": tile, "blend_depth": bd, "schedule": sched, "timings": timings}
    if cache_path:
        cache[key] = out
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return out


def autotune(gm: R.GaussianMap, cams, backward: bool = True, candidates=None, capacity: int | None = None,
             reps: int = 5, warmup: int = 2, device="cuda", cache_path: str | None = None, targets=None,
             verbose: bool = False):
    """(tile, blend_depth, schedule, timings) of autotune_config: the schedule is part of the
    choice (a tile size and depth timed under the bucketed schedule are only the fastest with it)."""
    r = autotune_config(gm, cams, backward, candidates, capacity, reps, warmup, device, cache_path, targets, verbose)
    return r["tile"], r["blend_depth"], r["schedule"], r["timings"]
