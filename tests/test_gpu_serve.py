"""Serving loop and autotuner (needs an MI355X).

Every served frame, batched or one at a time, must match the float64 oracle's render of its
camera (1e-4 on pixels the oracle does not flag as marginal) and equal the plain single-view
render of the same camera bitwise (the batch path runs the same per-pixel arithmetic); the
autotuner must pick one of its candidates and cache it.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S
from paper_2507_04004_amd.autotune import autotune
from paper_2507_04004_amd.serve import RenderServer, poisson_arrivals, simulate

import oracle

from gpu_common import DEV, HipRun, assert_images_close, oracle_cam

pytestmark = pytest.mark.gpu


def small_map(n=20000, seed=41):
    return S.street_map(n, seed=seed, z_range=(-5.0, 120.0), n_boxes=20, n_clusters=40)


def small_requests(k, seed):
    rng = np.random.default_rng(seed)
    res = [(160, 90), (320, 180), (480, 270)]
    cams = []
    for _ in range(k):
        W, H = res[int(rng.integers(0, 3))]
        cams.append(S.look_camera((float(rng.uniform(-2, 2)), 0.0, float(rng.uniform(0, 100))),
                                  float(rng.uniform(-30, 30)), float(rng.uniform(-5, 5)), W, H, 0.8 * W))
    return cams


@pytest.mark.parametrize("batched", [True, False])
def test_served_frames_equal_plain_renders(batched):
    g = small_map()
    gm = R.GaussianMap.from_numpy(g, DEV)
    cams = small_requests(12, seed=3)
    server = RenderServer(gm, max_batch=16, memory_budget=1 << 30, device=DEV)
    arrivals = poisson_arrivals(len(cams), rate=2000.0, seed=1)
    stats = simulate(server, cams, arrivals, batched=batched, keep_frames=True)
    assert stats["requests"] == len(cams) and stats["p99_ms"] >= stats["p50_ms"] > 0
    # every served frame matches the oracle and equals the plain single-view render of its camera
    for i, (c, fr) in enumerate(zip(cams, stats["frames"])):
        got = {key: getattr(fr, key).cpu().numpy() for key in ("color", "depth", "alpha", "t_final")}
        e = assert_images_close(got, oracle.render(g, oracle_cam(c), tile=16, band=1e-4))
        print(f"[serve] batched={batched} request {i} {c.w}x{c.h}: {e}", flush=True)
        ref = HipRun(g, c, tile=server.tile, blend_depth=server.bd).image()
        for key in ("color", "depth", "alpha", "t_final"):
            assert np.array_equal(got[key], ref[key]), (i, key)
    server.close()


def test_admission_respects_budget_and_batch_size():
    """Admitted batches fit the budget with the memory the server then allocates: the plan it
    renders them with (forward-only, sized for the batch) and the output planes."""
    from paper_2507_04004_amd.serve import PIXEL_BYTES, Request
    g = small_map(20000)
    gm = R.GaussianMap.from_numpy(g, DEV)
    cams = small_requests(10, seed=5)
    one = RenderServer(gm, device=DEV).batch_bytes([Request(0, cams[0], 0.0)])
    budget = int(2.5 * one)
    server = RenderServer(gm, max_batch=4, memory_budget=budget, device=DEV)
    queue = [Request(i, c, 0.0) for i, c in enumerate(cams)]
    served = 0
    while queue:
        batch = server.admit(queue)
        assert 1 <= len(batch) <= 4
        assert [r.rid for r in batch] == list(range(served, served + len(batch)))  # arrival order
        est = server.batch_bytes(batch)
        assert est <= budget or len(batch) == 1
        server.render(batch)
        held = server.plan.nbytes + sum(r.frame.color.numel() * 4 + r.frame.depth.numel() * 4 +
                                        r.frame.alpha.numel() * 4 + r.frame.t_final.numel() * 4 +
                                        r.frame.last.numel() * 4 for r in batch)
        frames = sum(r.pixels for r in batch) * PIXEL_BYTES
        assert held - frames == server.plan.nbytes
        assert held <= max(budget, est), (held, budget, est)
        assert server.plan.fwd_only
        queue = queue[len(batch):]
        served += len(batch)
    server.close()


def test_autotune_picks_a_candidate_and_caches(tmp_path):
    g = small_map(10000)
    gm = R.GaussianMap.from_numpy(g, DEV)
    cams = small_requests(3, seed=7)
    cache = str(tmp_path / "tune.json")
    cands = [(8, 64), (16, 128), (16, 256)]
    tile, bd, sched, timings = autotune(gm, cams, backward=True, candidates=cands, reps=3, warmup=1, device=DEV,
                                 cache_path=cache)
    assert (tile, bd) in cands and len(timings) == 3
    assert all(np.isfinite(v) and v > 0 for v in timings.values())
    with open(cache) as fh:
        assert len(json.load(fh)) == 1
    # cached answer comes back without re-timing
    t2, b2, s2, _ = autotune(gm, cams, backward=True, candidates=cands, cache_path=cache, device=DEV)
    assert (t2, b2, s2) == (tile, bd, sched)
