"""Autotuner selection logic without a GPU: the timing of one candidate is replaced by a stub,
so the test checks which candidates are tried (the bucketed schedule only at 8x8 and 16x16,
no duplicates, no schedule without a backward), that the fastest is kept, and that the cache
returns the same choice, schedule included."""
import dataclasses
import json

import numpy as np

from paper_2507_04004_amd import _native as N
from paper_2507_04004_amd import autotune as A


@dataclasses.dataclass
class _Map:
    n: int = 1000
    sh_degree: int = 3


@dataclasses.dataclass
class _Cam:
    w: int = 64
    h: int = 48
    fx: float = 50.0


def test_candidates_selection_and_cache(monkeypatch, tmp_path):
    tried = []
    cost = {(8, 128, 0): 5.0, (8, 256, 0): 6.0, (16, 128, 0): 7.0, (16, 256, 0): 8.0, (32, 256, 0): 9.0,
            (8, 128, 1): 4.0, (16, 128, 1): 4.5}

    def fake(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets, schedule):
        tried.append((tile, bd, schedule))
        return cost.get((tile, bd, schedule), 10.0 + bd / 1000.0), 123

    monkeypatch.setattr(A, "_time_candidate", fake)
    cache = tmp_path / "tune.json"
    # the default search: tile sides {8, 16, 32} squared, chunk lengths {32, ..., 256}
    assert len(A.DEFAULT_CANDIDATES) == 9 * 4 + 2
    assert {(8, 16), (32, 8), (16, 32)} <= {c[0] for c in A.DEFAULT_CANDIDATES if not isinstance(c[0], int)}
    assert {c[1] for c in A.DEFAULT_CANDIDATES} == {32, 64, 128, 256}
    cands = A.DEFAULT_CANDIDATES + [(8, 128), ((8, 8), 128), (32, 256, N.GS_BWD_BUCKETS),
                                    ((16, 32), 64, N.GS_BWD_BUCKETS)]
    r = A.autotune_config(_Map(), [_Cam()], backward=True, candidates=cands, cache_path=str(cache))
    assert (r["tile"], r["blend_depth"], r["schedule"]) == (8, 128, N.GS_BWD_BUCKETS)
    # duplicates (also (8, 8) for 8) and buckets on tiles over 256 pixels skipped
    assert len(tried) == len(set(tried)) == 38
    assert (32, 256, N.GS_BWD_BUCKETS) not in tried and ((16, 32), 64, N.GS_BWD_BUCKETS) not in tried
    assert r["timings"]["16x32/64"] > 0 and "8x16/32" in r["timings"]
    assert r["timings"]["8x8/128/buckets"] == 4.0 and r["timings"]["8x8/128"] == 5.0
    # the cache answers without timing again, schedule included
    tried.clear()
    r2 = A.autotune_config(_Map(), [_Cam()], backward=True, candidates=cands, cache_path=str(cache))
    assert not tried and r2["schedule"] == N.GS_BWD_BUCKETS and r2["tile"] == 8
    assert json.loads(cache.read_text())
    # the tuple form carries the schedule with the tile and depth
    t, b, sched, timings = A.autotune(_Map(), [_Cam()], backward=True, candidates=cands, cache_path=str(cache))
    assert (t, b, sched) == (8, 128, N.GS_BWD_BUCKETS) and "8x8/128/buckets" in timings
    # another candidate set is another cache entry: tuned again, not answered from the first
    tried.clear()
    r3 = A.autotune_config(_Map(), [_Cam()], backward=True, candidates=[(16, 256), (32, 256)],
                           cache_path=str(cache))
    assert tried == [(16, 256, 0), (32, 256, 0)] and (r3["tile"], r3["blend_depth"]) == (16, 256)
    assert len(json.loads(cache.read_text())) == 2


def test_forward_only_ignores_schedules(monkeypatch):
    tried = []

    def fake(gm, cams, tile, bd, backward, capacity, reps, warmup, device, targets, schedule):
        tried.append((tile, bd, schedule))
        tw, th = (tile, tile) if isinstance(tile, int) else tile
        return float(tw * th + bd / 1000.0 + np.float64(schedule)), 1

    monkeypatch.setattr(A, "_time_candidate", fake)
    r = A.autotune_config(_Map(), [_Cam()], backward=False)
    assert all(s == N.GS_BWD_CHUNKS for _, _, s in tried)
    assert len(tried) == len(set(tried))
    assert r["schedule"] == N.GS_BWD_CHUNKS and r["tile"] == 8 and r["blend_depth"] == 32
    assert len(tried) == 36
