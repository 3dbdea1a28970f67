"""Pin of the float32 binning oracle (bins32.c) against the float64 definition (CPU only).

The float32 tile lists are the expected values of every bit-exact pair-list test of the GPU
path, so they are pinned here against something other than themselves: the float64 oracle's
own tile lists (footprint span and alpha-max cull of Sec. "CUDA-Related Acceleration
Strategies", fast tile-based culling at 1/255; depth order of eq:rendered_rgb), worked cases
whose pair sets are derived by hand, and planted mistakes that must fail.

Agreement rule: a (Gaussian, tile) decision may differ between float32 and float64 only where
its float64 margin (the smallest relative perturbation of the compared quantities that flips
it, `or_pair_margins`) is at most 1e-5; such decisions are counted, and the disagreements
must stay below 1e-4 of the pairs. Within each tile both sides order the Gaussians they both
list alike (float32 depth, then index), and that order is the float64 depth order up to two
float32 roundings of the depth.
"""
import os
import subprocess

import ctypes
import numpy as np
import pytest

import oracle
from paper_2507_04004_amd import scenes as S

from test_oracle_pins import rand_pose, tiny_scene

BAND = 1e-5
HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")


def compare_lists(g, cam, tile, handle=None):
    """Pair sets of float32 and float64 binning on the union of their pairs, with margins."""
    b = oracle.bin32(g, cam, tile=tile, handle=handle)
    L = oracle.lists(g, cam, tile)
    n = max(g.n, 1)
    T = L["start"].size - 1
    k32 = b["tiles"].astype(np.int64) * n + b["vals"].astype(np.int64)
    k64 = np.repeat(np.arange(T), np.diff(L["start"])) * n + L["ids"].astype(np.int64)
    U = np.union1d(k32, k64)
    in32, in64 = np.isin(U, k32), np.isin(U, k64)
    listed, margin = oracle.pair_margins(g, cam, U % n, U // n, tile=tile)
    assert np.array_equal(listed, in64)  # the two float64 exports take the same decisions
    dis = in32 != in64
    clear = margin > BAND
    return dict(pairs=int(U.size), disagree=int(dis.sum()), bad=int((dis & clear).sum()),
                marginal=int((~clear).sum()), worst=float(margin[dis].max(initial=0.0)), b32=b, l64=L)


# A float32 depth is within 8.9 * 2^-24 s of the float64 one, s = max(|mu|, |t|) (the rounding
# of ((R6 mx + R7 my) + R8 mz) + tz, each step at most 2^-24 of a magnitude <= (sqrt(3) + 1) s).
ORDER_BOUND = 2 * 8.9 * 2.0 ** -24


def order_violations(g, cam, tile, r):
    """Depth order inside each tile: both sides order the Gaussians they both list alike (the
    key of R12: float32 depth, then index), and along each list the float64 depths never fall by
    more than two float32 depth roundings (the order is the float64 depth order up to them)."""
    d64 = oracle.project(g, cam)["depth"]
    scale = np.maximum(np.abs(g.mean.astype(np.float64)).max(axis=0), max(1.0, float(np.abs(cam.t_cw).max())))
    b, L = r["b32"], r["l64"]
    tr = b["tile_range"].reshape(-1, 2)
    bad = 0
    for t in range(tr.shape[0]):
        a = b["vals"][tr[t, 0]:tr[t, 1]].astype(np.int64)
        c = L["ids"][L["start"][t]:L["start"][t + 1]].astype(np.int64)
        common = np.intersect1d(a, c)
        if common.size >= 2:
            bad += int(np.sum(a[np.isin(a, common)] != c[np.isin(c, common)]))
        for seq in (a, c):
            if seq.size >= 2:
                runmax = np.maximum.accumulate(d64[seq])
                bad += int(np.sum(d64[seq][1:] < runmax[:-1] - ORDER_BOUND * np.maximum(scale[seq][1:], scale[seq][:-1])))
    return bad


def _scenes():
    out = {}
    g, cam = tiny_scene(0, n=400, W=93, H=61, deg=0)
    out["tiny_ragged"] = (g, cam)
    g, cam = tiny_scene(1, n=400, W=96, H=64, deg=1)
    out["tiny_window"] = (g, cam.window(11, 5, 70, 50))
    g, cam = tiny_scene(2, n=400, W=80, H=56, deg=0)
    R, t = rand_pose(np.random.default_rng(2), 0.1)
    out["tiny_posed"] = (g, S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R, t))
    g, cam, _ = S.config_small(0)
    out["small_frustum"] = (g, cam)
    g = S.street_scene(6000, 5, z_range=(1.0, 40.0), x_half=15.0, n_boxes=6, frac=(0.6, 0.3, 0.1), n_clusters=20,
                       sh_degree=0)
    W, H = 203, 117
    out["street_ragged"] = (g, S.Camera(W, H, 0.7 * W, 0.7 * W, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3)))
    return out


SCENES = _scenes()


@pytest.mark.parametrize("case", list(SCENES))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bins32_agrees_with_fp64_lists(case, tile):
    g, cam = SCENES[case]
    cam = oracle.camera_f32(cam)
    r = compare_lists(g, cam, tile)
    print(f"[bins32] {case} tile {tile}: pairs {r['pairs']} marginal {r['marginal']} disagree {r['disagree']}")
    assert r["pairs"] > 300
    assert r["bad"] == 0, r["worst"]
    assert r["disagree"] <= 1e-4 * r["pairs"]
    assert order_violations(g, cam, tile, r) == 0


def test_bins32_agrees_at_the_benchmark_view():
    """The 1M-Gaussian street map seen by the 1280x720 headline camera at 8x8 tiles (4.3 M
    pairs): the pair lists every full-size GPU test compares against."""
    g = S.street_map(1_000_000, seed=2)
    cam = oracle.camera_f32(S.headline_camera())
    r = compare_lists(g, cam, 8)
    print(f"[bins32] headline: pairs {r['pairs']} marginal {r['marginal']} disagree {r['disagree']} "
          f"(largest margin of a disagreement {r['worst']:.1e})")
    assert r["pairs"] > 4_000_000
    assert r["bad"] == 0
    assert r["disagree"] <= 1e-4 * r["pairs"]
    assert r["marginal"] <= 2e-3 * r["pairs"]


# ---- worked cases -----------------------------------------------------------------------------
# One isotropic Gaussian (scale s, identity rotation) on the optical axis of an identity-pose
# camera at depth z = fx: J = I, Sigma' = (s^2 + 0.3) I, the conic is isotropic (b = 0), so the
# smallest q over a tile is a (dx^2 + dy^2) with dx, dy the per-axis distances from the centre
# to the tile's pixel-centre rectangle, and the footprint half-extent is h = sqrt(kappa^2 s00).
# Tiles are 8x8 over a 24x24 image: pixel-centre ranges [0, 7], [8, 15], [16, 23].

def _one(cx, cy, s, o, x=0.0, y=0.0, f=16.0, W=24):
    g = S.Gaussians(np.array([[x], [y], [f]], np.float32), np.full((3, 1), s, np.float32),
                    np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), np.array([o], np.float32),
                    np.zeros((3, 1), np.float32), np.zeros((0, 1), np.float32), 0)
    return g, S.Camera(W, W, f, f, cx, cy, np.eye(3), np.zeros(3))


def _opacity_for(kappa2):
    return float(np.exp(kappa2 / 2.0) / 255.0)


def _pairs(g, cam):
    b = oracle.bin32(g, cam, tile=8)
    L = oracle.lists(g, cam, 8)
    t32 = sorted((int(t) % 3, int(t) // 3) for t in b["tiles"])
    t64 = sorted((int(t) % 3, int(t) // 3) for t in np.repeat(np.arange(9), np.diff(L["start"])))
    return t32, t64


WORKED = {
    # centre on the corner shared by four tiles, (7.5, 7.5): each tile's nearest pixel centre is
    # (0.5, 0.5) away, q_min = 0.5 / 0.55. kappa^2 = 2 ln(127.5) = 9.70 keeps all four ...
    "corner_all_four": (dict(cx=7.5, cy=7.5, s=0.5, o=0.5), [(0, 0), (0, 1), (1, 0), (1, 1)]),
    # ... and kappa^2 = 2 ln(1.275) = 0.486 < 0.909 culls all four, though the footprint
    # span (h = 0.52, pixels 7..8) still covers them.
    "corner_culled": (dict(cx=7.5, cy=7.5, s=0.5, o=0.005), []),
    # centre at (7.5, 7.0): row-0 tiles have q_min = 0.25 / 0.55 = 0.45, row-1 tiles
    # (1.25) / 0.55 = 2.27; kappa^2 = 2 keeps row 0 only, while the span (h = 1.05, rows
    # 6..8) reaches row 1.
    "corner_two_of_four": (dict(cx=7.5, cy=7.0, s=0.5, o=_opacity_for(2.0)), [(0, 0), (1, 0)]),
    # centre (4, 4), s00 = 2.55, h = 4.001: the span's upper end floor(8.001) = 8 is the first
    # pixel of tile 1, and q = 16 / 2.55 <= kappa^2 = 4.001^2 / 2.55 there (the diagonal tile
    # has q = 32 / 2.55 and is culled) ...
    "span_end_reached": (dict(cx=4.0, cy=4.0, s=1.5, o=_opacity_for(4.001 ** 2 / 2.55)), [(0, 0), (0, 1), (1, 0)]),
    # ... and h = 3.999 stops at pixel 7: tile 0 alone.
    "span_end_missed": (dict(cx=4.0, cy=4.0, s=1.5, o=_opacity_for(3.999 ** 2 / 2.55)), [(0, 0)]),
    # centre (12, 12) in the middle tile, h = 5.001: ceil(6.999) = 7 reaches the last pixel
    # column of tile 0 and floor(17.001) the first of tile 2; with per-axis distances 5 (tile
    # 0) and 4 (tile 2) the kept tiles are those with dx^2 + dy^2 <= 25.01: a plus sign ...
    "span_both_ends": (dict(cx=12.0, cy=12.0, s=1.5, o=_opacity_for(5.001 ** 2 / 2.55)),
                       [(0, 1), (1, 0), (1, 1), (1, 2), (2, 1)]),
    # ... and at h = 4.999, ceil(7.001) = 8: the distance-5 tiles drop out.
    "span_lower_end_missed": (dict(cx=12.0, cy=12.0, s=1.5, o=_opacity_for(4.999 ** 2 / 2.55)),
                              [(1, 1), (1, 2), (2, 1)]),
}


@pytest.mark.parametrize("case", list(WORKED))
def test_worked_tile_decisions(case):
    kw, expect = WORKED[case]
    g, cam = _one(**kw)
    t32, t64 = _pairs(g, cam)
    assert t32 == sorted(expect), (case, t32)
    assert t64 == sorted(expect), (case, t64)
    if expect:  # every decision of these cases is far from its threshold
        r = compare_lists(g, cam, 8)
        assert r["marginal"] == 0 and r["disagree"] == 0


def test_worked_offset_centre_y():
    """The centre moved off the axis by y = -0.5 m at z = 16: v = 16 (-0.5 / 16) + cy exactly."""
    g, cam = _one(cx=7.5, cy=7.5, s=0.5, o=_opacity_for(2.0), y=-0.5)
    t32, t64 = _pairs(g, cam)
    assert t32 == t64 == [(0, 0), (1, 0)]


# ---- planted mistakes: a wrong float32 mirror must fail the pin ---------------------------------
MUTANTS = {
    # the footprint span's upper end one pixel short
    "span_off_by_one": ("xhi = fminf(floorf(u + hx), ", "xhi = fminf(floorf(u + hx) - 1.0f, "),
    # the far vertical edge instead of the one facing the centre
    "wrong_facing_edge": ("float X = (u < xl) ? xl : xh;", "float X = (u < xl) ? xh : xl;"),
}


def _build_mutant(tmp_path, name):
    src = open(os.path.join(ORACLE_DIR, "bins32.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / f"bins32_{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"bins32_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                    "-D_DEFAULT_SOURCE", "-o", str(lib), str(path), "-lm"], check=True)
    return oracle.bind_bin32(ctypes.CDLL(str(lib)))


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_binning_mistakes_fail(tmp_path, name):
    handle = _build_mutant(tmp_path, name)
    failed = []
    for case in ("tiny_ragged", "street_ragged"):
        g, cam = SCENES[case]
        cam = oracle.camera_f32(cam)
        for tile in (8, 16):
            r = compare_lists(g, cam, tile, handle=handle)
            failed.append(r["bad"] > 0)
    worked = []
    for kw, expect in WORKED.values():
        g, cam = _one(**kw)
        b = oracle.bin32(g, cam, tile=8, handle=handle)
        worked.append(sorted((int(t) % 3, int(t) // 3) for t in b["tiles"]) != sorted(expect))
    print(f"[bins32] mutant {name}: scene checks failing {sum(failed)}/4, worked cases failing {sum(worked)}")
    assert any(failed) and any(worked)
