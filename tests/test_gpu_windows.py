"""Windowed forward compositing against the oracle (needs an MI355X).

The forward composites and scans a tile's chunks in windows (the first 512 splats of its list,
up to 2048, the rest) and goes on to a window only while some pixel of the tile is still
running. The scene heaps hundreds to thousands of small splats on each tile of a 32x16 view,
so pixels stop in each of the three windows and some never stop, at every chunk length;
images and gradients must match the oracle (the bars of the other parity tests), and the run
must show stopped pixels whose last blended splat lies in each window.
"""
import numpy as np
import pytest

import oracle
from paper_2507_04004_amd import scenes as S

from gpu_common import HipRun, assert_grads_close, assert_images_close, marginal_gaussians, oracle_cam

pytestmark = pytest.mark.gpu

WIN0, WIN1 = 512, 2048


# (tile x, tile y, splats, opacity range): a few hundred splats stop the pixels of a tile
# early, a few thousand faint ones late, and sparse tiles never stop
STACKS = [(0, 0, 400, 0.1, 0.3), (1, 0, 2500, 0.04, 0.1), (2, 0, 6000, 0.02, 0.05), (3, 0, 150, 0.05, 0.1),
          (0, 1, 1200, 0.06, 0.15), (1, 1, 4000, 0.03, 0.07), (2, 1, 300, 0.05, 0.1), (3, 1, 3500, 0.015, 0.04)]


def translucent_stack(seed=41, W=32, H=16, deg=1):
    """Per 8x8 tile of a 32x16 view, a heap of small splats (0.4-0.8 px) centred inside the tile
    at random depths, with the tile's count and opacity range: pixels stop after tens to
    thousands of splats, or never. Small footprints keep the pixels that take a marginal
    decision (some alpha at the 1/255 cut) few."""
    rng = np.random.default_rng(seed)
    f = 40.0
    parts = []
    for tx, ty, n, o_lo, o_hi in STACKS:
        z = rng.uniform(2.0, 30.0, n)
        px = rng.uniform(tx * 8 + 1.5, tx * 8 + 5.5, n) - (W - 1) / 2
        py = rng.uniform(ty * 8 + 1.5, ty * 8 + 5.5, n) - (H - 1) / 2
        mean = np.stack([px * z / f, py * z / f, z])
        scale = np.exp(rng.uniform(np.log(0.4), np.log(0.8), (3, n))) * z / f
        parts.append((mean, scale, rng.standard_normal((4, n)), rng.uniform(o_lo, o_hi, n)))
    mean, scale, q, opac = (np.concatenate([p[i] for p in parts], axis=-1) for i in range(4))
    n = opac.size
    k = (deg + 1) ** 2 - 1
    g = S.Gaussians(*(a.astype(np.float32) for a in (mean, scale, q, opac, rng.uniform(-1.0, 1.0, (3, n)),
                                                     rng.normal(0, 0.2, (3 * k, n)))), deg)
    cam = S.Camera(W, H, f, f, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3))
    return g, cam


@pytest.fixture(scope="module")
def stack():
    g, cam = translucent_stack()
    ref = oracle.render(g, oracle_cam(cam), tile=8, band=1e-4)
    return g, cam, ref


@pytest.mark.parametrize("tile,bd", [(8, 32), (8, 64), (8, 128), (8, 256), (16, 64), ((16, 8), 128)])
def test_windows_match_oracle(stack, tile, bd):
    g, cam, ref = stack
    run = HipRun(g, cam, tile=tile, blend_depth=bd)
    got = run.image()
    e = assert_images_close(got, ref)
    last = np.asarray(got["last"]).ravel()
    stopped = np.asarray(got["t_final"]).ravel() < 1.05e-4  # T at most 1e-4 / (1 - alpha) after a stop
    in_win = [int(((last >= lo) & (last < hi) & stopped).sum()) for lo, hi in ((0, WIN0), (WIN0, WIN1), (WIN1, 1 << 30))]
    print(f"[windows] tile={tile} bd={bd} errors={e} stopped pixels by window of the last splat: {in_win}", flush=True)
    # the scene exercises the windows: stopped pixels with their last splat in each (the first
    # window only with 8x8 tiles, whose lists are the shortest)
    assert all(in_win[w] > 0 for w in ((0, 1, 2) if tile == 8 else (1, 2))), in_win
    assert (~stopped).sum() > 0  # and pixels that never stop keep their tiles running to the end
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=23)
    gC, gD, gO = gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)
    gg = run.backward(gC, gD, gO)
    gref = oracle.backward(g, oracle_cam(cam), gC.astype(np.float64), gD.astype(np.float64), gO.astype(np.float64))
    assert_grads_close(gg, gref, exclude=marginal_gaussians(g, cam))


def test_windows_repeatable(stack):
    """Two forward calls give the same planes bit for bit (the windows' work lists are filled
    by atomics, but every chunk and pixel is computed the same way)."""
    g, cam, _ = stack
    a = HipRun(g, cam, tile=8, blend_depth=128).image()
    b = HipRun(g, cam, tile=8, blend_depth=128).image()
    for k in ("color", "depth", "alpha", "t_final", "last"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
