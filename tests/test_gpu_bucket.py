"""The per-Gaussian bucketed compositing backward (GS_BWD_BUCKETS, needs an MI355X): gradients
against the float64 oracle element by element (2e-3 relative plus the float32 summation floor,
Gaussians taking marginal decisions left out), and against the pixel-parallel schedule on the
same forward. The two schedules apply the same operations to
every pixel's state in the same order and differ only in the order in which a splat's terms
are summed (lane-serial over the tile's pixels here, a wavefront tree there), so they agree to
float32 summation rounding (per element 1e-4 relative plus 2e-6 of the block's largest). Tiles 8x8 and 16x16, chunk lengths 64,
128 and 256, lists of many chunks, and RGB, depth and opacity upstream gradients; 32x32 tiles
are refused with GS_ERR_UNSUPPORTED.
"""
import numpy as np
import pytest

import oracle
from paper_2507_04004_amd import _native as N
from paper_2507_04004_amd import scenes as S

from gpu_common import HipRun, assert_grads_close, marginal_gaussians, oracle_cam
from test_gpu_parity import CASES, dense_tile

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case,tile,bd", [("small_sh0", 8, 128), ("street_sh3_posed", 8, 64),
                                          ("street_sh3_posed", 16, 256), ("dense", 8, 64), ("dense", 16, 128),
                                          ("street_sh3_posed", (16, 8), 32), ("dense", (8, 32), 64)])
def test_bucketed_backward_matches_oracle_and_chunks(case, tile, bd):
    print(f"[bucket] {case} tile={tile} chunk={bd}", flush=True)
    g, cam = dense_tile() if case == "dense" else CASES[case]()
    run = HipRun(g, cam, tile=tile, blend_depth=bd)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=23)
    gC, gD, gO = gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)
    got = run.backward(gC, gD, gO, schedule=N.GS_BWD_BUCKETS)
    ref = oracle.backward(g, oracle_cam(cam), gC.astype(np.float64), gD.astype(np.float64), gO.astype(np.float64))
    chunks = run.backward(gC, gD, gO, schedule=N.GS_BWD_CHUNKS)
    assert_grads_close(got, ref, exclude=marginal_gaussians(g, cam))
    assert_grads_close(got, chunks, rtol=1e-4, atol=2e-6)


def test_bucketed_backward_overwrite_and_refusals():
    g, cam = CASES["street_sh3_posed"]()
    run = HipRun(g, cam, tile=16, blend_depth=128)
    gC = np.random.default_rng(3).standard_normal((3, cam.h, cam.w)).astype(np.float32)
    acc = run.backward(gC, schedule=N.GS_BWD_BUCKETS)
    from paper_2507_04004_amd import raster as R
    junk = R.ParamGrads.empty(run.gm)
    for t in (junk.mean, junk.scale, junk.rot, junk.opacity, junk.sh_dc, junk.sh_rest, junk.pose):
        t.fill_(3.0)
    ow = run.backward(gC, overwrite=True, grads=junk, schedule=N.GS_BWD_BUCKETS)
    for k in acc:
        np.testing.assert_allclose(ow[k], acc[k], rtol=1e-5, atol=1e-5 * max(np.abs(acc[k]).max(), 1e-30), err_msg=k)
    for tile in (32, (16, 32), (32, 16)):
        big = HipRun(g, cam, tile=tile, blend_depth=128)
        with pytest.raises(N.GSError, match="code 3"):
            big.backward(gC, schedule=N.GS_BWD_BUCKETS)
    with pytest.raises(N.GSError, match="code 1"):
        run.backward(gC, schedule=7)
