"""gs_render_bwd_noalloc (needs an MI355X): the backward with the library-owned scratch array
gives the gradients of gs_render_bwd (same kernels; float atomics may sum in another order, so
the element-wise gradient bound applies), on two calls in a row, the second with a smaller
input, different tiles, accumulation instead of overwrite and no depth or opacity terms, so
nothing the first call left in the shared array can leak into the second."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S

from gpu_common import DEV, HipRun, assert_grads_close, oracle_cam

pytestmark = pytest.mark.gpu


def _lidar(g, cam, pix):
    tgt = oracle.render(S.perturb(g, 0.01, seed=1), oracle_cam(cam), band=0.0)
    keep = tgt["alpha"].ravel()[pix] > 0
    pix = pix[keep]
    ds = (tgt["depth"].ravel()[pix] / tgt["alpha"].ravel()[pix]).astype(np.float32)
    return R.LidarHits(torch.from_numpy(pix.astype(np.int32)).to(DEV), torch.from_numpy(ds).to(DEV), weight=0.5)


def test_noalloc_backward_equals_plain_backward_twice():
    # call 1: 100k Gaussians (SH 3) at 640x512, 8x8 tiles, LiDAR hits, depth and opacity terms,
    # overwrite mode
    g, cam, pix = S.config_street_view(1, n=100_000)
    run = HipRun(g, cam, tile=8, blend_depth=128, lidar=_lidar(g, cam, pix))
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=21)
    gC, gD, gO = gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)
    print(f"[noalloc] call 1: {g.n} Gaussians, {cam.w}x{cam.h}, tile 8, overwrite", flush=True)
    ref = run.backward(gC, gD, gO, overwrite=True)
    got = run.backward(gC, gD, gO, overwrite=True, noalloc=True)
    assert_grads_close(got, ref)
    assert np.abs(ref["pose"]).max() > 0 and np.abs(ref["mean"]).max() > 0
    del run
    torch.cuda.synchronize()

    # call 2: 2k Gaussians (SH 0) at 128x96, 16x16 tiles, colour term only, accumulated into
    # seeded values
    g2, cam2, _ = S.config_small(0)
    run2 = HipRun(g2, cam2, tile=16, blend_depth=256)
    gC2 = np.random.default_rng(22).standard_normal((3, cam2.h, cam2.w)).astype(np.float32)
    print(f"[noalloc] call 2: {g2.n} Gaussians, {cam2.w}x{cam2.h}, tile 16, accumulate", flush=True)
    outs = []
    for noalloc in (False, True):
        base = R.ParamGrads.zeros(run2.gm)
        rng = np.random.default_rng(23)
        for k in ("mean", "scale", "rot", "opacity", "sh_dc", "pose"):
            t = getattr(base, k)
            t.copy_(torch.from_numpy(rng.standard_normal(tuple(t.shape)).astype(np.float32)))
        outs.append(run2.backward(gC2, grads=base, noalloc=noalloc))
    assert_grads_close(outs[1], outs[0])
