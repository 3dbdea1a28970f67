"""The batched pass at the benchmark's size (needs an MI355X).

The 1M-Gaussian street map and its 8 keyframes of uneven intrinsics and resolutions (4.0 Mpix
in total), forward and backward graph-captured in one plan, at the tile shapes the benchmark's
tuner picks between (16x8 and 8x8, chunk 128). Each view's planes must equal its plain
single-view render bit for bit (the same per-pixel operation sequence, compositing windows
included), a graph replay must repeat them, and the batched parameter gradients must equal the
sum of the plain per-view gradients element by element within the bound of the other gradient
tests (the float32 atomics add in another order); so must each view's pose gradient. The plain
path itself is held to the oracle at this size by test_gpu_fullsize.py.
"""
import numpy as np
import pytest
import torch

from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S
from paper_2507_04004_amd.batch import BatchPlan, ViewSlot

from gpu_common import DEV, HipRun, assert_grads_close

pytestmark = pytest.mark.gpu

KEYS = ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")


@pytest.fixture(scope="module")
def world():
    g = S.street_map(1_000_000, seed=2)
    cams = S.keyframe_cameras(8, seed=2)
    return g, R.GaussianMap.from_numpy(g, DEV), cams


def upstream(cam, seed):
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed)
    return gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)


@pytest.mark.parametrize("tile", [(16, 8), 8])
def test_fullsize_batch_equals_plain(world, tile):
    g, gm, cams = world
    total = sum(c.w * c.h for c in cams)
    ups = [upstream(c, 300 + k) for k, c in enumerate(cams)]
    cap = 8 << 20
    while True:
        plan = BatchPlan(g.n, g.sh_degree, len(cams), total, tile=tile, blend_depth=128, capacity=cap, device=DEV)
        slots = []
        for c, (gC, gD, gO) in zip(cams, ups):
            s = ViewSlot.make(c, DEV, backward=True)
            s.dL_dC, s.dL_dD, s.dL_dO = (torch.from_numpy(a).to(DEV) for a in (gC, gD, gO))
            slots.append(s)
        grads = R.ParamGrads.zeros(gm)
        plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=True)
        torch.cuda.synchronize()
        need = plan.num_pairs()
        if need <= plan.capacity:
            break
        plan.close()
        cap = int(need * 1.25)
    print(f"[fullsize batch] tile={tile} pairs={need} capacity={plan.capacity}", flush=True)
    first = [{k: getattr(s.frame, k).clone() for k in ("color", "depth", "alpha", "t_final", "last")} for s in slots]
    got = {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in KEYS}
    poses = [s.pose_grad.cpu().numpy().astype(np.float64) for s in slots]
    # a replay of the captured graph repeats the planes
    for key in KEYS + ("pose",):
        getattr(grads, key).zero_()
    plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=True)
    torch.cuda.synchronize()
    for k, s in enumerate(slots):
        for key, v in first[k].items():
            assert torch.equal(getattr(s.frame, key), v), (k, key)
    plan.close()
    tot = None
    for k, (c, (gC, gD, gO)) in enumerate(zip(cams, ups)):
        run = HipRun(g, c, tile=tile, blend_depth=128)
        ref = run.image()
        for key in ("color", "depth", "alpha", "t_final", "last"):
            assert np.array_equal(first[k][key].cpu().numpy(), ref[key]), (k, key)
        gr = run.backward(gC, gD, gO)
        assert_grads_close({"pose": poses[k]}, gr, keys=("pose",))
        tot = {key: gr[key].astype(np.float64) for key in KEYS} if tot is None else \
            {key: tot[key] + gr[key] for key in KEYS}
        del run
        torch.cuda.empty_cache()
    assert_grads_close(got, tot, keys=KEYS)
