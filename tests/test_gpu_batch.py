"""Batched form (several views per launch) and hipGraph replay (needs an MI355X).

Batched view k must equal the plain single-view render of view k bitwise (same per-pixel
operation sequence); parameter gradients summed over views must match, element by element, the sum of the
plain per-view gradients (float32 atomics) and of the oracle (2e-3 relative plus the float32
summation floor; Gaussians taking marginal decisions in some view left out); graph replays must
equal eager execution bitwise, replay after replay, with eager work in between.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S
from paper_2507_04004_amd.batch import BatchPlan, ViewSlot

from gpu_common import DEV, HipRun, assert_grads_close, marginal_gaussians, oracle_cam

pytestmark = pytest.mark.gpu


def views_and_map(n=8000, seed=21):
    g = S.street_scene(n, seed, z_range=(-5.0, 60.0), x_half=15.0, n_boxes=8, frac=(0.5, 0.3, 0.2),
                       n_clusters=30, sh_degree=3)
    cams = [S.look_camera((0.5, 0.0, 2.0), 5.0, -2.0, 160, 120, 120.0),
            S.look_camera((-1.0, 0.2, 8.0), -12.0, 3.0, 200, 96, 90.0),
            S.look_camera((0.0, 0.0, 15.0), 0.0, 0.0, 131, 77, 150.0).window(9, 5, 100, 60)]
    return g, cams


def upstream(cam, seed):
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed)
    return gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)


@pytest.mark.parametrize("tile", [8, 16, (16, 8), (8, 32)])
def test_batch_forward_equals_plain(tile):
    g, cams = views_and_map()
    gm = R.GaussianMap.from_numpy(g, DEV)
    plan = BatchPlan(g.n, 3, len(cams), sum(c.w * c.h for c in cams), tile=tile, blend_depth=128, device=DEV)
    slots = [ViewSlot.make(c, DEV) for c in cams]
    plan.run(gm, slots, fwd=True)
    torch.cuda.synchronize()
    assert plan.num_pairs() <= plan.capacity
    for k, cam in enumerate(cams):
        ref = HipRun(g, cam, tile=tile, blend_depth=128).image()
        fr = slots[k].frame
        for key in ("color", "depth", "alpha", "t_final"):
            assert np.array_equal(getattr(fr, key).cpu().numpy(), ref[key]), (k, key)


def test_batch_backward_matches_plain_and_oracle():
    g, cams = views_and_map()
    gm = R.GaussianMap.from_numpy(g, DEV)
    plan = BatchPlan(g.n, 3, len(cams), sum(c.w * c.h for c in cams), device=DEV)
    slots = []
    ups = []
    for k, c in enumerate(cams):
        s = ViewSlot.make(c, DEV, backward=True)
        gC, gD, gO = upstream(c, 100 + k)
        ups.append((gC, gD, gO))
        s.dL_dC = torch.from_numpy(gC).to(DEV)
        s.dL_dD = torch.from_numpy(gD).to(DEV)
        s.dL_dO = torch.from_numpy(gO).to(DEV)
        slots.append(s)
    grads = R.ParamGrads.zeros(gm)
    plan.run(gm, slots, fwd=True, bwd=True, grads=grads)
    torch.cuda.synchronize()
    got = {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in
           ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")}
    ref_sum = {k: 0.0 for k in got}
    marg = np.zeros(g.n, bool)
    for k, c in enumerate(cams):
        ref = oracle.backward(g, oracle_cam(c), *(u.astype(np.float64) for u in ups[k]))
        for key in got:
            ref_sum[key] = ref_sum[key] + ref[key]
        marg |= marginal_gaussians(g, c)
        pose = slots[k].pose_grad.cpu().numpy().astype(np.float64)
        assert_grads_close({"pose": pose}, ref, keys=("pose",))
    assert_grads_close(got, ref_sum, keys=tuple(got), exclude=marg)


def test_batch_fused_l1_and_lidar():
    """Targets inside the batch: the L1 term and LiDAR term match the plain path's gradients."""
    g, cams = views_and_map(seed=23)
    gm = R.GaussianMap.from_numpy(g, DEV)
    gp = S.perturb(g, 0.02, seed=4)
    slots, refs = [], []
    for k, c in enumerate(cams):
        tgt_run = HipRun(gp, c)
        tgt = tgt_run.fr.color.clone()
        O = tgt_run.fr.alpha.flatten().cpu().numpy()
        D = tgt_run.fr.depth.flatten().cpu().numpy()
        pix = np.nonzero(O > 0)[0][::37].astype(np.int32)
        lid = R.LidarHits(torch.from_numpy(pix).to(DEV), torch.from_numpy((D[pix] / O[pix]).astype(np.float32)).to(DEV),
                          weight=0.5)
        s = ViewSlot.make(c, DEV, backward=True, lidar=lid, target=tgt)
        slots.append(s)
        # plain reference: forward, L1 loss, backward with the same LiDAR term
        run = HipRun(g, c, lidar=lid)
        loss, dC = R.loss_l1(run.fr.color, tgt)
        refs.append((run, dC, loss))
    plan = BatchPlan(g.n, 3, len(cams), sum(c.w * c.h for c in cams), device=DEV)
    grads = R.ParamGrads.zeros(gm)
    plan.run(gm, slots, fwd=True, bwd=True, grads=grads)
    torch.cuda.synchronize()
    tot = None
    for k, (run, dC, loss) in enumerate(refs):
        assert abs(slots[k].rgb_loss.item() - loss.item()) <= 1e-5 * max(1.0, loss.item())
        assert abs(slots[k].lidar_loss.item() - run.lidar_loss.item()) <= 1e-5 * max(1.0, run.lidar_loss.item())
        gr = run.backward(dC.cpu().numpy())
        tot = gr if tot is None else {key: tot[key] + gr[key] for key in tot}
        assert_grads_close({"pose": slots[k].pose_grad.cpu().numpy()}, gr, keys=("pose",))
    got = {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in ("mean", "opacity", "sh_dc", "rot")}
    assert_grads_close(got, tot, keys=tuple(got))


def test_graph_replay_equals_eager():
    g, cams = views_and_map(seed=25)
    gm = R.GaussianMap.from_numpy(g, DEV)
    plan = BatchPlan(g.n, 3, len(cams), sum(c.w * c.h for c in cams), device=DEV)
    slots = [ViewSlot.make(c, DEV) for c in cams]
    plan.run(gm, slots, fwd=True, graph=False)
    torch.cuda.synchronize()
    eager = [{k: getattr(s.frame, k).clone() for k in ("color", "depth", "alpha", "t_final", "last")} for s in slots]
    for rep in range(4):
        for s in slots:
            s.frame.color.fill_(-1.0)
            s.frame.last.fill_(-7)
        plan.run(gm, slots, fwd=True, graph=True)
        torch.cuda.synchronize()
        _ = (gm.mean * 2).sum().item()  # unrelated eager work between replays
        for k, s in enumerate(slots):
            for key, ref in eager[k].items():
                assert torch.equal(getattr(s.frame, key), ref), (rep, k, key)


def test_graph_backward_replays():
    g, cams = views_and_map(seed=27)
    gm = R.GaussianMap.from_numpy(g, DEV)
    plan = BatchPlan(g.n, 3, 2, sum(c.w * c.h for c in cams[:2]), device=DEV)
    slots = []
    for k, c in enumerate(cams[:2]):
        s = ViewSlot.make(c, DEV, backward=True)
        s.dL_dC = torch.from_numpy(upstream(c, 200 + k)[0]).to(DEV)
        slots.append(s)
    grads = R.ParamGrads.zeros(gm)
    plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=False)
    torch.cuda.synchronize()
    ref = {k: getattr(grads, k).clone() for k in ("mean", "opacity", "sh_rest")}
    for rep in range(3):
        for t in (grads.mean, grads.scale, grads.rot, grads.opacity, grads.sh_dc, grads.sh_rest):
            t.zero_()
        plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=True)
        torch.cuda.synchronize()
        got = {k: getattr(grads, k).cpu().numpy() for k in ref}
        assert_grads_close(got, {k: r.cpu().numpy() for k, r in ref.items()}, keys=tuple(ref), rtol=1e-4, atol=2e-6)


@pytest.mark.parametrize("tile", [8, 16, (8, 16)])
def test_graph_backward_bucketed_schedule_equals_chunks(tile):
    """The autotuner's second backward schedule inside a captured multi-view batch: every replay
    equals the pixel-parallel schedule's gradients up to float32 summation order."""
    from paper_2507_04004_amd import _native as N
    g, cams = views_and_map(seed=29)
    gm = R.GaussianMap.from_numpy(g, DEV)
    plan = BatchPlan(g.n, 3, 3, sum(c.w * c.h for c in cams), tile=tile, blend_depth=128, device=DEV)
    slots = []
    for k, c in enumerate(cams):
        s = ViewSlot.make(c, DEV, backward=True)
        gC, gD, gO = upstream(c, 300 + k)
        s.dL_dC, s.dL_dD, s.dL_dO = (torch.from_numpy(a).to(DEV) for a in (gC, gD, gO))
        slots.append(s)
    grads = R.ParamGrads.empty(gm)
    plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=False, overwrite=True, schedule=N.GS_BWD_CHUNKS)
    torch.cuda.synchronize()
    keys = ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest", "pose")
    ref = {k: getattr(grads, k).clone() for k in keys if k != "pose"}
    ref_pose = [s.pose_grad.clone() for s in slots]
    for rep in range(3):
        for s in slots:
            s.pose_grad.zero_()
        plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=True, overwrite=True, schedule=N.GS_BWD_BUCKETS)
        torch.cuda.synchronize()
        got = {k: getattr(grads, k).cpu().numpy() for k in ref}
        assert_grads_close(got, {k: r.cpu().numpy() for k, r in ref.items()}, keys=tuple(ref), rtol=1e-4, atol=2e-6)
        for s, r in zip(slots, ref_pose):
            assert_grads_close({"pose": s.pose_grad.cpu().numpy()}, {"pose": r.cpu().numpy()}, keys=("pose",),
                               rtol=1e-4, atol=2e-6)
        torch.randn(100, device=DEV).sum().item()  # eager work between replays
