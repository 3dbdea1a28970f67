"""Photometric tracking loop (needs an MI355X): gs_track_pose against the float64 oracle.

A loop's trajectory is compared one iteration at a time, so that float32 rounding early on
cannot be mistaken for an error later (Adam's normalised steps amplify any difference in a
near-zero gradient component):
  - at the pose the GPU rendered in iteration k (read from the trace), the oracle's loss terms
    and pose gradient: loss terms within 1e-4 absolute (images within 1e-4), the gradient
    within 2e-3 relative (norm) of the oracle's;
  - the chain Adam + Exp replayed in float64 by the oracle from the GPU's own gradients gives
    the GPU's next pose to float32 rounding (2e-7 of the entry's magnitude, at least 2e-7).
Also: convergence from a perturbed pose, graph replays with new starting poses against the
eager loop, and recovery when the tile lists overflow the plan.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from oracle import track as OT
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S
from paper_2507_04004_amd import track as T

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
F32 = lambda x: float(np.float32(x))


def _scene(seed=3, n=3000, W=160, H=120, deg=3):
    cam = S.Camera(W, H, 0.75 * W, 0.75 * W, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3), bg=(0.2, 0.3, 0.4))
    g = S.frustum_scene(n, cam, (2.0, 12.0), sh_degree=deg, seed=seed)
    return g, cam


def _moved(cam, xi):
    R_, t_ = OT.left_update(cam.R_cw, cam.t_cw, np.asarray(xi, np.float64))
    return dataclasses.replace(cam, R_cw=R_, t_cw=t_)


def _at(cam, pose12):
    p = np.asarray(pose12, np.float64)
    return dataclasses.replace(cam, R_cw=p[:9].reshape(3, 3), t_cw=p[9:12])


def _setup(seed=3, xi0=(0.01, -0.008, 0.012, 0.003, -0.004, 0.002), **kw):
    g, cam = _scene(seed, **kw)
    target = oracle.render(g, oracle.camera_f32(cam))["color"].astype(np.float32)
    start = _moved(cam, xi0)
    gm = R.GaussianMap.from_numpy(g, DEV)
    return g, cam, start, gm, torch.from_numpy(target).to(DEV)


def _params():
    p = OT.TrackParams()
    return OT.TrackParams(iters=p.iters, l1_weight=F32(p.l1_weight), ssim_weight=F32(p.ssim_weight),
                          lr_rho=F32(p.lr_rho), lr_phi=F32(p.lr_phi), beta1=F32(p.beta1), beta2=F32(p.beta2),
                          eps=F32(p.eps))


@pytest.mark.parametrize("graph", [False, True])
def test_each_iteration_matches_oracle(graph):
    print(f"[track] per-iteration parity graph={graph}", flush=True)
    g, cam, start, gm, target = _setup()
    trk = T.PoseTracker(gm, cam.w * cam.h, tile=8, blend_depth=128, device=DEV)
    res = trk.track(start, target, graph=graph, trace=True)
    tr = res.trace.double().cpu().numpy()
    pose_out = res.pose.double().cpu().numpy()
    assert res.pairs <= trk.capacity
    q = _params()
    tgt = target.double().cpu().numpy()
    # the first pose rendered is the starting camera in float32
    np.testing.assert_array_equal(tr[0, :12], np.r_[np.asarray(start.R_cw, np.float32).ravel(),
                                                    np.asarray(start.t_cw, np.float32)].astype(np.float64))
    worst = 0.0
    for k in range(q.iters):
        ck = oracle.camera_f32(_at(cam, tr[k, :12]))
        img = oracle.render(g, ck)
        l1, ls, gC = OT.tracking_loss(img["color"], tgt, q.l1_weight, q.ssim_weight)
        ref = oracle.backward(g, ck, gC)["pose"]
        err = np.linalg.norm(tr[k, 12:18] - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        assert err <= 2e-3, (k, tr[k, 12:18], ref)
        assert abs(tr[k, 18] - l1) <= 1e-4 and abs(tr[k, 19] - ls) <= 1e-4, (k, tr[k, 18:], l1, ls)
    # Adam + Exp from the GPU's gradients, in float64, starting at the first rendered pose
    Rk, tk = tr[0, :9].reshape(3, 3), tr[0, 9:12]
    m, v = np.zeros(6), np.zeros(6)
    for k in range(q.iters):
        delta, m, v = OT.adam_step(tr[k, 12:18], m, v, k + 1, q)
        Rk, tk = OT.left_update(Rk, tk, delta)
        want = np.r_[Rk.ravel(), tk]
        got = tr[k + 1, :12] if k + 1 < q.iters else pose_out
        np.testing.assert_allclose(got, want, rtol=2e-7, atol=2e-7, err_msg=f"step {k + 1}")
    print(f"[track] worst gradient error {worst:.2e}; loss {tr[0, 18] + tr[0, 19]:.4f} -> "
          f"{tr[-1, 18] + tr[-1, 19]:.4f}", flush=True)


def test_loop_converges_and_graph_replays_match_eager():
    g, cam, start, gm, target = _setup(seed=4)
    trk = T.PoseTracker(gm, cam.w * cam.h, tile=8, blend_depth=128, device=DEV)
    eager = trk.track(start, target, graph=False, trace=True)
    e_tr = eager.trace.clone()
    e_pose = eager.pose.clone()
    err0 = OT.se3_log(start.R_cw @ cam.R_cw.T, start.t_cw - start.R_cw @ cam.R_cw.T @ cam.t_cw)
    fin = eager.camera(cam)
    err = OT.se3_log(fin.R_cw @ cam.R_cw.T, fin.t_cw - fin.R_cw @ cam.R_cw.T @ cam.t_cw)
    print(f"[track] pose error {np.linalg.norm(err0[:3]):.4f} m / {np.linalg.norm(err0[3:]):.4f} rad -> "
          f"{np.linalg.norm(err[:3]):.4f} / {np.linalg.norm(err[3:]):.4f}", flush=True)
    assert np.linalg.norm(err[:3]) < 0.5 * np.linalg.norm(err0[:3])
    assert np.linalg.norm(err[3:]) < 0.5 * np.linalg.norm(err0[3:])
    # graph: captured on the first call, replayed from other starting poses, with eager work between
    other = _moved(cam, (-0.006, 0.01, -0.008, -0.002, 0.003, -0.003))
    for rep, st in enumerate([start, other, start, other]):
        res = trk.track(st, target, graph=True, trace=True)
        torch.cuda.synchronize()
        ref = trk.track(st, target, graph=False, trace=False).pose.clone() if rep % 2 else e_pose
        got = res.pose.double().cpu().numpy()
        print(f"[track] replay {rep}: max pose difference to eager {np.abs(got - ref.double().cpu().numpy()).max():.2e}",
              flush=True)
        # the backward sums with float atomics: eager and replay differ by rounding, which Adam
        # carries forward; a few ulp per step over 30 steps
        np.testing.assert_allclose(got, ref.double().cpu().numpy(), atol=5e-5)
        if rep == 0:
            np.testing.assert_allclose(res.trace.double().cpu().numpy()[0], e_tr.double().cpu().numpy()[0],
                                       rtol=1e-4, atol=1e-6)
        x = torch.randn(1000, device=DEV).sum()  # unrelated eager work between replays
        assert torch.isfinite(x)


def test_overflowing_plan_grows_and_reruns():
    g, cam, start, gm, target = _setup(seed=5)
    full = T.PoseTracker(gm, cam.w * cam.h, tile=8, blend_depth=128, device=DEV)
    ref = full.track(start, target, graph=False).pose.double().cpu().numpy()
    need = full.pairs_at(R.camera_struct(start))
    small = T.PoseTracker(gm, cam.w * cam.h, tile=8, blend_depth=128, capacity=need // 2, device=DEV)
    print(f"[track] overflow: capacity {need // 2} for ~{need} pairs", flush=True)
    res = small.track(start, target, graph=False)
    assert small.capacity >= res.pairs > need // 2
    np.testing.assert_allclose(res.pose.double().cpu().numpy(), ref, atol=5e-5)
