"""Photometric tracking loop (needs an MI355X): gs_track_pose against the float64 oracle.

Both run the loop from the same seeded scene, target and starting pose:
  - first iteration (same pose on both sides): the L1 and D-SSIM terms within 1e-4 absolute
    (images within 1e-4) and the pose gradient within 2e-3 relative (norm) of the oracle's;
  - the whole trajectory: every pose the GPU rendered within 1e-5 of the oracle's pose at the
    same iteration, and the summed loss within 1e-5. Adam's normalised steps would turn a
    sign difference in a near-zero gradient component into a difference of a whole step; on
    these seeded scenes no component comes near zero, the gradients agree to ~2e-6 relative
    and the trajectories stay within float32 rounding (~3e-7), so 1e-5 leaves a 30x margin;
  - the update rule as a property of the GPU's own trace (any size): every next pose equals
    expm(delta^) applied to the previous one (scipy's matrix exponential), with delta the Adam
    step of the reported gradients, to float32 rounding.
Also: convergence from a perturbed pose, graph replays with new starting poses against the
eager loop, recovery when the tile lists overflow the plan, and the loop at the benchmark's
size (2M Gaussians, 1280x720) checked through the same update-rule property, graph/eager
agreement and a falling loss.
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


def _params(**over):
    """The loop's parameters as both sides use them (float32 values): the oracle's defaults
    with `over` applied (product=True: the library's defaults)."""
    if over.pop("product", False):
        over = {**{k: T.DEFAULTS[k] for k in ("lr_rho", "lr_phi")}, **over}
    p = dataclasses.replace(OT.TrackParams(), **over)
    return OT.TrackParams(iters=p.iters, l1_weight=F32(p.l1_weight), ssim_weight=F32(p.ssim_weight),
                          lr_rho=F32(p.lr_rho), lr_phi=F32(p.lr_phi), beta1=F32(p.beta1), beta2=F32(p.beta2),
                          eps=F32(p.eps))


def _kw(q):
    """The same parameters for PoseTracker.track."""
    return dict(iters=q.iters, l1_weight=q.l1_weight, ssim_weight=q.ssim_weight, lr_rho=q.lr_rho, lr_phi=q.lr_phi,
                beta1=q.beta1, beta2=q.beta2, eps=q.eps)


def _twist(xi):
    T = np.zeros((4, 4))
    T[:3, :3] = [[0.0, -xi[5], xi[4]], [xi[5], 0.0, -xi[3]], [-xi[4], xi[3], 0.0]]
    T[:3, 3] = xi[:3]
    return T


def check_update_rule(tr, pose_out, lr_rho, lr_phi, b1, b2, eps):
    """Every next pose of the trace = expm(delta^) times the previous one, delta = the Adam step
    (bias-corrected moments over the iterations) of the reported gradients."""
    import scipy.linalg
    m, v = np.zeros(6), np.zeros(6)
    lr = np.array([lr_rho] * 3 + [lr_phi] * 3)
    T = np.eye(4)
    T[:3, :3], T[:3, 3] = tr[0, :9].reshape(3, 3), tr[0, 9:12]
    worst = 0.0
    for k in range(tr.shape[0]):
        g = tr[k, 12:18]
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        delta = -lr * (m / (1 - b1 ** (k + 1))) / (np.sqrt(v / (1 - b2 ** (k + 1))) + eps)
        T = scipy.linalg.expm(_twist(delta)) @ T
        got = tr[k + 1, :12] if k + 1 < tr.shape[0] else pose_out
        want = np.r_[T[:3, :3].ravel(), T[:3, 3]]
        np.testing.assert_allclose(got, want, rtol=2e-7, atol=2e-7, err_msg=f"step {k + 1}")
        worst = max(worst, float(np.abs(got - want).max()))
    return worst


@pytest.mark.parametrize("graph,deg,tile,bd,product", [(False, 3, 8, 128, False), (True, 3, 8, 128, False),
                                                       (False, 0, 16, 256, False), (True, 1, 8, 64, False),
                                                       (False, 2, 32, 128, False), (True, 3, 8, 128, True)])
def test_loop_matches_oracle(graph, deg, tile, bd, product):
    print(f"[track] oracle parity graph={graph} sh_degree={deg} tile={tile} chunk={bd} "
          f"{'library' if product else 'oracle'} step sizes", flush=True)
    g, cam, start, gm, target = _setup(deg=deg)
    q = _params(product=product)
    trk = T.PoseTracker(gm, cam.w * cam.h, tile=tile, blend_depth=bd, device=DEV)
    res = trk.track(start, target, graph=graph, trace=True, **_kw(q))
    tr = res.trace.double().cpu().numpy()
    pose_out = res.pose.double().cpu().numpy()
    assert res.pairs <= trk.capacity
    tgt = target.double().cpu().numpy()
    # the oracle's own loop from the same float32 starting pose
    R_or, t_or, otr = OT.track(g, oracle.camera_f32(start), tgt, q)
    # the first pose rendered is the starting camera in float32, on both sides
    first = np.r_[np.asarray(start.R_cw, np.float32).ravel(), np.asarray(start.t_cw, np.float32)].astype(np.float64)
    np.testing.assert_array_equal(tr[0, :12], first)
    np.testing.assert_array_equal(np.r_[otr[0]["R"].ravel(), otr[0]["t"]], first)
    err = np.linalg.norm(tr[0, 12:18] - otr[0]["grad"]) / np.linalg.norm(otr[0]["grad"])
    assert err <= 2e-3, (tr[0, 12:18], otr[0]["grad"])
    assert abs(tr[0, 18] - otr[0]["l1"]) <= 1e-4 and abs(tr[0, 19] - otr[0]["ssim"]) <= 1e-4
    # the trajectories
    dpose = max(float(np.abs(tr[k, :12] - np.r_[otr[k]["R"].ravel(), otr[k]["t"]]).max()) for k in range(q.iters))
    dpose = max(dpose, float(np.abs(pose_out - np.r_[R_or.ravel(), t_or]).max()))
    dloss = max(abs(tr[k, 18] + tr[k, 19] - otr[k]["l1"] - otr[k]["ssim"]) for k in range(q.iters))
    print(f"[track] first-iteration gradient error {err:.2e}; largest pose difference {dpose:.2e}, "
          f"loss difference {dloss:.2e} over the trajectory", flush=True)
    assert dpose <= 1e-5 and dloss <= 1e-5
    worst = check_update_rule(tr, pose_out, q.lr_rho, q.lr_phi, q.beta1, q.beta2, q.eps)
    print(f"[track] update rule: largest deviation {worst:.2e}; loss {tr[0, 18] + tr[0, 19]:.4f} -> "
          f"{tr[-1, 18] + tr[-1, 19]:.4f}", flush=True)


def test_loop_in_a_render_window_matches_oracle():
    """A 112x80 window inside the 160x120 image: the render, L1 and D-SSIM run on the window."""
    g, cam = _scene(seed=7)
    win = cam.window(21, 17, 112, 80)
    target = oracle.render(g, oracle.camera_f32(win))["color"].astype(np.float32)
    start = _moved(win, (0.008, 0.01, -0.01, -0.003, 0.002, 0.004))
    gm = R.GaussianMap.from_numpy(g, DEV)
    trk = T.PoseTracker(gm, win.w * win.h, tile=8, blend_depth=128, device=DEV)
    q = _params()
    res = trk.track(start, torch.from_numpy(target).to(DEV), graph=True, trace=True, **_kw(q))
    tr = res.trace.double().cpu().numpy()
    _, _, otr = OT.track(g, oracle.camera_f32(start), target.astype(np.float64), q)
    err = np.linalg.norm(tr[0, 12:18] - otr[0]["grad"]) / np.linalg.norm(otr[0]["grad"])
    dpose = max(float(np.abs(tr[k, :12] - np.r_[otr[k]["R"].ravel(), otr[k]["t"]]).max()) for k in range(q.iters))
    print(f"[track] window: first-iteration gradient error {err:.2e}, largest pose difference {dpose:.2e}",
          flush=True)
    assert err <= 2e-3 and dpose <= 1e-5
    assert abs(tr[0, 18] - otr[0]["l1"]) <= 1e-4 and abs(tr[0, 19] - otr[0]["ssim"]) <= 1e-4


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


def test_loop_at_benchmark_size():
    """2M Gaussians, 1280x720, 8x8 tiles, chunk 128, the benchmark's starts and graph mode."""
    print("[track] benchmark size: generating the 2M-Gaussian map", flush=True)
    g = S.street_map(2_000_000, seed=6)
    cam = S.headline_camera()
    gm = R.GaussianMap.from_numpy(g, DEV)
    del g
    cs = R.camera_struct(cam)
    spl = R.preprocess(gm.struct(), cs, 8, DEV)
    bins = R.bin_sort_fit(spl, gm.n, cs, 8, DEV)
    target = R.render_fwd(spl, gm.n, bins, cs, 128, DEV).color.clone()
    del spl, bins
    rng = np.random.default_rng(8)
    start = R.camera_left_update(cs, np.r_[rng.normal(0, 0.03, 3), rng.normal(0, 0.003, 3)])
    trk = T.PoseTracker(gm, cam.w * cam.h, tile=8, blend_depth=128, device=DEV)
    res = trk.track(start, target, graph=True, trace=True)  # the library's default step sizes
    tr = res.trace.double().cpu().numpy()
    pose = res.pose.double().cpu().numpy()
    assert res.pairs <= trk.capacity
    q = _params(product=True)
    worst = check_update_rule(tr, pose, q.lr_rho, q.lr_phi, q.beta1, q.beta2, q.eps)
    loss = tr[:, 18] + tr[:, 19]
    print(f"[track] benchmark size: pairs {res.pairs}, loss {loss[0]:.4f} -> {loss[-1]:.4f}, update rule "
          f"deviation {worst:.2e}", flush=True)
    assert loss[-1] < 0.5 * loss[0]
    d0 = T.pose_residual(np.r_[np.asarray(cs.R_cw[:]), np.asarray(cs.t_cw[:])], tr[0, :12])
    d1 = T.pose_residual(np.r_[np.asarray(cs.R_cw[:]), np.asarray(cs.t_cw[:])], pose)
    print(f"[track] benchmark size: pose error {np.linalg.norm(d0[:3]):.4f} m / {np.linalg.norm(d0[3:]):.5f} rad "
          f"-> {np.linalg.norm(d1[:3]):.4f} / {np.linalg.norm(d1[3:]):.5f}", flush=True)
    assert np.linalg.norm(d1[:3]) < 0.5 * np.linalg.norm(d0[:3]) and np.linalg.norm(d1[3:]) < 0.5 * np.linalg.norm(d0[3:])
    eager = trk.track(start, target, graph=False).pose.double().cpu().numpy()
    np.testing.assert_allclose(eager, pose, atol=5e-5)
