"""GPU-vs-oracle parity of every stage, through the C ABI (needs an MI355X).

Bars: tile/pair lists, sort order, tile counts, rectangles and depth keys bit-exact against
the float32 binning oracle; images within 1e-4 max-abs (depth 1e-4 relative beyond 1 m) on
pixels the FP64 oracle does not flag as marginal; gradients element by element within 2e-3
relative (plus a float32 summation floor of 2e-5 of the block's largest element) of the FP64
analytic oracle, itself pinned to finite differences; Gaussians the oracle flags as taking a
marginal decision at some pixel are left out of the per-Gaussian blocks (not of the pose).
The small scenes run at 16x16 tiles / chunk 256 and at the benchmark's 8x8 / 128.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.loss import loss_and_grads
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S

from gpu_common import (DEV, HipRun, assert_grads_close, assert_images_close, compare_images, grad_errors,
                        marginal_gaussians, oracle_cam)

pytestmark = pytest.mark.gpu


def small_street(n=6000, seed=5, W=200, H=150, deg=3):
    g = S.street_scene(n, seed, z_range=(1.0, 40.0), x_half=15.0, n_boxes=6, frac=(0.6, 0.3, 0.1), n_clusters=20,
                       sh_degree=deg)
    cam = S.Camera(W, H, 0.7 * W, 0.7 * W, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3))
    return g, cam


def posed(cam, seed, scale=0.05, bg=(0.0, 0.0, 0.0)):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    Rm = Rotation.from_rotvec(rng.normal(0, scale, 3)).as_matrix()
    return S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, Rm, rng.normal(0, scale, 3), cam.x0,
                    cam.y0, cam.w, cam.h, bg)


def dense_tile(n=4000, seed=31, W=64, H=64, deg=2):
    """Thousands of splats over a few tiles: long lists, many chunks, early stops in late chunks."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(2.0, 30.0, n)
    f = 60.0
    u = rng.normal(0.0, 10.0, n)
    v = rng.normal(0.0, 10.0, n)
    mean = np.stack([u * z / f, v * z / f, z])
    scale = np.exp(rng.uniform(-3.5, -1.5, (3, n))) * z / 8.0
    q = rng.standard_normal((4, n))
    opac = rng.uniform(0.05, 0.95, n)
    dc = rng.uniform(-1.0, 1.0, (3, n))
    k = (deg + 1) ** 2 - 1
    g = S.Gaussians(*(a.astype(np.float32) for a in (mean, scale, q, opac, dc, rng.normal(0, 0.2, (3 * k, n)))), deg)
    cam = S.Camera(W, H, f, f, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3))
    return g, cam


CASES = {
    "small_sh0": lambda: S.config_small(0)[:2],
    "dense_tile": lambda: dense_tile(),
    "street_sh3_posed": lambda: (small_street()[0], posed(small_street()[1], 3, bg=(0.1, 0.2, 0.3))),
    "street_sh1_window": lambda: (small_street(deg=1, seed=8)[0], small_street()[1].window(13, 7, 150, 101)),
    "street_sh2_ragged": lambda: small_street(deg=2, seed=9, W=203, H=117),
}


# ---- stage a1 + a2: records and tile lists ----------------------------------------------------
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("tile", [8, 16, 32, (8, 16), (32, 8), (16, 32)])
def test_bins_bit_exact(case, tile):
    g, cam = CASES[case]()
    print(f"[bins] case={case} tile={tile} n={g.n}", flush=True)
    run = HipRun(g, cam, tile=tile)
    got = run.bins_np()
    ref = oracle.bin32(g, cam, tile=tile)
    np.testing.assert_array_equal(got["n_tiles"], ref["n_tiles"])
    vis = ref["n_tiles"] > 0
    np.testing.assert_array_equal(got["rect"][vis], ref["rect"][vis])
    np.testing.assert_array_equal(got["dkey"], ref["dkey"])
    assert got["num_pairs"] == ref["num_pairs"]
    np.testing.assert_array_equal(got["vals"], ref["vals"])
    np.testing.assert_array_equal(got["tile_range"], ref["tile_range"])


@pytest.mark.parametrize("case", ["small_sh0", "street_sh3_posed"])
def test_projection_records(case):
    g, cam = CASES[case]()
    run = HipRun(g, cam)
    ref = oracle.project(g, oracle_cam(cam))
    vis = run.bins_np()["n_tiles"] > 0
    assert np.all(ref["valid"][vis] == 1)
    ra = run.spl.rec_a.cpu().numpy().astype(np.float64)
    rb = run.spl.rec_b.cpu().numpy().astype(np.float64)
    rgb = run.spl.rgb.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(ra[vis, 0], ref["uv"][0, vis], rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(ra[vis, 1], ref["uv"][1, vis], rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(ra[vis, 3], ref["depth"][vis], rtol=1e-6)
    for j in range(3):
        scale = np.abs(ref["conic"][:, vis]).max(axis=0)
        assert np.all(np.abs(rb[vis, j] - ref["conic"][j, vis]) <= 1e-4 * scale + 1e-7), j
        np.testing.assert_allclose(rgb[vis, j], ref["rgb"][j, vis], atol=2e-5)
    np.testing.assert_allclose(rb[vis, 3], ref["kappa2"][vis], rtol=1e-6)


# ---- stage a3: compositing ------------------------------------------------------------------
LAUNCH = [(16, 256), (8, 128), ((8, 16), 32), ((32, 16), 64)]


@pytest.mark.parametrize("tile,bd", LAUNCH)
@pytest.mark.parametrize("case", list(CASES))
def test_render_matches_oracle(case, tile, bd):
    g, cam = CASES[case]()
    print(f"[render] case={case} tile={tile} chunk={bd}", flush=True)
    run = HipRun(g, cam, tile=tile, blend_depth=bd)
    got = run.image()
    ref = oracle.render(g, oracle_cam(cam), tile=16, band=1e-4)
    e = assert_images_close(got, ref)
    print(f"[render] case={case} errors={e}", flush=True)
    # the checkpoint: the record at `last` is the oracle's last contributor
    ok = (ref["marginal"] == 0) & (ref["last_id"] >= 0)
    vals = run.bins_np()["vals"]
    tr = run.bins_np()["tile_range"]
    tw, th = R.tile_wh(tile)
    tiles_x = (cam.w + tw - 1) // tw
    ys, xs = np.nonzero(ok)
    t = (ys // th) * tiles_x + xs // tw
    idx = tr[2 * t] + got["last"][ys, xs]
    np.testing.assert_array_equal(vals[idx], ref["last_id"][ys, xs])
    assert np.all(got["last"][ref["last_id"] < 0] == -1)


def _max_list(run):
    tr = run.bins_np()["tile_range"].reshape(-1, 2).astype(np.int64)
    return int((tr[:, 1] - tr[:, 0]).max(initial=0))


@pytest.mark.parametrize("case", ["street_sh3_posed", "dense_tile"])
def test_tile_size_and_blend_depth_invariance(case):
    """Images do not depend on the tile size or chunk length: bitwise when every list fits in
    one chunk (same per-pixel operation sequence), else up to float32 reassociation."""
    g, cam = CASES[case]()
    base_run = HipRun(g, cam, tile=16, blend_depth=256)
    base = base_run.image()
    base_single = _max_list(base_run) <= 256
    for tile, bd in [(8, 32), (8, 64), (8, 256), (16, 64), (16, 128), (32, 128), (32, 256), ((8, 16), 64),
                     ((16, 8), 32), ((8, 32), 128), ((32, 8), 256), ((16, 32), 64), ((32, 16), 32)]:
        run = HipRun(g, cam, tile=tile, blend_depth=bd)
        got = run.image()
        bitwise = base_single and _max_list(run) <= bd
        for k in ("color", "depth", "alpha", "t_final"):
            if bitwise:
                assert np.array_equal(got[k], base[k]), (tile, bd, k)
            else:
                scale = np.maximum(1.0, np.abs(base[k])) if k == "depth" else 1.0
                assert np.max(np.abs(got[k] - base[k]) / scale) <= 2e-5, (tile, bd, k)


@pytest.mark.parametrize("bd", [32, 64, 128, 256])
def test_multichunk_tiles_match_oracle(bd):
    """Long tile lists split into many chunks, with pixels stopping in late chunks."""
    g, cam = dense_tile()
    run = HipRun(g, cam, tile=16, blend_depth=bd)
    assert _max_list(run) > 4 * bd
    got = run.image()
    ref = oracle.render(g, oracle_cam(cam), tile=16, band=1e-4)
    assert (ref["t_final"] < 2e-4).mean() > 0.05  # plenty of pixels reach the early stop
    e = assert_images_close(got, ref)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=17)
    gC, gD, gO = gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)
    gg = run.backward(gC, gD, gO)
    gref = oracle.backward(g, oracle_cam(cam), gC.astype(np.float64), gD.astype(np.float64), gO.astype(np.float64))
    print(f"[multichunk] bd={bd} image errors={e}", flush=True)
    assert_grads_close(gg, gref, exclude=marginal_gaussians(g, cam))


def test_forward_deterministic():
    g, cam = CASES["street_sh3_posed"]()
    a = HipRun(g, cam).image()
    b = HipRun(g, cam).image()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


# ---- stages a4 + a5: backward ----------------------------------------------------------------
@pytest.mark.parametrize("tile,bd", LAUNCH)
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("which", ["all", "rgb_only", "depth_only"])
def test_backward_matches_oracle(case, which, tile, bd):
    g, cam = CASES[case]()
    print(f"[backward] case={case} which={which} tile={tile} chunk={bd}", flush=True)
    run = HipRun(g, cam, tile=tile, blend_depth=bd)
    npx = cam.w * cam.h
    gC, gD, gO = S.upstream_grads(npx, seed=11)
    gC = gC.reshape(3, cam.h, cam.w) * (which != "depth_only")
    gD = gD.reshape(cam.h, cam.w) if which != "rgb_only" else None
    gO = gO.reshape(cam.h, cam.w) if which == "all" else None
    got = run.backward(gC, gD, gO)
    ref = oracle.backward(g, oracle_cam(cam), gC.astype(np.float64), None if gD is None else gD.astype(np.float64),
                          None if gO is None else gO.astype(np.float64))
    assert_grads_close(got, ref, exclude=marginal_gaussians(g, cam))


@pytest.mark.parametrize("case", ["street_sh3_posed", "small_sh0"])
def test_backward_overwrite_and_accumulate(case):
    """overwrite=1 writes every element (NaN garbage beforehand does not leak through) and
    matches accumulation into zeros; overwrite=0 adds to what the outputs hold. (Runs are
    compared to float32 summation-order level: the compositing backward adds its per-splat
    sums with float atomics.)"""
    g, cam = CASES[case]()
    run = HipRun(g, cam)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=13)
    gC, gD, gO = gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w)
    acc = run.backward(gC, gD, gO)
    junk = R.ParamGrads.empty(run.gm)
    for t in (junk.mean, junk.scale, junk.rot, junk.opacity, junk.sh_dc, junk.sh_rest, junk.pose):
        t.fill_(float("nan"))
    ow = run.backward(gC, gD, gO, overwrite=True, grads=junk)
    for k in acc:
        assert np.isfinite(ow[k]).all(), k
        assert np.array_equal(ow[k] == 0, acc[k] == 0) or k == "pose", k  # untouched Gaussians read 0
        # atomics add per-tile sums that cancel: reordering them moves an element by up to a
        # few 1e-6 of the largest one
        np.testing.assert_allclose(ow[k], acc[k], rtol=1e-4, atol=1e-5 * max(1.0, np.abs(acc[k]).max(initial=0)),
                                   err_msg=k)
    base = R.ParamGrads.zeros(run.gm)
    rng = np.random.default_rng(3)
    pre = {}
    for k in acc:
        t = getattr(base, k)
        v = rng.standard_normal(tuple(t.shape)).astype(np.float32)
        t.copy_(torch.from_numpy(v))
        pre[k] = v.astype(np.float64)
    added = run.backward(gC, gD, gO, grads=base)
    for k in acc:
        untouched = acc[k] == 0
        assert np.array_equal(added[k][untouched], pre[k][untouched]), k
        np.testing.assert_allclose(added[k] - pre[k], acc[k], rtol=1e-4,
                                   atol=1e-5 * max(1.0, np.abs(acc[k]).max(initial=0)), err_msg=k)


def test_lidar_depth_term():
    g, cam, pix = S.config_small(0)
    gp = S.perturb(g, 0.01, seed=1)
    tgt = oracle.render(gp, oracle_cam(cam), band=0.0)
    ds_full = (tgt["depth"] / np.where(tgt["alpha"] > 0, tgt["alpha"], 1)).ravel()
    keep = tgt["alpha"].ravel()[pix] > 0
    pix = pix[keep]
    ds = ds_full[pix].astype(np.float32)
    lid = R.LidarHits(torch.from_numpy(pix.astype(np.int32)).to(DEV), torch.from_numpy(ds).to(DEV), weight=0.7)
    run = HipRun(g, cam, lidar=lid)
    ref_img = oracle.render(g, oracle_cam(cam), band=1e-4)
    _, l_ref, _, gD_ref, gO_ref = loss_and_grads(ref_img["color"], ref_img["depth"], ref_img["alpha"],
                                                 ref_img["color"], pix, ds, gamma=0.7)
    l_gpu = float(run.lidar_loss.item())
    assert abs(l_gpu - l_ref) <= 1e-4 * max(1.0, abs(l_ref)), (l_gpu, l_ref)
    gC = np.zeros((3, cam.h, cam.w), np.float32)
    got = run.backward(gC, None, None)
    ref = oracle.backward(g, oracle_cam(cam), gC.astype(np.float64), gD_ref, gO_ref)
    print(f"[lidar] loss gpu={l_gpu:.6f} ref={l_ref:.6f}", flush=True)
    assert_grads_close(got, ref, exclude=marginal_gaussians(g, cam))


def test_autograd_function_and_checkpoint():
    g, cam = CASES["street_sh3_posed"]()
    gm = R.GaussianMap.from_numpy(g, DEV)
    for t in (gm.mean, gm.scale, gm.rot, gm.opacity, gm.sh_dc, gm.sh_rest):
        t.requires_grad_(True)
    xi = torch.zeros(6, device=DEV, requires_grad=True)
    color, depth, alpha, _ = R.render(R.RenderSettings(cam), gm, xi)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=12)
    tt = lambda a, *s: torch.from_numpy(a.reshape(*s)).to(DEV)
    loss = (color * tt(gC, 3, cam.h, cam.w)).sum() + (depth * tt(gD, cam.h, cam.w)).sum() + \
           (alpha * tt(gO, cam.h, cam.w)).sum()
    loss.backward()
    ref = oracle.backward(g, oracle_cam(cam), gC.reshape(3, cam.h, cam.w).astype(np.float64),
                          gD.reshape(cam.h, cam.w).astype(np.float64), gO.reshape(cam.h, cam.w).astype(np.float64))
    got = dict(mean=gm.mean.grad, scale=gm.scale.grad, rot=gm.rot.grad, opacity=gm.opacity.grad,
               sh_dc=gm.sh_dc.grad, sh_rest=gm.sh_rest.grad, pose=xi.grad)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in got.items()}
    assert_grads_close(got, ref, exclude=marginal_gaussians(g, cam))
    assert R.checkpoint_bytes(cam) == cam.w * cam.h * 8


def test_pose_translation_identity_gpu():
    """d L / d rho = R sum_k d L / d mu_k on the GPU's own gradients."""
    g, cam = CASES["street_sh3_posed"]()
    run = HipRun(g, cam)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=13)
    got = run.backward(gC.reshape(3, cam.h, cam.w), gD.reshape(cam.h, cam.w), gO.reshape(cam.h, cam.w))
    lhs = got["pose"][:3]
    rhs = np.asarray(cam.R_cw) @ got["mean"].sum(1)
    assert np.linalg.norm(lhs - rhs) <= 1e-3 * np.linalg.norm(rhs)


# ---- edge cases ------------------------------------------------------------------------------
def test_edge_cases():
    g, cam = S.config_small(0)[:2]
    # empty map
    empty = g.subset(np.arange(0))
    run = HipRun(empty, cam)
    img = run.image()
    assert np.all(img["alpha"] == 0) and np.all(img["t_final"] == 1) and np.all(img["last"] == -1)
    gr = run.backward(np.ones((3, cam.h, cam.w), np.float32))
    assert np.all(gr["pose"] == 0)
    # overwrite mode writes the (zero) pose gradient over whatever the buffer held
    junk = R.ParamGrads.empty(run.gm)
    junk.pose.fill_(7.0)
    gr = run.backward(np.ones((3, cam.h, cam.w), np.float32), overwrite=True, grads=junk)
    assert np.all(gr["pose"] == 0)
    # every Gaussian behind the camera
    behind = g.subset(np.arange(g.n))
    behind.mean[2] *= -1
    run_b = HipRun(behind, cam)
    img = run_b.image()
    assert np.all(img["alpha"] == 0) and np.all(img["last"] == -1)
    assert run_b.bins_np()["num_pairs"] == 0  # no record survives the first depth pass
    gr = run_b.backward(np.ones((3, cam.h, cam.w), np.float32), overwrite=True)
    for k in ("mean", "opacity", "sh_dc", "pose"):
        assert np.all(np.asarray(gr[k]) == 0), k
    # degenerate Gaussians are dropped, the rest render as without them
    bad = g.subset(np.arange(50))
    bad.rot[:, 0] = 0.0
    bad.scale[:, 1] = 0.0
    bad.mean[0, 2] = np.nan
    bad.opacity[3] = 1e-4
    ok_idx = np.setdiff1d(np.arange(50), [0, 1, 2, 3])
    a = HipRun(bad, cam).image()
    b = HipRun(g.subset(ok_idx), cam).image()
    for k in ("color", "depth", "alpha", "t_final"):
        assert np.array_equal(a[k], b[k]), k
    # a one-pixel window
    one = cam.window(40, 30, 1, 1)
    img = HipRun(g, one).image()
    ref = oracle.render(g, oracle_cam(one), band=1e-4)
    assert_images_close(img, ref)


def test_capacity_overflow_is_reported_and_recovers():
    g, cam = CASES["street_sh3_posed"]()
    gm = R.GaussianMap.from_numpy(g, DEV)
    cs = R.camera_struct(cam)
    gs = gm.struct()
    spl = R.preprocess(gs, cs, 16, DEV)
    small = R.bin_sort(spl, gs.n, cs, R.alloc_bins(gs.n, cs, 16, 100, DEV))
    need = small.pairs()
    assert need > 100
    fr = R.render_fwd(spl, gs.n, small, cs, 256, DEV)  # clamped lists: must not fault
    torch.cuda.synchronize()
    assert torch.isfinite(fr.color).all()
    full = R.bin_sort(spl, gs.n, cs, R.alloc_bins(gs.n, cs, 16, need, DEV))
    assert full.pairs() == need
    ref = oracle.bin32(g, cam, tile=16)
    np.testing.assert_array_equal(full.vals[:need].cpu().numpy().view(np.uint32), ref["vals"])
