"""Map initialization / expansion (needs an MI355X): gs_expand_select + gs_expand_write against
the oracle. The selection (count, which points, their order) is bit-exact: both sides take it in
float32 with the same operation order. Copied planes, means, rotations, opacities and zeroed SH
are exact; scale = z / fx and the DC coefficient are within float32 rounding of the oracle's
float64 values (the depth is a float32 sum of three products: a few ulp, 1e-6 relative).
Masks come from the oracle's rendered opacity or from a synthetic recipe, never from the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import expand as OE
from paper_2507_04004_amd import expand as X
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _scene(seed=5, n=20000, W=200, H=150):
    g = S.street_scene(n, seed, z_range=(1.0, 40.0), x_half=15.0, n_boxes=6, frac=(0.6, 0.3, 0.1), n_clusters=20,
                       sh_degree=3)
    cam = S.look_camera((0.5, -0.3, -2.0), 8.0, -3.0, W, H, 0.7 * W)
    return g, cam


def _points(n, seed, cam):
    """Points around the view: most in front, some behind, outside, NaN and on the near plane."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-2.0, 40.0, n)
    x = rng.uniform(-1.2, 1.2, n) * np.abs(z) * cam.width / (2 * cam.fx)
    y = rng.uniform(-1.2, 1.2, n) * np.abs(z) * cam.height / (2 * cam.fy)
    pc = np.stack([x, y, z])
    R_wc = np.asarray(cam.R_cw).T
    xyz = (R_wc @ (pc - np.asarray(cam.t_cw)[:, None])).astype(np.float32)
    xyz[:, rng.choice(n, max(1, n // 500), replace=False)] = np.nan
    rgb = rng.uniform(0, 1, (3, n)).astype(np.float32)
    return xyz, rgb


def _compare(new, added, g_old, xyz, rgb, cam, O, tau=0.99):
    sel = OE.select(xyz, cam, O, tau)
    ref = OE.new_gaussians(xyz, rgb, cam, sel, new.sh_degree)
    m = int(sel.sum())
    assert added == m, (added, m)
    n_old = 0 if g_old is None else g_old.n
    got = {k: getattr(new, k).cpu().numpy().reshape(-1, n_old + m) for k in
           ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")}
    if g_old is not None:
        for k in got:
            old = getattr(g_old, k).reshape(-1, n_old)
            np.testing.assert_array_equal(got[k][:, :n_old], old, err_msg=k)
    tail = {k: v[:, n_old:].astype(np.float64) for k, v in got.items()}
    np.testing.assert_array_equal(tail["mean"], ref["mean"])
    np.testing.assert_array_equal(tail["rot"], ref["rot"])
    np.testing.assert_array_equal(tail["opacity"][0], np.full(m, float(np.float32(0.1))))
    assert not tail["sh_rest"].any()
    np.testing.assert_allclose(tail["scale"], ref["scale"], rtol=1e-6)
    np.testing.assert_allclose(tail["sh_dc"], ref["sh_dc"], rtol=1e-6, atol=1e-6)
    return m


@pytest.mark.parametrize("n_pts", [1, 1023, 1025, 200_003])
def test_expansion_matches_oracle(n_pts):
    print(f"[expand] points={n_pts}", flush=True)
    g, cam = _scene()
    O = oracle.render(g, oracle.camera_f32(cam))["alpha"].astype(np.float32)
    assert 0.05 < (O < 0.99).mean() < 0.95
    xyz, rgb = _points(n_pts, n_pts, cam)
    gm = R.GaussianMap.from_numpy(g, DEV)
    new, added = X.expand_map(gm, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), cam,
                              torch.from_numpy(O).to(DEV), 0.99, device=DEV)
    torch.cuda.synchronize()
    m = _compare(new, added, g, xyz, rgb, cam, O)
    print(f"[expand] added {m} of {n_pts}", flush=True)


def test_initialization_window_and_synthetic_mask():
    g, cam = _scene(seed=6)
    xyz, rgb = _points(50_000, 3, cam)
    # initialization: no map, no mask
    new, added = X.expand_map(None, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), cam, None,
                              device=DEV)
    torch.cuda.synchronize()
    _compare(new, added, None, xyz, rgb, cam, None)
    # a render window with a striped synthetic mask, values straddling tau
    win = cam.window(23, 17, 131, 97)
    rng = np.random.default_rng(4)
    O = rng.choice(np.array([0.0, 0.5, np.nextafter(np.float32(0.99), np.float32(0)), 0.99, 1.0], np.float32),
                   (97, 131))
    O[::7] = 1.0
    gm = R.GaussianMap.from_numpy(g, DEV)
    new, added = X.expand_map(gm, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), win,
                              torch.from_numpy(O).to(DEV), 0.99, device=DEV)
    torch.cuda.synchronize()
    _compare(new, added, g, xyz, rgb, win, O)


def test_no_points_and_new_gaussians_cover_the_holes():
    g, cam = _scene(seed=7)
    gm = R.GaussianMap.from_numpy(g, DEV)
    e = torch.empty(3, 0, device=DEV)
    new, added = X.expand_map(gm, e, e, cam, torch.zeros(cam.h, cam.w, device=DEV), device=DEV)
    torch.cuda.synchronize()
    assert added == 0
    for k in ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest"):
        assert torch.equal(getattr(new, k), getattr(gm, k)), k
    # rendering the grown map: opacity rises where points filled the mask, and drops nowhere
    # beyond the early stop's slack (a Gaussian added in front can end a pixel one Gaussian
    # earlier, with T < 1e-4 / (1 - alpha) <= 0.01 where the old T was below that)
    O = oracle.render(g, oracle.camera_f32(cam))["alpha"].astype(np.float32)
    xyz, rgb = _points(30_000, 9, cam)
    new, added = X.expand_map(gm, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), cam,
                              torch.from_numpy(O).to(DEV), 0.99, device=DEV)
    cs = R.camera_struct(cam)

    def alpha(m):
        spl = R.preprocess(m.struct(), cs, 16, DEV)
        bins = R.bin_sort_fit(spl, m.n, cs, 16, DEV)
        return R.render_fwd(spl, m.n, bins, cs, 256, DEV).alpha.cpu().numpy()

    a0, a1 = alpha(gm), alpha(new)
    assert added > 1000
    assert (a1 >= a0 - 0.0101).all()
    assert (a1 - a0 > 0.05).mean() > 0.05


@pytest.mark.parametrize("tau", [0.5, 0.9999])
def test_expansion_at_other_thresholds(tau):
    g, cam = _scene(seed=8)
    O = oracle.render(g, oracle.camera_f32(cam))["alpha"].astype(np.float32)
    xyz, rgb = _points(50_000, 13, cam)
    gm = R.GaussianMap.from_numpy(g, DEV)
    new, added = X.expand_map(gm, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), cam,
                              torch.from_numpy(O).to(DEV), tau, device=DEV)
    torch.cuda.synchronize()
    m = _compare(new, added, g, xyz, rgb, cam, O, tau)
    print(f"[expand] tau={tau}: added {m} of 50000", flush=True)


def test_expansion_of_a_degree_zero_map():
    """No higher SH planes: only the 14 planes of degree 0 are copied and filled."""
    cam = S.look_camera((0.0, 0.0, 0.0), 0.0, 0.0, 160, 120, 120.0)
    g = S.frustum_scene(5000, cam, (2.0, 20.0), sh_degree=0, seed=11)
    O = oracle.render(g, oracle.camera_f32(cam))["alpha"].astype(np.float32)
    xyz, rgb = _points(20_000, 12, cam)
    gm = R.GaussianMap.from_numpy(g, DEV)
    new, added = X.expand_map(gm, torch.from_numpy(xyz).to(DEV), torch.from_numpy(rgb).to(DEV), cam,
                              torch.from_numpy(O).to(DEV), 0.99, device=DEV)
    torch.cuda.synchronize()
    assert new.sh_degree == 0 and new.sh_rest.shape[0] == 0
    _compare(new, added, g, xyz, rgb, cam, O)
