"""Differentiation at full map size (needs an MI355X): a frozen 2M-Gaussian street map, the
pose gradient and per-Gaussian gradients on a centred 256x192 window of a 1280x720 view,
against the float64 oracle element by element (2e-3 relative plus the float32 summation floor),
whose own pose gradient is checked by central finite differences on the frozen branch at the
same size."""
import math

import numpy as np
import pytest

import oracle
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S

from gpu_common import DEV, HipRun, assert_grads_close, marginal_gaussians, oracle_cam

pytestmark = pytest.mark.gpu


def _se3_exp(xi):
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-12:
        Rm, V = np.eye(3) + K, np.eye(3) + 0.5 * K
    else:
        Rm = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K
        V = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K
    return Rm, V @ rho


def _cam_left(cam, xi):
    dR, dt = _se3_exp(xi)
    return S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, dR @ cam.R_cw, dR @ cam.t_cw + dt,
                    cam.x0, cam.y0, cam.w, cam.h, cam.bg)


def _functional(img, gC):
    return float((img["color"] * gC).sum())


@pytest.fixture(scope="module")
def c4():
    print("[c4] generating the 2M-Gaussian map", flush=True)
    g = S.street_map(2_000_000, seed=3)
    cam = oracle_cam(S.headline_camera().window(512, 264, 256, 192))
    delta = np.random.default_rng(3).normal(0.0, 0.01, 6)
    tgt = oracle.render(g, oracle_cam(_cam_left(cam, delta)), tile=8, band=0.0)
    base = oracle.render(g, cam, tile=8)
    n = base["color"].size
    gC = np.sign(base["color"] - tgt["color"]) / n  # L1 of the RGB window
    return g, cam, base, gC


def test_c4_gradients_match_oracle(c4):
    g, cam, base, gC = c4
    print("[c4] GPU backward", flush=True)
    run = HipRun(g, cam, tile=8, blend_depth=128)
    got = run.backward(gC.astype(np.float32))
    print("[c4] oracle backward", flush=True)
    an = oracle.backward(g, cam, gC, None, None, tile=8)
    marg = marginal_gaussians(g, cam, tile=8)
    live = np.nonzero((an["opacity"] != 0) & ~marg)[0]
    assert live.size >= 64
    sel = np.sort(np.random.default_rng(4).choice(live, 64, replace=False))
    print(f"[c4] live Gaussians {live.size}, marginal Gaussians {int(marg.sum())}, "
          f"marginal pixels {int(base['marginal'].sum())}", flush=True)
    assert_grads_close(got, an, keys=("pose",))
    # the 64 seeded Gaussians, against the scale of every live Gaussian's gradient
    for k in ("mean", "opacity"):
        scale = np.abs(an[k][..., live]).max()
        a, b = got[k][..., sel], an[k][..., sel]
        assert np.all(np.abs(a - b) <= 2e-3 * np.abs(b) + 2e-5 * scale), k
    # and every live Gaussian
    assert_grads_close(got, an, keys=("mean", "opacity", "scale", "rot", "sh_dc", "sh_rest"), exclude=marg)


def test_c4_oracle_pose_gradient_against_frozen_fd(c4):
    g, cam, base, gC = c4
    an = oracle.backward(g, cam, gC, None, None, tile=8)
    fz = oracle.Frozen(g, cam, tile=8)
    h = 1e-6
    for i in range(6):
        xi = np.zeros(6)
        xi[i] = h
        fd = (_functional(oracle.replay(g, _cam_left(cam, xi), fz), gC)
              - _functional(oracle.replay(g, _cam_left(cam, -xi), fz), gC)) / (2 * h)
        assert abs(fd - an["pose"][i]) <= 1e-6 * max(abs(an["pose"][i]), 1e-3 * np.abs(an["pose"]).max()) + 1e-9, \
            (i, fd, an["pose"][i])


def test_c4_checkpoint_memory():
    """What the forward leaves for the backward, counted from the buffers themselves: the 8-B
    per-pixel checkpoint, the chunk state (gs_image_state_bytes of the capacity and of this
    view's pairs), the tile lists and the splat records; against per-fragment state."""
    g = S.street_map(1_000_000, seed=2)
    cam = S.headline_camera()
    gm = R.GaussianMap.from_numpy(g, DEV)
    gs, cs = gm.struct(), R.camera_struct(cam)
    spl = R.preprocess(gs, cs, 8, DEV)
    bins = R.bin_sort_fit(spl, gs.n, cs, 8, DEV)
    fr = R.Frame.empty(cam.h, cam.w, DEV, count=True)
    R.render_fwd(spl, gs.n, bins, cs, 128, DEV, out=fr)
    fragments = int(fr.n_contrib.long().sum().item())
    kept = R.kept_bytes(spl, bins, fr, cs, 128)
    lib = R.N.lib()
    T = R.tiles_of(cs, 8)
    print(f"[c4] kept MB { {k: round(v / 1e6, 2) for k, v in kept.items()} } vs per-fragment state >= "
          f"{8 * fragments / 1e6:.1f} MB ({fragments} contributing fragments)", flush=True)
    assert kept["checkpoint"] == R.checkpoint_bytes(cam) == cam.w * cam.h * 8
    assert kept["chunk_state_allocated"] == lib.gs_image_state_bytes(bins.capacity, T, 8, 8, 128)
    assert kept["chunk_state_needed"] == lib.gs_image_state_bytes(bins.pairs(), T, 8, 8, 128)
    assert kept["chunk_state_needed"] <= kept["chunk_state_allocated"]
    assert kept["splat_records"] == gs.n * (64 + 8)
    assert kept["total_allocated"] < 8 * fragments
