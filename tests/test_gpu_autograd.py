"""The autograd function without host round trips (needs an MI355X): a pose tangent on the
device is applied on the device (gs_pose_left_update + the projection's device pose) and
gives the image and gradients of the host-side left update; the pair capacity is learned by
the first call and an overflow of a later call is reported by RenderSettings.check."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_04004_amd import raster as R
from paper_2507_04004_amd import scenes as S

from gpu_common import DEV, assert_grads_close, oracle_cam

pytestmark = pytest.mark.gpu

XI = np.array([0.02, -0.01, 0.015, 0.004, -0.006, 0.003], np.float32)


def _render(g, cam, xi_dev, settings):
    gm = R.GaussianMap.from_numpy(g, DEV)
    for t in (gm.mean, gm.opacity, gm.sh_dc):
        t.requires_grad_(True)
    xi = torch.from_numpy(XI).to(xi_dev).requires_grad_(True)
    color, depth, alpha, _ = R.render(settings, gm, xi)
    gC, gD, gO = S.upstream_grads(cam.w * cam.h, seed=31)
    tt = lambda a, *s: torch.from_numpy(a.reshape(*s)).to(DEV)
    loss = (color * tt(gC, 3, cam.h, cam.w)).sum() + (depth * tt(gD, cam.h, cam.w)).sum() + \
        (alpha * tt(gO, cam.h, cam.w)).sum()
    loss.backward()
    torch.cuda.synchronize()
    img = dict(color=color.detach().cpu().numpy(), depth=depth.detach().cpu().numpy(),
               alpha=alpha.detach().cpu().numpy(), t_final=(1 - alpha).detach().cpu().numpy())
    grads = dict(mean=gm.mean.grad.cpu().numpy().astype(np.float64),
                 opacity=gm.opacity.grad.cpu().numpy().astype(np.float64),
                 sh_dc=gm.sh_dc.grad.cpu().numpy().astype(np.float64),
                 pose=xi.grad.cpu().numpy().astype(np.float64))
    return img, grads, (gC, gD, gO)


@pytest.mark.parametrize("tile,bd", [(8, 128), (16, 256)])
def test_device_pose_tangent_equals_host_update(tile, bd):
    g, cam, _ = S.config_street_view(1, n=20_000)
    cam = cam.window(40, 30, 320, 240)
    dev_img, dev_g, up = _render(g, cam, DEV, R.RenderSettings(cam, tile=tile, blend_depth=bd))
    host_img, host_g, _ = _render(g, cam, "cpu", R.RenderSettings(cam, tile=tile, blend_depth=bd))
    for k in ("color", "depth", "alpha"):
        np.testing.assert_allclose(dev_img[k], host_img[k], rtol=0, atol=2e-6, err_msg=k)
    assert_grads_close(dev_g, host_g, keys=("mean", "opacity", "sh_dc", "pose"))


def test_capacity_overflow_is_reported_one_call_late():
    g, cam, _ = S.config_small(0)
    gm = R.GaussianMap.from_numpy(g, DEV)
    settings = R.RenderSettings(cam, capacity=64)  # far below the ~6k pairs of this view
    R.render(settings, gm)
    with pytest.raises(RuntimeError, match="capacity"):
        settings.check()
    assert settings.capacity > 64
    color, _, _, _ = R.render(settings, gm)
    settings.check()  # grown capacity: no overflow
    ref = oracle.render(g, oracle_cam(cam), tile=16, band=1e-4)
    got = dict(color=color.cpu().numpy(), depth=np.zeros((cam.h, cam.w)), alpha=ref["alpha"], t_final=ref["t_final"])
    ok = ref["marginal"] == 0
    assert np.abs(got["color"] - ref["color"])[:, ok].max() <= 1e-4


def test_learned_capacity_then_no_readback():
    g, cam, _ = S.config_small(0)
    gm = R.GaussianMap.from_numpy(g, DEV)
    settings = R.RenderSettings(cam)
    R.render(settings, gm)
    assert settings.capacity is not None and not settings._pending  # first call: counted on the host
    for _ in range(3):
        R.render(settings, gm)
    assert len(settings._pending) >= 1  # later calls: checked asynchronously
    settings.check()
    assert not settings._pending
