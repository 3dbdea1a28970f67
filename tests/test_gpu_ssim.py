"""D-SSIM term (needs an MI355X): gs_loss_dssim against the float64 oracle, for ragged tile
edges, images smaller than the window, one channel, and 640x360 and 1280x720 colour images (the
tracking loop's size); the gradient is accumulated onto what dL_dC held.

Tolerances from the arithmetic: every filtered statistic is a float32 sum of 121 weighted terms
(relative error ~1e-6 of the largest term), and the derivative maps subtract such ratios, so
gradients are compared against 2e-5 of the largest oracle gradient of the image; the loss is a
mean of values within [-1, 1]: 1e-5 absolute (times the weight).
"""
import numpy as np
import pytest
import torch

from oracle import ssim as O
from paper_2507_04004_amd import raster as R

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pair(c, h, w, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (c, h, w))
    # a smooth target plus noise, so SSIM is far from both 0 and 1
    yy, xx = np.mgrid[0:h, 0:w]
    base = 0.5 + 0.4 * np.sin(xx / 7.0 + c * 0.3)[None] * np.cos(yy / 5.0)[None]
    y = np.clip(0.6 * base + 0.4 * x + rng.normal(0, 0.05, (c, h, w)), 0, 1)
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("shape", [(3, 50, 77), (1, 7, 5), (3, 16, 32), (2, 33, 129), (3, 360, 640), (3, 720, 1280)])
def test_dssim_matches_oracle(shape):
    c, h, w = shape
    print(f"[dssim] shape={shape}", flush=True)
    x, y = _pair(c, h, w, seed=h * 7 + w)
    weight = 0.5
    pre = np.random.default_rng(1).normal(0, 1e-6, (c, h, w)).astype(np.float32)
    d = torch.from_numpy(pre.copy()).to(DEV)
    loss = R.loss_dssim(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV), weight=weight, dL_dC=d)
    torch.cuda.synchronize()
    ref_loss, ref_g = O.dssim(x.astype(np.float64), y.astype(np.float64), weight=weight)
    got = d.cpu().numpy().astype(np.float64) - pre.astype(np.float64)
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * weight, (float(loss.item()), ref_loss)
    scale = np.abs(ref_g).max()
    err = np.abs(got - ref_g).max()
    print(f"[dssim] loss {float(loss.item()):.6f} (oracle {ref_loss:.6f}); max grad error {err / scale:.2e} of max",
          flush=True)
    assert err <= 2e-5 * scale


def test_dssim_identical_images_and_loss_only():
    x, _ = _pair(3, 40, 48, seed=5)
    xt = torch.from_numpy(x).to(DEV)
    d = torch.zeros_like(xt)
    loss = R.loss_dssim(xt, xt.clone(), weight=1.0, dL_dC=d)
    torch.cuda.synchronize()
    assert abs(float(loss.item())) < 1e-6
    assert float(d.abs().max()) < 1e-9
    # without a gradient buffer only the loss is produced
    x2, y2 = _pair(3, 40, 48, seed=6)
    l2 = R.loss_dssim(torch.from_numpy(x2).to(DEV), torch.from_numpy(y2).to(DEV), weight=2.0)
    torch.cuda.synchronize()
    assert abs(float(l2.item()) - O.dssim(x2.astype(np.float64), y2.astype(np.float64), 2.0)[0]) <= 2e-5


def test_dssim_is_deterministic():
    """The loss is summed in a fixed order and the gradient has no atomics: repeated calls agree
    bit for bit."""
    x, y = _pair(3, 360, 640, seed=9)
    xt, yt = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    outs = []
    for _ in range(3):
        d = torch.zeros_like(xt)
        loss = R.loss_dssim(xt, yt, weight=0.5, dL_dC=d)
        torch.cuda.synchronize()
        outs.append((loss.cpu().numpy().copy(), d.cpu().numpy()))
    for l, d in outs[1:]:
        assert np.array_equal(l, outs[0][0]) and np.array_equal(d, outs[0][1])
