"""FP64 D-SSIM term of the tracking loss — TEST INFRASTRUCTURE ONLY.

The photometric tracking loss (eq:tracking_loss) is 1/2 mean|C_hat - C| + 1/2 D-SSIM(C_hat, C)
with the D-SSIM term of the original 3DGS loss: 1 - SSIM, the structural similarity averaged
over pixels and channels. SSIM is computed per channel from local statistics under an 11x11
Gaussian window (sigma 1.5, weights summing to one), taken as zero outside the image so the
map keeps the image size, with the constants C1 = 0.01^2 and C2 = 0.03^2 of intensities in
[0, 1]:
    SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
    mu = G * x,  s_x^2 = G * x^2 - mu_x^2,  s_xy = G * (x y) - mu_x mu_y.
The window is applied as one 2-D filter here; the gradient is torch's autograd of this float64
expression.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

WINDOW, SIGMA = 11, 1.5
C1, C2 = 0.01 ** 2, 0.03 ** 2


def window2d() -> np.ndarray:
    r = np.arange(WINDOW) - WINDOW // 2
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * SIGMA ** 2))
    return g / g.sum()


def ssim_map(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """x, y: float64 [c][h][w] -> SSIM [c][h][w]."""
    c = x.shape[0]
    w = torch.tensor(window2d(), dtype=torch.float64)[None, None].expand(c, 1, WINDOW, WINDOW).contiguous()
    conv = lambda z: F.conv2d(z[None], w, padding=WINDOW // 2, groups=c)[0]
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def dssim(x, y, weight: float = 1.0):
    """weight * (1 - mean SSIM) and its gradient w.r.t. x (numpy float64 [c][h][w])."""
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    yt = torch.tensor(np.asarray(y, np.float64))
    loss = weight * (1.0 - ssim_map(xt, yt).mean())
    loss.backward()
    return float(loss.detach()), xt.grad.numpy()
