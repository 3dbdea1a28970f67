"""FP64 loss of the rasterizer outputs — TEST INFRASTRUCTURE ONLY.

Depth-regularised mapping loss (eq:depth_loss) with the D-SSIM weight set to zero:
    L = mean over pixels and channels |C_hat - C|  +  gamma * mean over LiDAR hits |D_hat/O_hat - D_s|
The depth residual uses the opacity-normalised depth D_hat / O_hat (Sec. "Depth-Regularized Map
Optimization"). The LiDAR term is averaged over the m listed hits (D_s > 0); a hit whose
rendered opacity is zero has no defined normalised depth and adds nothing to the sum.
The L1 subgradient takes sign(0) = 0.
"""
from __future__ import annotations

import numpy as np


def loss_and_grads(color, depth, alpha, target, pix, ds, gamma=1.0, rgb_weight=1.0):
    """Returns (L_rgb, L_depth, dL/dC [3][h][w], dL/dD [h][w], dL/dO [h][w])."""
    color = np.asarray(color, np.float64)
    h, w = depth.shape
    npx = h * w
    r = color - np.asarray(target, np.float64)
    l_rgb = rgb_weight * np.abs(r).sum() / (3 * npx)
    gC = rgb_weight * np.sign(r) / (3 * npx)
    gD = np.zeros(npx)
    gO = np.zeros(npx)
    l_d = 0.0
    m = len(pix)
    D = np.asarray(depth, np.float64).ravel()
    O = np.asarray(alpha, np.float64).ravel()
    for i, p in enumerate(pix):
        if not O[p] > 0:
            continue
        res = D[p] / O[p] - float(ds[i])
        l_d += gamma * abs(res) / m
        s = gamma * np.sign(res) / m
        gD[p] += s / O[p]
        gO[p] += -s * D[p] / (O[p] * O[p])
    return l_rgb, l_d, gC, gD.reshape(h, w), gO.reshape(h, w)
