"""FP64 photometric tracking loop — TEST INFRASTRUCTURE ONLY.

Camera factor option 2 (Sec. "Camera Factor (Option 2)", eq:tracking_loss and
eq:map_optimize_pose): with the Gaussian map frozen, the camera pose is refined by N_t Adam
iterations on
    L = w_1 mean |C_hat - C| + w_s D-SSIM(C_hat, C),   w_1 = w_s = 1/2,
and the refined pose T~ gives the factor residual r_C2 = Log(T(t) T~^-1) on camera-to-world
poses.

Readings (the paper states the loss, the optimiser and N_t = 30, nothing more):
  - the pose is optimised on the manifold: each iteration takes the gradient dL/dxi of the
    left perturbation T_cw <- Exp(xi) T_cw at xi = 0 (translation rho first, then rotation
    phi), turns it into an Adam step delta (moments and bias correction kept over the
    iterations, the parameter itself reset to zero after every update), and applies
    T_cw <- Exp(delta) T_cw;
  - the Adam step sizes for the translation and rotation parts are separate parameters;
  - the L1 term is the mean over channels and pixels, its derivative sign(C_hat - C) / n
    with sign(0) = 0.
Exp and Log are the closed-form SE(3) maps (Rodrigues' formula and the left Jacobian V).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import backward as _backward
from . import render as _render
from . import ssim as _ssim


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """xi = (rho, phi) -> (R, t) of Exp(xi): R = exp(phi^), t = V rho."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    th = float(np.linalg.norm(phi))
    P = hat(phi)
    if th < 1e-5:
        # series: A = 1 - th^2/6, B = 1/2 - th^2/24, C = 1/6 - th^2/120
        A, B, Cc = 1.0 - th * th / 6.0, 0.5 - th * th / 24.0, 1.0 / 6.0 - th * th / 120.0
    else:
        A, B, Cc = np.sin(th) / th, (1.0 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
    R = np.eye(3) + A * P + B * (P @ P)
    V = np.eye(3) + B * P + Cc * (P @ P)
    return R, V @ rho


def se3_log(R, t):
    """Inverse of se3_exp for rotation angles below pi: (R, t) -> xi = (rho, phi)."""
    R = np.asarray(R, np.float64)
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = float(np.arccos(c))
    W = R - R.T
    if th < 1e-5:
        # th / (2 sin th) = 1/2 + th^2 / 12 + ...
        phi = (0.5 + th * th / 12.0) * np.array([W[2, 1], W[0, 2], W[1, 0]])
    else:
        phi = th / (2.0 * np.sin(th)) * np.array([W[2, 1], W[0, 2], W[1, 0]])
    P = hat(phi)
    th = float(np.linalg.norm(phi))
    if th < 1e-5:
        D = 1.0 / 12.0 + th * th / 720.0
    else:
        # V^-1 = I - P/2 + D P^2,  D = (1 - th sin th / (2 (1 - cos th))) / th^2
        D = (1.0 - th * np.sin(th) / (2.0 * (1.0 - np.cos(th)))) / th ** 2
    Vinv = np.eye(3) - 0.5 * P + D * (P @ P)
    return np.concatenate([Vinv @ np.asarray(t, np.float64), phi])


def left_update(R, t, xi):
    """Exp(xi) T for T = (R, t)."""
    dR, dt = se3_exp(xi)
    return dR @ R, dR @ t + dt


def pose_residual(R_wc_pred, t_wc_pred, R_wc_opt, t_wc_opt):
    """r_C2 = Log(T(t) T~^-1) for camera-to-world poses (eq:map_optimize_pose)."""
    Ri = R_wc_opt.T
    ti = -Ri @ t_wc_opt
    return se3_log(R_wc_pred @ Ri, R_wc_pred @ ti + t_wc_pred)


@dataclasses.dataclass
class TrackParams:
    iters: int = 30
    l1_weight: float = 0.5
    ssim_weight: float = 0.5
    lr_rho: float = 1e-3
    lr_phi: float = 3e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def tracking_loss(color, target, l1_weight=0.5, ssim_weight=0.5):
    """(L1 term, D-SSIM term, dL/dC) of eq:tracking_loss for [3][h][w] images."""
    color = np.asarray(color, np.float64)
    target = np.asarray(target, np.float64)
    n = color.size
    diff = color - target
    l1 = l1_weight * float(np.abs(diff).sum()) / n
    g = l1_weight * np.sign(diff) / n
    ls, gs = _ssim.dssim(color, target, weight=ssim_weight)
    return l1, ls, g + gs


def adam_step(grad, m, v, k, params: TrackParams):
    """One Adam step on the pose tangent (step k >= 1): returns (delta, m, v)."""
    g = np.asarray(grad, np.float64)
    m = params.beta1 * m + (1.0 - params.beta1) * g
    v = params.beta2 * v + (1.0 - params.beta2) * g * g
    mh = m / (1.0 - params.beta1 ** k)
    vh = v / (1.0 - params.beta2 ** k)
    lr = np.array([params.lr_rho] * 3 + [params.lr_phi] * 3)
    return -lr * mh / (np.sqrt(vh) + params.eps), m, v


def track(g, cam, target, params: TrackParams, tile=16):
    """The full loop: per iteration the pose rendered, the gradient, the two loss terms; and
    the refined pose. cam: scenes.Camera-like (float64 pose), target [3][h][w]."""
    R, t = np.asarray(cam.R_cw, np.float64), np.asarray(cam.t_cw, np.float64)
    m, v = np.zeros(6), np.zeros(6)
    trace = []
    for k in range(1, params.iters + 1):
        c = dataclasses.replace(cam, R_cw=R, t_cw=t)
        img = _render(g, c, tile=tile)
        l1, ls, gC = tracking_loss(img["color"], target, params.l1_weight, params.ssim_weight)
        grad = _backward(g, c, gC, tile=tile)["pose"]
        trace.append(dict(R=R, t=t, grad=grad, l1=l1, ssim=ls))
        delta, m, v = adam_step(grad, m, v, k, params)
        R, t = left_update(R, t, delta)
    return R, t, trace
