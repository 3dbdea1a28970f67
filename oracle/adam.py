"""FP64 sparse Adam over the Gaussian attributes — TEST INFRASTRUCTURE ONLY.

Map optimisation updates the Gaussians with Adam, but only those that took part in the
rendering (Sec. "Additional Strategies", a, sparse Adam): a Gaussian that no view of the pass
reached keeps its parameters and both moments unchanged, while the step counter is shared by
all of them. "Took part" is read as: the projection kept at least one tile for it in some view
(tile count > 0 after the alpha-max cull), the same set the compositing walks.

Adam is the published algorithm (first and second moment estimates with bias correction):
    m <- b1 m + (1 - b1) g,    v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
with t the step number (1 for the first step).

Parameters are optimised in the raw form of the original 3DGS recipe, whose learning rates
the paper keeps (no decay): mean, log-scale, unnormalised quaternion, opacity logit and the
SH coefficients. The renderer reads scale = exp(log-scale) and opacity = sigmoid(logit); its
gradients are w.r.t. those, so the raw gradient is g * exp(raw) and g * o (1 - o), taken at
the values before the step, and the activated values are recomputed after it.
"""
from __future__ import annotations

import numpy as np

ACT_NONE, ACT_EXP, ACT_SIGMOID = 0, 1, 2


def activate(raw, act):
    raw = np.asarray(raw, np.float64)
    if act == ACT_EXP:
        return np.exp(raw)
    if act == ACT_SIGMOID:
        return 1.0 / (1.0 + np.exp(-raw))
    return raw


def raw_grad(raw, grad_act, act):
    """Gradient w.r.t. the raw parameter from the gradient w.r.t. the renderer's value."""
    raw = np.asarray(raw, np.float64)
    g = np.asarray(grad_act, np.float64)
    if act == ACT_EXP:
        return g * np.exp(raw)
    if act == ACT_SIGMOID:
        s = 1.0 / (1.0 + np.exp(-raw))
        return g * s * (1.0 - s)
    return g


def visible_mask(n_tiles):
    """[views][n] tile counts -> bool [n]: reached by some view."""
    nt = np.asarray(n_tiles).reshape(-1, np.asarray(n_tiles).shape[-1])
    return (nt > 0).any(axis=0)


def sparse_adam_step(group, visible, step, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step on one parameter group, in place on float64 copies.

    group: dict with 'param' [k][n], 'exp_avg' [k][n], 'exp_avg_sq' [k][n], 'grad' [k][n]
    (w.r.t. the renderer's value), 'act', 'lr'. Returns the activated values [k][n].
    """
    p, m, v = group["param"], group["exp_avg"], group["exp_avg_sq"]
    g = raw_grad(p, group["grad"], group["act"])
    vis = np.asarray(visible, bool)
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    m_new = beta1 * m + (1.0 - beta1) * g
    v_new = beta2 * v + (1.0 - beta2) * g * g
    p_new = p - group["lr"] * (m_new / bc1) / (np.sqrt(v_new / bc2) + eps)
    m[:, vis] = m_new[:, vis]
    v[:, vis] = v_new[:, vis]
    p[:, vis] = p_new[:, vis]
    return activate(p, group["act"])
