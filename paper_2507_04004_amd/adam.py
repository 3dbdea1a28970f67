"""Sparse Adam over a Gaussian map (Sec. "Additional Strategies", a): binding of gs_adam_sparse.

SparseAdam keeps the raw parameters the optimiser works on and their moments. The map's mean,
quaternion and SH planes are optimised in place; scale and opacity have raw twins (log-scale,
opacity logit), and every step writes the renderer's scale = exp(log-scale) and opacity =
1 / (1 + exp(-logit)) back into the map for the Gaussians it updated. A step updates the
Gaussians that the rendering reached: those with a non-zero tile count in some view.
Learning rates default to the original 3DGS recipe, which the paper keeps without decay.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .raster import GaussianMap, ParamGrads, _p, _stream

# mean (times the scene scale), log-scale, quaternion, opacity logit, SH DC, SH rest
LR_3DGS = {"mean": 1.6e-4, "scale": 5e-3, "rot": 1e-3, "opacity": 5e-2, "sh_dc": 2.5e-3, "sh_rest": 2.5e-3 / 20}


class SparseAdam:
    def __init__(self, gm: GaussianMap, lr: dict | None = None, scene_scale: float = 1.0,
                 betas: tuple[float, float] = (0.9, 0.999), eps: float = 1e-15):
        self.gm = gm
        lr = {**LR_3DGS, **(lr or {})}
        self.log_scale = torch.log(gm.scale)
        self.logit_opacity = torch.log(gm.opacity) - torch.log1p(-gm.opacity)
        # (raw parameter, plane the renderer reads when it differs, gradient name, activation, lr)
        self.groups = [
            (gm.mean, None, "mean", N.GS_ACT_NONE, lr["mean"] * scene_scale),
            (self.log_scale, gm.scale, "scale", N.GS_ACT_EXP, lr["scale"]),
            (gm.rot, None, "rot", N.GS_ACT_NONE, lr["rot"]),
            (self.logit_opacity, gm.opacity, "opacity", N.GS_ACT_SIGMOID, lr["opacity"]),
            (gm.sh_dc, None, "sh_dc", N.GS_ACT_NONE, lr["sh_dc"]),
            (gm.sh_rest, None, "sh_rest", N.GS_ACT_NONE, lr["sh_rest"]),
        ]
        self.exp_avg = [torch.zeros_like(g[0]) for g in self.groups]
        self.exp_avg_sq = [torch.zeros_like(g[0]) for g in self.groups]
        self.betas, self.eps, self.step_count = betas, eps, 0

    def struct(self, grads: ParamGrads, visible: torch.Tensor | None) -> N.Adam:
        n = self.gm.n
        a = N.Adam()
        a.n, a.n_groups = n, len(self.groups)
        if visible is not None:
            if visible.dtype != torch.int32 and visible.dtype != torch.uint32:
                raise ValueError("visible must hold the uint32 tile counts of gs_preprocess")
            visible = visible.reshape(-1, n)
            if not visible.is_contiguous():
                raise ValueError("visible must be contiguous [views][n]")
            a.visible, a.n_views = _p(visible), int(visible.shape[0])
        t = self.step_count
        # the kernel runs on the float32 betas: the bias terms use the same values
        b1, b2 = (float(np.float32(b)) for b in self.betas)
        a.beta1, a.beta2, a.eps = b1, b2, self.eps
        a.bias1, a.bias2 = 1.0 - b1 ** t, 1.0 - b2 ** t
        for i, (raw, act_out, name, act, lr) in enumerate(self.groups):
            k = raw.numel() // n if n else 0  # planes (opacity is a single [n] plane)
            g = getattr(grads, name)
            a.group[i] = N.AdamGroup(_p(raw) if k else None, _p(self.exp_avg[i]) if k else None,
                                     _p(self.exp_avg_sq[i]) if k else None, _p(g) if k else None,
                                     _p(act_out), k, act, lr)
        return a

    def step(self, grads: ParamGrads, visible: torch.Tensor | None = None) -> None:
        """One step; visible: tile counts [views][n] of the rendering (None: every Gaussian)."""
        self.step_count += 1
        a = self.struct(grads, visible)
        N.check(N.lib().gs_adam_sparse(C.byref(a), _stream()), "gs_adam_sparse")
