"""Photometric tracking (camera factor option 2, eq:tracking_loss): binding of gs_track_pose.

With the Gaussian map frozen, a PoseTracker refines a camera pose against an observed image by
N_t Adam iterations (30 in the paper's setup) on L = 1/2 mean |C_hat - C| + 1/2 D-SSIM. Each
iteration renders, evaluates both terms, differentiates to the 6-DoF pose tangent and steps the
pose; all of it runs in the HIP library with the pose kept on the device, and with graph=True the
iterations are one captured hipGraph replayed for every frame with the same buffers. The refined
pose T~ feeds the factor residual r_C2 = Log(T(t) T~^-1) (eq:map_optimize_pose).

The paper gives no step sizes for the pose; the defaults here (1e-3 for the translation in map
units, 3e-3 rad for the rotation) are parameters.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _native as N
from . import raster as R

DEFAULTS = dict(iters=30, l1_weight=0.5, ssim_weight=0.5, lr_rho=1e-2, lr_phi=1e-3, beta1=0.9, beta2=0.999,
                eps=1e-8)


@dataclasses.dataclass
class TrackResult:
    """pose and trace are the tracker's own buffers: the next track() call overwrites them
    (clone them to keep a result)."""

    pose: torch.Tensor            # [12] device: refined R_cw (row-major) then t_cw
    trace: torch.Tensor | None    # [iters, 20] device: pose rendered, dL/dxi, L1 term, D-SSIM term
    pairs: int | None = None      # largest pair count over the iterations (when checked)

    def camera(self, cam):
        """A copy of `cam` (scenes.Camera-like) at the refined pose."""
        p = self.pose.double().cpu().numpy()
        return dataclasses.replace(cam, R_cw=p[:9].reshape(3, 3), t_cw=p[9:12])


class PoseTracker:
    """Owns one tracking plan; calls are ordered on the current torch stream."""

    def __init__(self, gm: R.GaussianMap, max_pixels: int, tile: int = 8, blend_depth: int = 128,
                 capacity: int | None = None, device="cuda"):
        self.gm, self.max_pixels, self.tile, self.blend_depth = gm, int(max_pixels), tile, blend_depth
        self.device = device
        self.capacity = int(capacity) if capacity else 0
        self._plan = C.c_void_p()
        self.pose = torch.empty(12, dtype=torch.float32, device=device)
        self._trace = None

    def _create(self, capacity: int):
        self.close()
        self.capacity = int(capacity)
        N.check(N.lib().gs_track_plan_create(C.byref(self._plan), self.gm.n, self.gm.sh_degree, self.max_pixels,
                                             *R.tile_wh(self.tile), self.blend_depth, self.capacity),
                "gs_track_plan_create")

    def close(self):
        if self._plan:
            N.lib().gs_track_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pairs_at(self, cs: N.Camera) -> int:
        """(tile, Gaussian) pairs of one render at camera `cs` (synchronises)."""
        spl = R.preprocess(self.gm.struct(), cs, self.tile, self.device)
        return int(spl.n_tiles.to(torch.int64).sum().item())

    def required_pairs(self) -> int:
        out = C.c_int64()
        N.check(N.lib().gs_track_required_pairs(self._plan, C.byref(out), R._stream()), "gs_track_required_pairs")
        return int(out.value)

    def track(self, cam, target: torch.Tensor, graph: bool = True, trace: bool = False, check: bool = True,
              **params) -> TrackResult:
        """Refine the pose of `cam` (scenes.Camera-like or gs_camera) against target [3, h, w].

        check=True reads back the largest pair count (one synchronisation) and, if the tile
        lists overflowed, grows the plan and runs the loop again."""
        cs = cam if isinstance(cam, N.Camera) else R.camera_struct(cam)
        q = {**DEFAULTS, **params}
        qp = N.TrackParams(int(q["iters"]), float(q["l1_weight"]), float(q["ssim_weight"]), float(q["lr_rho"]),
                           float(q["lr_phi"]), float(q["beta1"]), float(q["beta2"]), float(q["eps"]),
                           N.GS_GRAPH if graph else 0)
        if not self._plan:
            self._create(self.capacity or max(1 << 16, math.ceil(1.5 * self.pairs_at(cs))))
        if trace and (self._trace is None or self._trace.shape[0] != qp.iters):
            self._trace = torch.empty(qp.iters, N.TRACK_TRACE_STRIDE, dtype=torch.float32, device=self.device)
        tr = self._trace if trace else None
        gs = self.gm.struct()
        target = target.contiguous()
        while True:
            N.check(N.lib().gs_track_pose(self._plan, C.byref(gs), C.byref(cs), R._p(target), C.byref(qp),
                                          R._p(self.pose), R._p(tr), R._stream()), "gs_track_pose")
            if not check:
                return TrackResult(self.pose, tr)
            need = self.required_pairs()
            if need <= self.capacity:
                return TrackResult(self.pose, tr, need)
            self._create(math.ceil(1.25 * need))


def pose_residual(pred_cw, refined_cw) -> np.ndarray:
    """r_C2 = Log(T_wc(t) T~_wc^-1) from two world-to-camera poses given as 12 floats (R_cw
    row-major, t_cw), as gs_pose_residual computes it on the host."""
    a = (C.c_float * 12)(*[float(x) for x in np.asarray(pred_cw, np.float64).ravel()])
    b = (C.c_float * 12)(*[float(x) for x in np.asarray(refined_cw, np.float64).ravel()])
    r = (C.c_double * 6)()
    N.check(N.lib().gs_pose_residual(C.byref(a), C.byref(b), C.byref(r)), "gs_pose_residual")
    return np.array(r[:])
