"""Batched rendering of several views of one map per launch (gs_render_batch).

A BatchPlan owns the splat records, tile lists and scratch for up to 16 views; one launch per
stage covers every view's Gaussians or tiles. With graph=True the stage sequence is captured
into a hipGraph by the library on first use and replayed while the arguments are unchanged.
This is the multi-keyframe form of the map optimisation (several keyframes per pass instead
of one at a time) and the batching layer of the serving loop.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import torch

from . import _native as N
from . import raster as R


@dataclasses.dataclass
class ViewSlot:
    """One view of a batch: camera, output planes and (for the backward) its loss inputs."""

    camera: object
    frame: R.Frame
    target: torch.Tensor | None = None        # [3,h,w]: RGB L1 term computed inside the batch
    rgb_weight: float = 1.0
    rgb_loss: torch.Tensor | None = None      # [1]
    dL_dC: torch.Tensor | None = None         # used when target is None
    dL_dD: torch.Tensor | None = None
    dL_dO: torch.Tensor | None = None
    lidar: R.LidarHits | None = None
    lidar_loss: torch.Tensor | None = None    # [1]
    pose_grad: torch.Tensor | None = None     # [6], accumulated

    @staticmethod
    def make(camera, device, backward=False, lidar=None, target=None):
        fr = R.Frame.empty(camera.h, camera.w, device)
        z = lambda k: torch.zeros(k, dtype=torch.float32, device=device)
        return ViewSlot(camera, fr, target=target, rgb_loss=z(1) if target is not None else None, lidar=lidar,
                        lidar_loss=z(1) if lidar is not None else None, pose_grad=z(6) if backward else None)

    def struct(self) -> N.View:
        p = R._p
        lid = self.lidar.struct(self.lidar_loss) if self.lidar is not None and self.lidar.m > 0 else N.Lidar()
        return N.View(R.camera_struct(self.camera), self.frame.struct(), p(self.dL_dC), p(self.dL_dD), p(self.dL_dO),
                      lid, p(self.target), float(self.rgb_weight), p(self.rgb_loss), p(self.pose_grad))


def plan_bytes(n: int, sh_degree: int, max_views: int, max_total_pixels: int, tile: int, blend_depth: int,
               capacity: int, fwd_only: bool = False) -> int:
    """Device bytes of a BatchPlan with these arguments (gs_batch_plan_bytes)."""
    return int(N.lib().gs_batch_plan_bytes(n, sh_degree, max_views, max_total_pixels, *R.tile_wh(tile), blend_depth,
                                           capacity, N.GS_PLAN_FWD_ONLY if fwd_only else 0))


class BatchPlan:
    def __init__(self, n: int, sh_degree: int, max_views: int, max_total_pixels: int, tile: int = 16,
                 blend_depth: int = 256, capacity: int | None = None, device="cuda", fwd_only: bool = False):
        """fwd_only: a plan that only renders (no backward scratch)."""
        self.n, self.sh_degree, self.max_views = n, sh_degree, max_views
        self.max_total_pixels = max_total_pixels
        self.tile, self.blend_depth = tile, blend_depth
        self.capacity = int(capacity or max(1 << 16, 8 * n * max_views // 4))
        self.device = device
        self.fwd_only = fwd_only
        self._plan = C.c_void_p()
        N.check(N.lib().gs_batch_plan_create(C.byref(self._plan), n, sh_degree, max_views, max_total_pixels, *R.tile_wh(tile),
                                             blend_depth, self.capacity, N.GS_PLAN_FWD_ONLY if fwd_only else 0),
                "gs_batch_plan_create")
        self.nbytes = plan_bytes(n, sh_degree, max_views, max_total_pixels, tile, blend_depth, self.capacity,
                                 fwd_only)
        self._keep = None

    def close(self):
        if self._plan:
            N.lib().gs_batch_plan_destroy(self._plan)
            self._plan = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, gm: R.GaussianMap, views: list[ViewSlot], fwd=True, bwd=False, grads: R.ParamGrads | None = None,
            graph=False, grad_scratch=None, overwrite=False, schedule: int = N.GS_BWD_CHUNKS):
        """overwrite=False adds the batch's gradients to `grads`; True writes every element.
        schedule: the compositing-backward schedule (GS_BWD_CHUNKS or GS_BWD_BUCKETS)."""
        mode = (N.GS_FWD if fwd else 0) | (N.GS_BWD if bwd else 0) | (N.GS_GRAPH if graph else 0)
        arr = (N.View * len(views))(*[v.struct() for v in views])
        gs = gm.struct()
        gst = (grads.struct(torch.empty(0, dtype=torch.uint8, device=self.device), overwrite, schedule)
               if grads is not None else None)
        self._keep = (arr, gs, gst)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        N.check(N.lib().gs_render_batch(self._plan, C.byref(gs), len(views), arr, mode,
                                        C.byref(gst) if gst is not None else None, st), "gs_render_batch")

    def num_pairs(self) -> int:
        """Required pair count of the last run (synchronises the current stream)."""
        out = C.c_int64()
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        N.check(N.lib().gs_batch_num_pairs(self._plan, C.byref(out), st), "gs_batch_num_pairs")
        return int(out.value)

    def overflowed(self) -> bool:
        return self.num_pairs() > self.capacity
