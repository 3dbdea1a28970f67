"""One plain single-view mapping step through the C ABI, with every buffer allocated once.

step() enqueues the whole hot path on the current stream with no host synchronisation and no
allocation: projection + SH (gs_preprocess), binning with the alpha-max cull and the (tile,
depth) sort (gs_bin_sort), compositing with the sparse-LiDAR depth term (gs_render_fwd), the
RGB L1 loss (gs_loss_l1), and the backward to every parameter and the pose (gs_render_bwd,
overwrite mode, so the gradients need no clearing). The pair capacity is fitted once, when the
step is built, with 25 % headroom; `overflowed()` (which synchronises) tells whether a later
step needed more.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from . import raster as R


class PlainStep:
    def __init__(self, gm: R.GaussianMap, cam, pix, target_color: torch.Tensor, ds, tile: int = 8, bd: int = 128,
                 dev="cuda:0", lidar_weight: float = 1.0, rgb_weight: float = 1.0):
        self.L = N.lib()
        self.gm = gm
        self.cs = R.camera_struct(cam)
        self.gs = gm.struct()
        self.n = self.gs.n
        self.tile, self.bd, self.dev = tile, bd, dev
        self.rgb_weight = float(rgb_weight)
        self.spl = R.Splats.empty(self.n, dev)
        R.preprocess(self.gs, self.cs, tile, dev, out=self.spl)
        fit = R.bin_sort_fit(self.spl, self.n, self.cs, tile, dev)
        self.capacity = int(fit.pairs() * 1.25) + 1024
        self.bins = R.alloc_bins(self.n, self.cs, tile, self.capacity, dev)
        del fit
        self.frame = R.Frame.empty(cam.h, cam.w, dev)
        self.frame.ensure_state(R.state_bytes(self.bins, self.cs, bd))
        pix_t = torch.as_tensor(pix, dtype=torch.int32).to(dev)
        ds_t = torch.as_tensor(ds, dtype=torch.float32).to(dev)
        self.lidar = R.LidarHits(pix_t, ds_t, weight=lidar_weight)
        self.lidar_loss = torch.zeros(1, device=dev)
        self.rgb_loss = torch.zeros(1, device=dev)
        self.target = target_color.contiguous()
        self.dLdC = torch.empty_like(self.frame.color)
        k = gm.sh_rest.shape[0]
        self.flat = torch.zeros(self.n * (3 + 3 + 4 + 1 + 3 + k) + 6, device=dev)
        views, off = [], 0
        for rows in (3, 3, 4, 1, 3, k):
            views.append(self.flat[off:off + rows * self.n].view(rows, self.n) if rows > 1 else
                         self.flat[off:off + self.n])
            off += rows * self.n
        self.grads = R.ParamGrads(*views, self.flat[off:off + 6])
        self.scratch = R.grads_scratch(self.n, cam.w * cam.h, dev)
        # structs built once (the pointers never change)
        self.s_proj = self.spl.struct()
        self.s_bins = self.bins.struct()
        self.s_img = self.frame.struct()
        has_lidar = self.lidar.m > 0
        self.s_lid_f = self.lidar.struct(self.lidar_loss) if has_lidar else None
        self.s_lid_b = self.lidar.struct(None) if has_lidar else None
        self.s_grads = self.grads.struct(self.scratch, overwrite=True)
        self.p_color = C.c_void_p(self.frame.color.data_ptr())
        self.p_target = C.c_void_p(self.target.data_ptr())
        self.p_dldc = C.c_void_p(self.dLdC.data_ptr())
        self.p_rgbloss = C.c_void_p(self.rgb_loss.data_ptr())
        self.nval = self.frame.color.numel()

    @staticmethod
    def stream():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    @staticmethod
    def _ref(s):
        return C.byref(s) if s is not None else None

    def forward(self, st=None):
        L = self.L
        st = st or self.stream()
        N.check(L.gs_preprocess(C.byref(self.gs), C.byref(self.cs), *R.tile_wh(self.tile), C.byref(self.s_proj), st),
                "gs_preprocess")
        N.check(L.gs_bin_sort(C.byref(self.s_proj), self.n, C.byref(self.cs), C.byref(self.s_bins), st),
                "gs_bin_sort")
        N.check(L.gs_render_fwd(C.byref(self.s_proj), self.n, C.byref(self.s_bins), C.byref(self.cs), self.bd,
                                self._ref(self.s_lid_f), C.byref(self.s_img), st), "gs_render_fwd")

    def step(self):
        L = self.L
        st = self.stream()
        self.forward(st)
        N.check(L.gs_loss_l1(self.p_color, self.p_target, self.nval, self.rgb_weight, self.p_dldc, self.p_rgbloss, st),
                "gs_loss_l1")
        N.check(L.gs_render_bwd(C.byref(self.gs), C.byref(self.cs), C.byref(self.s_proj), C.byref(self.s_bins),
                                C.byref(self.s_img), self.p_dldc, None, None, self._ref(self.s_lid_b), self.bd,
                                C.byref(self.s_grads), st), "gs_render_bwd")

    def overflowed(self) -> bool:
        """True when the last step needed more pairs than the capacity (synchronises)."""
        return self.bins.pairs() > self.capacity
