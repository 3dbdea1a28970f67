"""Torch-facing wrapper of the HIP rasterizer: device buffers, streams and autograd.

Every stage runs in the HIP library (libgs.so); this module only allocates device memory
with torch, passes pointers through the C ABI and keeps the backward checkpoint alive.
The forward saves the splat records, the tile lists and, per pixel, the final
transmittance and the last blended position (8 bytes per pixel) instead of per-fragment
state; the backward re-walks each pixel's list from that checkpoint.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _native as N


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def camera_struct(cam) -> N.Camera:
    """gs_camera from a scenes.Camera (or anything with the same attributes)."""
    R = np.asarray(cam.R_cw, np.float32).ravel()
    t = np.asarray(cam.t_cw, np.float32).ravel()
    bg = np.asarray(getattr(cam, "bg", (0.0, 0.0, 0.0)), np.float32)
    return N.Camera(int(cam.width), int(cam.height), int(cam.x0), int(cam.y0), int(cam.w), int(cam.h),
                    float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), (C.c_float * 9)(*R),
                    (C.c_float * 3)(*t), (C.c_float * 3)(*bg))


def camera_left_update(cs: N.Camera, xi) -> N.Camera:
    out = N.Camera()
    arr = (C.c_float * 6)(*[float(x) for x in xi])
    N.check(N.lib().gs_camera_left_update(C.byref(cs), C.byref(arr), C.byref(out)), "gs_camera_left_update")
    return out


@dataclasses.dataclass
class GaussianMap:
    """Device SoA planes of a Gaussian map (float32)."""

    mean: torch.Tensor
    scale: torch.Tensor
    rot: torch.Tensor
    opacity: torch.Tensor
    sh_dc: torch.Tensor
    sh_rest: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    @staticmethod
    def from_numpy(g, device="cuda") -> "GaussianMap":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        rest = g.sh_rest if g.sh_rest.size else np.zeros((0, g.n), np.float32)
        return GaussianMap(t(g.mean), t(g.scale), t(g.rot), t(g.opacity), t(g.sh_dc), t(rest), g.sh_degree)

    def struct(self) -> N.Gaussians:
        return gaussians_struct(self.mean, self.scale, self.rot, self.opacity, self.sh_dc, self.sh_rest,
                                self.sh_degree)


def gaussians_struct(mean, scale, rot, opacity, sh_dc, sh_rest, deg) -> N.Gaussians:
    for name, t in (("mean", mean), ("scale", scale), ("rot", rot), ("opacity", opacity), ("sh_dc", sh_dc)):
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
    n = int(opacity.shape[0])
    rest = sh_rest if (deg > 0 and sh_rest is not None and sh_rest.numel()) else None
    return N.Gaussians(n, int(deg), _p(mean), _p(scale), _p(rot), _p(opacity), _p(sh_dc), _p(rest))


@dataclasses.dataclass
class Splats:
    """Splat records: card [n][16] float32 (64 B each: centre/opacity/depth, conic/kappa^2,
    colour/clamp bits, tile rectangle/tile count/depth key), n_tiles [n], dkey [n]."""
    card: torch.Tensor
    n_tiles: torch.Tensor
    dkey: torch.Tensor
    pose: torch.Tensor | None = None  # device pose [16] used in place of the camera's (pose_left_update)

    @staticmethod
    def empty(n, device) -> "Splats":
        card = torch.empty(n, 16, dtype=torch.float32, device=device)
        if card.data_ptr() % 64:
            raise RuntimeError("splat cards must be 64-byte aligned")
        return Splats(card, torch.empty(n, dtype=torch.int32, device=device),
                      torch.empty(n, dtype=torch.int32, device=device))

    @property
    def rec_a(self) -> torch.Tensor:
        return self.card[:, 0:4]

    @property
    def rec_b(self) -> torch.Tensor:
        return self.card[:, 4:8]

    @property
    def rgb(self) -> torch.Tensor:
        return self.card[:, 8:12]

    @property
    def rect(self) -> torch.Tensor:
        return self.card[:, 12:14].contiguous().view(torch.int16)

    def struct(self) -> N.Projected:
        return N.Projected(_p(self.card), _p(self.n_tiles), _p(self.dkey), _p(self.pose))


@dataclasses.dataclass
class TileBins:
    tile: object  # side of a square tile, or (tile_w, tile_h)
    capacity: int
    vals: torch.Tensor
    tile_range: torch.Tensor
    num_pairs: torch.Tensor
    scratch: torch.Tensor

    def struct(self) -> N.Bins:
        return N.Bins(*tile_wh(self.tile), self.capacity, _p(self.vals), _p(self.tile_range), _p(self.num_pairs),
                      _p(self.scratch), self.scratch.numel())

    def pairs(self) -> int:
        return int(self.num_pairs.item())


@dataclasses.dataclass
class Frame:
    color: torch.Tensor
    depth: torch.Tensor
    alpha: torch.Tensor
    t_final: torch.Tensor
    last: torch.Tensor
    n_contrib: torch.Tensor | None = None
    state: torch.Tensor | None = None   # chunk work list + per-chunk backward state (uint8)

    @staticmethod
    def empty(h, w, device, count: bool = False) -> "Frame":
        f = lambda *s: torch.empty(*s, dtype=torch.float32, device=device)
        i = lambda: torch.empty(h, w, dtype=torch.int32, device=device)
        return Frame(f(3, h, w), f(h, w), f(h, w), f(h, w), i(), i() if count else None)

    def ensure_state(self, nbytes: int) -> None:
        if self.state is None or self.state.numel() < nbytes:
            self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.color.device)

    def struct(self) -> N.Image:
        st = self.state
        return N.Image(_p(self.color), _p(self.depth), _p(self.alpha), _p(self.t_final), _p(self.last),
                       _p(self.n_contrib), _p(st), st.numel() if st is not None else 0)


@dataclasses.dataclass
class LidarHits:
    """Sparse LiDAR depth: window-linear pixel indices (ascending, int32) and target depths."""

    pix: torch.Tensor
    depth: torch.Tensor
    weight: float = 1.0

    @property
    def m(self) -> int:
        return int(self.pix.numel())

    def struct(self, loss_out=None, grad_scale=None) -> N.Lidar:
        return N.Lidar(self.m, _p(self.pix), _p(self.depth), float(self.weight), _p(loss_out), _p(grad_scale))


def tile_wh(tile) -> tuple[int, int]:
    """(tile_w, tile_h) of a tile given as one side (square) or as a pair."""
    return (int(tile), int(tile)) if isinstance(tile, (int, np.integer)) else (int(tile[0]), int(tile[1]))


def tiles_of(cs: N.Camera, tile) -> int:
    tw, th = tile_wh(tile)
    return ((cs.w + tw - 1) // tw) * ((cs.h + th - 1) // th)


# ---- stage wrappers ------------------------------------------------------------------------

def pose_left_update(cs: N.Camera, xi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Device pose Exp(xi) T_cw of a device tangent xi (6,), in the layout of Splats.pose."""
    xi = xi.detach().to(torch.float32).contiguous()
    out = out if out is not None else torch.empty(16, dtype=torch.float32, device=xi.device)
    N.check(N.lib().gs_pose_left_update(C.byref(cs), _p(xi), _p(out), _stream()), "gs_pose_left_update")
    return out


def preprocess(gs: N.Gaussians, cs: N.Camera, tile: int, device, out: Splats | None = None,
               pose: torch.Tensor | None = None) -> Splats:
    out = out or Splats.empty(gs.n, device)
    out.pose = pose
    N.check(N.lib().gs_preprocess(C.byref(gs), C.byref(cs), *tile_wh(tile), C.byref(out.struct()), _stream()),
            "gs_preprocess")
    return out


def alloc_bins(n: int, cs: N.Camera, tile: int, capacity: int, device) -> TileBins:
    T = tiles_of(cs, tile)
    sb = N.lib().gs_bins_scratch_bytes(n, capacity, T)
    return TileBins(tile, capacity, torch.empty(max(capacity, 1), dtype=torch.int32, device=device),
                    torch.empty(2 * T, dtype=torch.int32, device=device), torch.zeros(1, dtype=torch.int64, device=device),
                    torch.empty(sb, dtype=torch.uint8, device=device))


def bin_sort(spl: Splats, n: int, cs: N.Camera, bins: TileBins) -> TileBins:
    N.check(N.lib().gs_bin_sort(C.byref(spl.struct()), n, C.byref(cs), C.byref(bins.struct()), _stream()),
            "gs_bin_sort")
    return bins


def bin_sort_fit(spl: Splats, n: int, cs: N.Camera, tile: int, device, capacity: int | None = None) -> TileBins:
    """Bin and sort; if the required pair count exceeds the capacity, grow and run again."""
    cap = int(capacity or max(1024, 4 * n))
    while True:
        bins = bin_sort(spl, n, cs, alloc_bins(n, cs, tile, cap, device))
        need = bins.pairs()
        if need <= cap:
            return bins
        cap = int(math.ceil(need * 1.25))


def state_bytes(bins: TileBins, cs: N.Camera, blend_depth: int) -> int:
    return N.lib().gs_image_state_bytes(bins.capacity, tiles_of(cs, bins.tile), *tile_wh(bins.tile), blend_depth)


def render_fwd(spl: Splats, n: int, bins: TileBins, cs: N.Camera, blend_depth: int, device,
               lidar: LidarHits | None = None, lidar_loss: torch.Tensor | None = None,
               out: Frame | None = None) -> Frame:
    out = out or Frame.empty(cs.h, cs.w, device)
    out.ensure_state(state_bytes(bins, cs, blend_depth))
    ls = lidar.struct(lidar_loss) if lidar is not None and lidar.m > 0 else None
    N.check(N.lib().gs_render_fwd(C.byref(spl.struct()), n, C.byref(bins.struct()), C.byref(cs), blend_depth,
                                  C.byref(ls) if ls is not None else None, C.byref(out.struct()), _stream()),
            "gs_render_fwd")
    return out


@dataclasses.dataclass
class ParamGrads:
    mean: torch.Tensor
    scale: torch.Tensor
    rot: torch.Tensor
    opacity: torch.Tensor
    sh_dc: torch.Tensor
    sh_rest: torch.Tensor
    pose: torch.Tensor

    @staticmethod
    def zeros(gm: GaussianMap) -> "ParamGrads":
        z = torch.zeros_like
        return ParamGrads(z(gm.mean), z(gm.scale), z(gm.rot), z(gm.opacity), z(gm.sh_dc), z(gm.sh_rest),
                          torch.zeros(6, dtype=torch.float32, device=gm.mean.device))

    @staticmethod
    def empty(gm: GaussianMap) -> "ParamGrads":
        """Uninitialised outputs, for a backward called with overwrite=True (writes every element)."""
        e = torch.empty_like
        return ParamGrads(e(gm.mean), e(gm.scale), e(gm.rot), e(gm.opacity), e(gm.sh_dc), e(gm.sh_rest),
                          torch.empty(6, dtype=torch.float32, device=gm.mean.device))

    def struct(self, scratch: torch.Tensor | None, overwrite: bool = False, schedule: int = N.GS_BWD_CHUNKS) -> N.Grads:
        rest = self.sh_rest if self.sh_rest.numel() else None
        return N.Grads(_p(self.mean), _p(self.scale), _p(self.rot), _p(self.opacity), _p(self.sh_dc), _p(rest),
                       _p(self.pose), _p(scratch), scratch.numel() if scratch is not None else 0,
                       int(bool(overwrite)), int(schedule))


def grads_scratch(n: int, pixels: int, device, views: int = 1) -> torch.Tensor:
    return torch.empty(N.lib().gs_grads_scratch_bytes(n, views, pixels), dtype=torch.uint8, device=device)


def render_bwd(gs: N.Gaussians, cs: N.Camera, spl: Splats, bins: TileBins, fr: Frame, dL_dC, dL_dD, dL_dO,
               blend_depth: int, grads: ParamGrads, scratch: torch.Tensor | None, lidar: LidarHits | None = None,
               grad_scale: torch.Tensor | None = None, overwrite: bool = False,
               schedule: int = N.GS_BWD_CHUNKS, noalloc: bool = False) -> ParamGrads:
    """overwrite=False adds the gradients to `grads`; overwrite=True writes every element.
    schedule: GS_BWD_CHUNKS (pixel-parallel, default) or GS_BWD_BUCKETS (per-Gaussian buckets).
    noalloc=True calls gs_render_bwd_noalloc (library-owned scratch; `scratch` is ignored)."""
    ls = lidar.struct(None, grad_scale) if lidar is not None and lidar.m > 0 else None
    fn = N.lib().gs_render_bwd_noalloc if noalloc else N.lib().gs_render_bwd
    N.check(fn(C.byref(gs), C.byref(cs), C.byref(spl.struct()), C.byref(bins.struct()),
               C.byref(fr.struct()), _p(dL_dC), _p(dL_dD), _p(dL_dO),
               C.byref(ls) if ls is not None else None, blend_depth,
               C.byref(grads.struct(None if noalloc else scratch, overwrite, schedule)), _stream()),
            "gs_render_bwd_noalloc" if noalloc else "gs_render_bwd")
    return grads


def loss_l1(color: torch.Tensor, target: torch.Tensor, weight: float = 1.0, dL_dC: torch.Tensor | None = None,
            loss_out: torch.Tensor | None = None):
    n = color.numel()
    dL_dC = dL_dC if dL_dC is not None else torch.empty_like(color)
    loss_out = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=color.device)
    N.check(N.lib().gs_loss_l1(_p(color), _p(target), n, float(weight), _p(dL_dC), _p(loss_out), _stream()),
            "gs_loss_l1")
    return loss_out, dL_dC


# ---- autograd --------------------------------------------------------------------------------

def loss_dssim(color: torch.Tensor, target: torch.Tensor, weight: float = 1.0,
               dL_dC: torch.Tensor | None = None, loss: torch.Tensor | None = None,
               scratch: torch.Tensor | None = None) -> torch.Tensor:
    """weight * (1 - mean SSIM) of [c][h][w] images; adds its gradient to dL_dC when given."""
    c, h, w = (int(v) for v in color.shape)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=color.device)
    nb = N.lib().gs_dssim_scratch_bytes(c, h, w)
    if scratch is None or scratch.numel() < nb:
        scratch = torch.empty(max(nb, 1), dtype=torch.uint8, device=color.device)
    N.check(N.lib().gs_loss_dssim(_p(color), _p(target), c, h, w, float(weight), _p(dL_dC), _p(loss), _p(scratch),
                                  scratch.numel(), _stream()), "gs_loss_dssim")
    return loss


@dataclasses.dataclass
class RenderSettings:
    camera: object                  # scenes.Camera-like
    tile: object = 8                # square side, or (tile_w, tile_h)
    blend_depth: int = 128
    lidar: LidarHits | None = None  # sparse depth term evaluated inside the library
    capacity: int | None = None     # pair capacity; learned from the first call when None
    sync_check: bool = False        # True: read the pair count back after every forward
    _pending: list = dataclasses.field(default_factory=list, repr=False)

    def check(self, wait: bool = True) -> None:
        """Raise if an earlier forward needed more pairs than its capacity (its lists were
        clamped and its outputs are invalid); the capacity is grown for later calls.
        wait=False only looks at forwards whose pair count has already arrived."""
        keep, bad = [], None
        for ev, host, cap in self._pending:
            if not wait and not ev.query():
                keep.append((ev, host, cap))
                continue
            ev.synchronize()
            need = int(host.item())
            if need > 0.8 * (self.capacity or 0):
                self.capacity = int(math.ceil(need * 1.25))
            if need > cap and bad is None:
                bad = (need, cap)
        self._pending = keep
        if bad is not None:
            raise RuntimeError(f"a forward needed {bad[0]} (tile, Gaussian) pairs but had capacity {bad[1]}: its "
                               f"outputs are invalid; capacity grown to {self.capacity}, render it again")


def _bin_sort_async(settings: RenderSettings, spl: Splats, n: int, cs: N.Camera, dev) -> TileBins:
    """Binning without a host round trip once the capacity is known: the pair count is copied
    to pinned host memory behind an event and checked by a later call (RenderSettings.check)."""
    settings.check(wait=False)
    if settings.capacity is None or settings.sync_check:
        bins = bin_sort_fit(spl, n, cs, settings.tile, dev, settings.capacity)
        settings.capacity = max(settings.capacity or 0, int(math.ceil(bins.pairs() * 1.25)), 1024)
        return bins
    bins = bin_sort(spl, n, cs, alloc_bins(n, cs, settings.tile, settings.capacity, dev))
    host = torch.empty(1, dtype=torch.int64, pin_memory=True)
    host.copy_(bins.num_pairs, non_blocking=True)
    ev = torch.cuda.Event()
    ev.record()
    settings._pending.append((ev, host, bins.capacity))
    return bins


class GSRender(torch.autograd.Function):
    """(mean, scale, rot, opacity, sh_dc, sh_rest, pose_tangent) -> (color, depth, alpha, lidar_loss).

    pose_tangent xi (6,) is applied as T_cw <- Exp(xi) T_cw; its gradient is the left-
    perturbation gradient at the rendered pose (exact at xi = 0, the way a tracking loop
    uses it: fold xi into the pose after each step and reset it to zero).

    No host round trip once the settings know the pair capacity: a device tangent is turned
    into the device pose the projection reads (gs_pose_left_update), and the pair count is
    checked one call late (RenderSettings.check).
    """

    @staticmethod
    def forward(ctx, settings: RenderSettings, mean, scale, rot, opacity, sh_dc, sh_rest, pose_tangent):
        dev = mean.device
        deg = int(round(math.sqrt(sh_rest.shape[0] // 3 + 1))) - 1 if sh_rest.numel() else 0
        cs = camera_struct(settings.camera)
        pose = None
        if pose_tangent is not None:
            if pose_tangent.device.type == "cpu":
                xi = pose_tangent.detach().float().numpy()
                if np.any(xi != 0):
                    cs = camera_left_update(cs, xi)
            else:
                pose = pose_left_update(cs, pose_tangent)
        gs = gaussians_struct(mean, scale, rot, opacity, sh_dc, sh_rest, deg)
        n = gs.n
        spl = preprocess(gs, cs, settings.tile, dev, pose=pose)
        bins = _bin_sort_async(settings, spl, n, cs, dev)
        lidar = settings.lidar
        lloss = torch.zeros(1, dtype=torch.float32, device=dev)
        fr = render_fwd(spl, n, bins, cs, settings.blend_depth, dev, lidar, lloss)
        ctx.settings, ctx.cs, ctx.deg = settings, cs, deg
        ctx.spl, ctx.bins, ctx.fr = spl, bins, fr
        ctx.has_pose = pose_tangent is not None
        ctx.pose_device = pose_tangent.device if pose_tangent is not None else None
        ctx.save_for_backward(mean, scale, rot, opacity, sh_dc, sh_rest)
        return fr.color, fr.depth, fr.alpha, lloss[0]

    @staticmethod
    def backward(ctx, gC, gD, gO, gL):
        mean, scale, rot, opacity, sh_dc, sh_rest = ctx.saved_tensors
        dev = mean.device
        gs = gaussians_struct(mean, scale, rot, opacity, sh_dc, sh_rest, ctx.deg)
        gm = GaussianMap(mean, scale, rot, opacity, sh_dc, sh_rest, ctx.deg)
        grads = ParamGrads.empty(gm)  # the backward writes every element
        cs = ctx.cs
        gC = torch.zeros_like(ctx.fr.color) if gC is None else gC.contiguous()
        gD = None if gD is None else gD.contiguous()
        gO = None if gO is None else gO.contiguous()
        lidar = ctx.settings.lidar
        scale_t = None
        if lidar is not None and lidar.m > 0:
            scale_t = (torch.ones(1, device=dev) if gL is None else gL.reshape(1).float().contiguous())
        scratch = grads_scratch(gs.n, cs.w * cs.h, dev)
        render_bwd(gs, cs, ctx.spl, ctx.bins, ctx.fr, gC, gD, gO, ctx.settings.blend_depth, grads, scratch,
                   lidar, scale_t, overwrite=True)
        gpose = grads.pose.to(ctx.pose_device) if ctx.has_pose else None
        return None, grads.mean, grads.scale, grads.rot, grads.opacity, grads.sh_dc, grads.sh_rest, gpose


def render(settings: RenderSettings, gm: GaussianMap, pose_tangent: torch.Tensor | None = None):
    """Differentiable render. Returns (color [3,h,w], depth [h,w], alpha [h,w], lidar_loss [])."""
    return GSRender.apply(settings, gm.mean, gm.scale, gm.rot, gm.opacity, gm.sh_dc, gm.sh_rest, pose_tangent)


def checkpoint_bytes(cam) -> int:
    """Bytes of the per-pixel checkpoint of one view (final transmittance + last contributor)."""
    return int(cam.w) * int(cam.h) * 8


def kept_bytes(spl: Splats, bins: TileBins, fr: Frame, cs: N.Camera, blend_depth: int) -> dict:
    """Device bytes the forward of one view leaves for its backward:
    checkpoint    final transmittance and last contributor per pixel (8 B);
    chunk_state   the compositing work list and, per (chunk, pixel) of tiles longer than one
                  chunk, the transmittance and colour behind the chunk (gs_image_state_bytes:
                  `allocated` from the pair capacity, `needed` from this view's pair count);
    tile_lists    sorted record indices (capacity) and per-tile ranges;
    splat_records the 64-B splat cards, tile counts and depth keys of every Gaussian.
    Reads the pair count back (synchronises)."""
    T = tiles_of(cs, bins.tile)
    lib = N.lib()
    pairs = bins.pairs()
    state_alloc = fr.state.numel() if fr.state is not None else 0
    state_needed = lib.gs_image_state_bytes(pairs, T, *tile_wh(bins.tile), blend_depth)
    out = {
        "checkpoint": fr.t_final.numel() * 4 + fr.last.numel() * 4,
        "chunk_state_allocated": int(state_alloc),
        "chunk_state_needed": int(state_needed),
        "tile_lists": bins.vals.numel() * 4 + bins.tile_range.numel() * 4,
        "splat_records": spl.card.numel() * 4 + spl.n_tiles.numel() * 4 + spl.dkey.numel() * 4,
    }
    out["total_allocated"] = out["checkpoint"] + out["chunk_state_allocated"] + out["tile_lists"] + \
        out["splat_records"]
    return out
