"""Shared helpers for the GPU tests: run the HIP path through the C ABI and compare it with
the CPU oracle under the stated tolerances."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2507_04004_amd import raster as R

DEV = "cuda:0"
IMG_ATOL = 1e-4        # colour / opacity / transmittance, max-abs, non-marginal pixels
DEPTH_RTOL = 1e-4      # depth: 1e-4 relative to the mean composited depth D/O, absolute below 1 m
GRAD_RTOL = 2e-3       # gradients: relative, per element
GRAD_ATOL = 2e-5       # per-element floor, a fraction of the block's largest element (float32 sums that cancel)


class HipRun:
    """One plain single-view pass through the C ABI, keeping every intermediate."""

    def __init__(self, g, cam, tile=16, blend_depth=256, lidar=None, capacity=None):
        self.g, self.cam, self.tile, self.bd = g, cam, tile, blend_depth
        self.gm = R.GaussianMap.from_numpy(g, DEV)
        self.cs = R.camera_struct(cam)
        self.gs = self.gm.struct()
        self.spl = R.preprocess(self.gs, self.cs, tile, DEV)
        self.bins = R.bin_sort_fit(self.spl, self.gs.n, self.cs, tile, DEV, capacity)
        self.lidar = lidar
        self.lidar_loss = torch.zeros(1, device=DEV)
        self.fr = R.render_fwd(self.spl, self.gs.n, self.bins, self.cs, blend_depth, DEV, lidar, self.lidar_loss)
        torch.cuda.synchronize()

    def image(self):
        f = self.fr
        return dict(color=f.color.cpu().numpy(), depth=f.depth.cpu().numpy(), alpha=f.alpha.cpu().numpy(),
                    t_final=f.t_final.cpu().numpy(), last=f.last.cpu().numpy())

    def backward(self, gC, gD=None, gO=None, grad_scale=None, overwrite=False, grads=None, schedule=0, noalloc=False):
        if grads is None:
            grads = R.ParamGrads.zeros(self.gm)
        scratch = None if noalloc else R.grads_scratch(self.gs.n, self.cam.w * self.cam.h, DEV)
        t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)
        R.render_bwd(self.gs, self.cs, self.spl, self.bins, self.fr, t(gC), t(gD), t(gO), self.bd, grads, scratch,
                     self.lidar, grad_scale, overwrite=overwrite, schedule=schedule, noalloc=noalloc)
        torch.cuda.synchronize()
        return {k: getattr(grads, k).cpu().numpy().astype(np.float64) for k in
                ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest", "pose")}

    def bins_np(self):
        P = self.bins.pairs()
        return dict(vals=self.bins.vals[:P].cpu().numpy().view(np.uint32),
                    tile_range=self.bins.tile_range.cpu().numpy().view(np.uint32), num_pairs=P,
                    n_tiles=self.spl.n_tiles.cpu().numpy().view(np.uint32),
                    rect=self.spl.rect.cpu().numpy().astype(np.int32),
                    dkey=self.spl.dkey.cpu().numpy().view(np.uint32))


def oracle_cam(cam):
    return oracle.camera_f32(cam)


MARGINAL_FRAC = 5e-3   # at most this share of the pixels may be left out as marginal
MARGINAL_ATOL = 2e-2   # colour / opacity at marginal pixels: a few decisions at 1/255 flipped


def compare_images(gpu, ref, mask=None):
    """Max-abs differences on non-marginal pixels (and colour / opacity on the marginal ones).
    Returns dict of errors."""
    ok = ref["marginal"] == 0 if mask is None else mask
    dc = np.abs(gpu["color"] - ref["color"])
    da = np.abs(gpu["alpha"] - ref["alpha"])
    dt = np.abs(gpu["t_final"] - ref["t_final"])
    dd = np.abs(gpu["depth"] - ref["depth"])
    out = {}
    out["color"] = float(dc[:, ok].max(initial=0.0))
    out["alpha"] = float(da[ok].max(initial=0.0))
    out["t_final"] = float(dt[ok].max(initial=0.0))
    # depth composites the splat depths with the colour weights, so its float32 error is the
    # weights' error times those depths: relative to the pixel's mean composited depth D / O
    # (at least 1 m)
    dref, oref = ref["depth"][ok], ref["alpha"][ok]
    dscale = np.maximum(1.0, np.abs(dref) / np.maximum(oref, 1e-12))
    out["depth"] = float((dd[ok] / dscale).max(initial=0.0))
    out["n_marginal"] = int((~ok).sum())
    out["marginal_color_alpha"] = float(max(dc[:, ~ok].max(initial=0.0), da[~ok].max(initial=0.0)))
    return out


def assert_images_close(gpu, ref, mask=None):
    """Non-marginal pixels within the image tolerances. A marginal pixel has a decision (alpha
    at 1/255, the stop at T = 1e-4) that float32 and float64 may take differently; one flipped
    1/255 decision moves colour and opacity by at most about 1/255, so they are checked at a
    loose bound there. The marginal share grows with the alpha evaluations per pixel (about 0.3 %
    of the pixels at the 1M-Gaussian 1280x720 view, ~300 evaluations each); at most 0.5 % may be
    left out."""
    e = compare_images(gpu, ref, mask)
    assert e["color"] <= IMG_ATOL and e["alpha"] <= IMG_ATOL and e["t_final"] <= IMG_ATOL, e
    assert e["depth"] <= DEPTH_RTOL, e
    assert e["n_marginal"] <= max(16, MARGINAL_FRAC * ref["alpha"].size), e
    assert e["marginal_color_alpha"] <= MARGINAL_ATOL, e
    return e


ALL_GRADS = ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest", "pose")


def grad_errors(gpu, ref, keys=ALL_GRADS, rtol=GRAD_RTOL, atol=GRAD_ATOL, exclude=None):
    """Element-wise gradient comparison. For every element of a block,
        |g - r| <= rtol |r| + atol max|r over the block|
    (atol: the float32 summation floor for elements whose per-pixel terms cancel). Returns, per
    block, the largest ratio of |g - r| to that bound (<= 1 passes) with the worst element.
    exclude: bool [n], Gaussians left out of the per-Gaussian blocks (those the oracle flags as
    taking a marginal decision at some pixel); the pose block keeps every Gaussian."""
    out = {}
    for k in keys:
        a, b = np.asarray(gpu[k], np.float64), np.asarray(ref[k], np.float64)
        if b.size == 0:
            continue
        if exclude is not None and k != "pose" and np.any(exclude):
            keep = ~np.asarray(exclude, bool)
            a, b = a[..., keep], b[..., keep]
        a, b = a.ravel(), b.ravel()
        if b.size == 0:
            continue
        scale = float(np.abs(b).max())
        err = np.abs(a - b)
        bound = rtol * np.abs(b) + atol * scale
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
        i = int(np.argmax(ratio))
        out[k] = dict(ratio=float(ratio[i]), at=i, got=float(a[i]), ref=float(b[i]),
                      max_err_over_block_max=float(err.max() / scale) if scale > 0 else float(err.max()),
                      n=int(b.size))
    return out


def assert_grads_close(gpu, ref, rtol=GRAD_RTOL, keys=ALL_GRADS, atol=GRAD_ATOL, exclude=None):
    e = grad_errors(gpu, ref, keys, rtol=rtol, atol=atol, exclude=exclude)
    worst = {k: (round(v["ratio"], 3), v["at"], v["got"], v["ref"]) for k, v in e.items()}
    print(f"[grads] ratio to bound, element, gpu, oracle: {worst}", flush=True)
    bad = {k: v for k, v in e.items() if not v["ratio"] <= 1.0}
    assert not bad, bad
    return e


def marginal_gaussians(g, cam, tile=16):
    """Gaussians the float64 oracle sees taking a decision within 1e-4 of a threshold."""
    return oracle.marginal_gaussians(g, oracle_cam(cam), tile=tile, band=1e-4)
