"""Map initialization and expansion (Sec. "Initialization of Gaussian Map", Sec. "Expansion of
Gaussian Map"): binding of gs_expand_select / gs_expand_write.

A keyframe's colourised points initialise new Gaussians where the map does not yet cover the
image: the rendered opacity at the point's pixel is below tau (0.99 in the paper's setup). With
no opacity map (the first keyframe) every point in front of the camera is used. The grown map
keeps the existing Gaussians first and adds the new ones in point order; the selection count is
read back once (one synchronisation) to size it.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from . import raster as R


def expand_map(gm: R.GaussianMap | None, xyz: torch.Tensor, rgb: torch.Tensor, cam,
               opacity: torch.Tensor | None = None, tau: float = 0.99, sh_degree: int = 3,
               device="cuda") -> tuple[R.GaussianMap, int]:
    """Returns (grown map, number of Gaussians added). xyz, rgb: [3, n] float32 on the device;
    cam: scenes.Camera-like or gs_camera; opacity: [h, w] window plane or None."""
    cs = cam if isinstance(cam, N.Camera) else R.camera_struct(cam)
    xyz, rgb = xyz.contiguous(), rgb.contiguous()
    n = int(xyz.shape[1])
    pts = N.Points(n, R._p(xyz), R._p(rgb))
    scratch = torch.empty(N.lib().gs_expand_scratch_bytes(n), dtype=torch.uint8, device=device)
    count = torch.zeros(1, dtype=torch.int64, device=device)
    st = R._stream()
    N.check(N.lib().gs_expand_select(C.byref(pts), C.byref(cs), R._p(opacity), float(tau), R._p(count), R._p(scratch),
                                     scratch.numel(), st), "gs_expand_select")
    added = int(count.item())
    deg = gm.sh_degree if gm is not None else sh_degree
    n_old = gm.n if gm is not None else 0
    m = n_old + added
    k = 3 * ((deg + 1) ** 2 - 1)
    e = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=device)
    new = R.GaussianMap(e(3, m), e(3, m), e(4, m), e(m), e(3, m), e(k, m), deg)
    out = N.GaussiansOut(m, deg, R._p(new.mean), R._p(new.scale), R._p(new.rot), R._p(new.opacity), R._p(new.sh_dc),
                         R._p(new.sh_rest) if k else None)
    old = gm.struct() if gm is not None else None
    N.check(N.lib().gs_expand_write(C.byref(pts), C.byref(cs), C.byref(old) if old is not None else None, added,
                                    R._p(scratch), scratch.numel(), C.byref(out), st), "gs_expand_write")
    return new, added
