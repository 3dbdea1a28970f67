"""Map initialization and expansion — TEST INFRASTRUCTURE ONLY.

Sec. "Initialization of Gaussian Map": every colourised point becomes a Gaussian at its 3D
location with its colour in the zeroth SH degree, opacity 0.1, identity rotation and scale
S = (d / f) (1, 1, 1), d the point's depth in the keyframe's camera frame and f the focal
length. Sec. "Expansion of Gaussian Map": for a later keyframe, the opacity O is rendered
(eq:rendered_opacity), the mask O < tau (tau = 0.99) marks newly observed regions, and only
the points that project into the mask initialise Gaussians.

Readings (the paper leaves them open):
  - a point's pixel is the nearest pixel centre (centres at integer coordinates) of its
    pinhole projection (fx x/z + cx, fy y/z + cy); a point behind the renderer's near plane
    (z <= 0.2) or outside the render window is not selected;
  - f is fx;
  - the colour's zeroth-degree coefficient is (rgb - 1/2) / Y_0, Y_0 = 1 / (2 sqrt(pi)), so the
    rendered colour of the new Gaussian seen alone is its point colour; higher degrees are 0;
  - the new Gaussians follow the existing ones, in the points' order;
  - initialization (no opacity map) selects every point in front of the near plane.
The selection is an integer decision taken from floating point: it is computed in float32
with the kernel's operation order (rotation row times point, left to right, plus translation;
x / z; fx times that plus cx; floor of u + 1/2), and the comparison O < tau in float32. The
new Gaussians' values are computed in float64.
"""
from __future__ import annotations

import numpy as np

NEAR = 0.2
Y0 = 0.28209479177387814  # 1 / (2 sqrt(pi))
OPACITY0 = 0.1


def project_f32(xyz, cam):
    """float32 camera-frame point and pixel of each point: (x, y, z) [3][n], (ix, iy) int64."""
    f = np.float32
    R = np.asarray(cam.R_cw, np.float32).reshape(3, 3)
    t = np.asarray(cam.t_cw, np.float32)
    P = np.asarray(xyz, np.float32)
    cam_pts = []
    for i in range(3):
        a = R[i, 0] * P[0]
        a = a + R[i, 1] * P[1]
        a = a + R[i, 2] * P[2]
        cam_pts.append(a + t[i])
    x, y, z = cam_pts
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = f(cam.fx) * (x / z) + f(cam.cx)
        v = f(cam.fy) * (y / z) + f(cam.cy)
        ix = np.floor(u + f(0.5))
        iy = np.floor(v + f(0.5))
    return (x, y, z), ix, iy


def select(xyz, cam, opacity=None, tau=0.99):
    """Boolean mask of the points that initialise Gaussians (opacity: [h][w] window plane)."""
    P = np.asarray(xyz, np.float32)
    (x, y, z), ix, iy = project_f32(P, cam)
    ok = np.isfinite(P).all(0) & (z > np.float32(NEAR))
    if opacity is None:
        return ok
    O = np.asarray(opacity, np.float32)
    inside = ok & (ix >= cam.x0) & (ix < cam.x0 + cam.w) & (iy >= cam.y0) & (iy < cam.y0 + cam.h)
    sel = np.zeros(P.shape[1], bool)
    idx = np.nonzero(inside)[0]
    px = (iy[idx] - cam.y0).astype(np.int64) * cam.w + (ix[idx] - cam.x0).astype(np.int64)
    sel[idx] = O.ravel()[px] < np.float32(tau)
    return sel


def new_gaussians(xyz, rgb, cam, sel, sh_degree=3):
    """The Gaussians initialised from the selected points, in point order (float64 values)."""
    P = np.asarray(xyz, np.float32)[:, sel].astype(np.float64)
    C = np.asarray(rgb, np.float32)[:, sel].astype(np.float64)
    R = np.asarray(cam.R_cw, np.float32).reshape(3, 3).astype(np.float64)
    t = np.asarray(cam.t_cw, np.float32).astype(np.float64)
    d = (R @ P + t[:, None])[2]
    m = P.shape[1]
    s = d / float(np.float32(cam.fx))
    k = 3 * ((sh_degree + 1) ** 2 - 1)
    return dict(mean=P, scale=np.stack([s, s, s]), rot=np.r_[np.ones((1, m)), np.zeros((3, m))],
                opacity=np.full(m, OPACITY0), sh_dc=(C - 0.5) / Y0, sh_rest=np.zeros((k, m)))


def expand(old, xyz, rgb, cam, opacity=None, tau=0.99):
    """old: dict of planes (or None); returns the grown map's planes and the selection mask."""
    deg = 3 if old is None else old["sh_degree"]
    sel = select(xyz, cam, opacity, tau)
    new = new_gaussians(xyz, rgb, cam, sel, deg)
    if old is None:
        out = new
    else:
        out = {k: np.concatenate([np.asarray(old[k], np.float64).reshape(new[k].shape[:-1] + (-1,)), new[k]], -1)
               for k in new}
    out["sh_degree"] = deg
    return out, sel
