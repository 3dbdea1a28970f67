"""Seeded synthetic inputs for the rasterizer: Gaussian maps, cameras and LiDAR masks.

This module only draws random numbers and lays them out; it holds none of the
renderer's arithmetic (no projection, covariance, SH evaluation or compositing).
Both the HIP path and the CPU oracle are fed from the arrays it returns, so the two
never share a code path beyond their inputs.

Parameter layout follows the 3D Gaussian representation of the paper (Sec. "3D
Gaussian Splatting Representation"): position mu, linear scale S > 0, rotation as a
unit quaternion (w, x, y, z), activated opacity o in (0, 1) and SH coefficients split
into the DC plane and the higher-order planes ("separated SH", Sec. "CUDA-Related
Acceleration Strategies", b). All per-Gaussian arrays are SoA float32 planes of shape
(components, N).

Camera convention: a pinhole with pixel centres at integer coordinates, world axes
x right, y down, z forward; the ground sits at y = +1.6 m below a camera at y = 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Real SH basis value of degree 0. Used only to turn a plain RGB colour into its DC
# coefficient when drawing inputs (colour u maps to DC = (u - 0.5) / Y0).
_Y0 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    """World-to-camera pose (R_cw, t_cw) with pinhole intrinsics and a render window."""

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R_cw: np.ndarray  # (3, 3) float64
    t_cw: np.ndarray  # (3,) float64
    x0: int = 0
    y0: int = 0
    w: int | None = None
    h: int | None = None
    bg: tuple = (0.0, 0.0, 0.0)

    def __post_init__(self):
        if self.w is None:
            self.w = self.width - self.x0
        if self.h is None:
            self.h = self.height - self.y0
        self.R_cw = np.asarray(self.R_cw, dtype=np.float64).reshape(3, 3)
        self.t_cw = np.asarray(self.t_cw, dtype=np.float64).reshape(3)

    def window(self, x0: int, y0: int, w: int, h: int) -> "Camera":
        return dataclasses.replace(self, x0=x0, y0=y0, w=w, h=h)

    @property
    def n_pixels(self) -> int:
        return int(self.w) * int(self.h)


@dataclasses.dataclass
class Gaussians:
    """SoA float32 planes; sh_rest holds plane 3*(k-1)+channel for basis k >= 1."""

    mean: np.ndarray      # (3, N)
    scale: np.ndarray     # (3, N) linear, > 0
    rot: np.ndarray       # (4, N) quaternion (w, x, y, z)
    opacity: np.ndarray   # (N,)
    sh_dc: np.ndarray     # (3, N)
    sh_rest: np.ndarray   # (3*((deg+1)^2-1), N)
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(self.mean[:, idx].copy(), self.scale[:, idx].copy(), self.rot[:, idx].copy(),
                         self.opacity[idx].copy(), self.sh_dc[:, idx].copy(), self.sh_rest[:, idx].copy(),
                         self.sh_degree)

    def astype(self, dtype) -> "Gaussians":
        return Gaussians(*(np.ascontiguousarray(a, dtype=dtype) for a in
                           (self.mean, self.scale, self.rot, self.opacity, self.sh_dc, self.sh_rest)),
                         self.sh_degree)


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def look_camera(position, yaw_deg: float, pitch_deg: float, width: int, height: int,
                fx: float, fy: float | None = None) -> Camera:
    """A centred pinhole at `position` (world), turned by yaw about y, then pitch about x."""
    fy = fx if fy is None else fy
    ya, pa = math.radians(yaw_deg), math.radians(pitch_deg)
    Ry = np.array([[math.cos(ya), 0.0, math.sin(ya)], [0.0, 1.0, 0.0], [-math.sin(ya), 0.0, math.cos(ya)]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, math.cos(pa), -math.sin(pa)], [0.0, math.sin(pa), math.cos(pa)]])
    R_wc = Ry @ Rx
    R_cw = R_wc.T
    t_cw = -R_cw @ np.asarray(position, dtype=np.float64)
    return Camera(width, height, fx, fy, (width - 1) / 2.0, (height - 1) / 2.0, R_cw, t_cw)


def _shape_params(rng, n: int, sh_degree: int, colours: np.ndarray, rest_sigma: float = 0.2):
    log_s = rng.uniform(-4.0, -1.0, size=(3, n))
    q = rng.standard_normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-rng.standard_normal(size=n)))
    sh_dc = (colours - 0.5) / _Y0
    k = (sh_degree + 1) ** 2 - 1
    sh_rest = rng.normal(0.0, rest_sigma, size=(3 * k, n)) if k else np.zeros((0, n))
    return np.exp(log_s), q, opacity, sh_dc, sh_rest


def _pack(mean, scale, rot, opacity, sh_dc, sh_rest, deg) -> Gaussians:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Gaussians(f(mean), f(scale), f(rot), f(opacity), f(sh_dc), f(sh_rest), deg)


def frustum_scene(n: int, cam: Camera, z_range=(2.0, 20.0), sh_degree: int = 0, seed: int = 0) -> Gaussians:
    """Means uniform in the camera's frustum box at depth z_range (identity pose assumed)."""
    rng = _rng(seed)
    d = rng.uniform(z_range[0], z_range[1], size=n)
    x = rng.uniform(-1.0, 1.0, size=n) * d * (cam.width / 2.0) / cam.fx
    y = rng.uniform(-1.0, 1.0, size=n) * d * (cam.height / 2.0) / cam.fy
    mean = np.stack([x, y, d])
    colours = rng.uniform(0.0, 1.0, size=(3, n))
    return _pack(mean, *_shape_params(rng, n, sh_degree, colours), sh_degree)


def _box_faces(rng, n: int, boxes) -> np.ndarray:
    """n points uniform over the four vertical faces of axis-aligned boxes (area-weighted)."""
    areas = []
    for (cx, cz, wx, wz, hgt) in boxes:
        areas += [wx * hgt, wx * hgt, wz * hgt, wz * hgt]
    areas = np.asarray(areas)
    face = rng.choice(len(areas), size=n, p=areas / areas.sum())
    pts = np.empty((3, n))
    b = face // 4
    f = face % 4
    bx = np.asarray(boxes)[b]
    cx, cz, wx, wz, hgt = bx.T
    s = rng.uniform(-0.5, 0.5, size=n)
    y = 1.6 - rng.uniform(0.0, 1.0, size=n) * hgt
    x = np.where(f < 2, cx + s * wx, cx + np.where(f == 2, -0.5, 0.5) * wx)
    z = np.where(f < 2, cz + np.where(f == 0, -0.5, 0.5) * wz, cz + s * wz)
    pts[0], pts[1], pts[2] = x, y, z
    return pts + rng.normal(0.0, 0.02, size=pts.shape)


def street_scene(n: int, seed: int, z_range=(1.0, 60.0), x_half: float = 25.0, n_boxes: int = 12,
                 frac=(0.7, 0.3, 0.0), n_clusters: int = 200, sh_degree: int = 3) -> Gaussians:
    """Outdoor-like map: noisy ground plane, box facades, optional vegetation clusters."""
    rng = _rng(seed)
    n_ground = int(round(n * frac[0]))
    n_fac = int(round(n * frac[1]))
    n_veg = n - n_ground - n_fac
    zlo, zhi = z_range
    ground = np.stack([rng.uniform(-x_half, x_half, n_ground),
                       1.6 + rng.normal(0.0, 0.03, n_ground),
                       rng.uniform(zlo, zhi, n_ground)])
    boxes = []
    for i in range(n_boxes):
        side = -1.0 if i % 2 == 0 else 1.0
        boxes.append((side * rng.uniform(6.0, 20.0), rng.uniform(zlo + 4.0, zhi - 5.0),
                      rng.uniform(3.0, 10.0), rng.uniform(3.0, 10.0), rng.uniform(3.0, 15.0)))
    facades = _box_faces(rng, n_fac, boxes)
    parts = [ground, facades]
    if n_veg > 0:
        centres = np.stack([np.where(rng.uniform(size=n_clusters) < 0.5, -1.0, 1.0) * rng.uniform(4.0, 25.0, n_clusters),
                            1.6 - rng.uniform(1.0, 5.0, n_clusters),
                            rng.uniform(zlo, zhi, n_clusters)])
        which = rng.integers(0, n_clusters, size=n_veg)
        parts.append(centres[:, which] + rng.normal(0.0, 1.0, size=(3, n_veg)))
    mean = np.concatenate(parts, axis=1)
    perm = rng.permutation(n)
    mean = mean[:, perm]
    colours = rng.uniform(0.0, 1.0, size=(3, n))
    return _pack(mean, *_shape_params(rng, n, sh_degree, colours), sh_degree)


def perturb(g: Gaussians, sigma: float, seed: int) -> Gaussians:
    """Copy with N(0, sigma^2) noise on mean, log-scale, quaternion (renormalised), logit-opacity, SH."""
    rng = _rng(seed)
    mean = g.mean + rng.normal(0.0, sigma, g.mean.shape)
    scale = np.exp(np.log(g.scale.astype(np.float64)) + rng.normal(0.0, sigma, g.scale.shape))
    rot = g.rot + rng.normal(0.0, sigma, g.rot.shape)
    rot /= np.linalg.norm(rot, axis=0, keepdims=True)
    o = np.clip(g.opacity.astype(np.float64), 1e-6, 1 - 1e-6)
    logit = np.log(o / (1.0 - o)) + rng.normal(0.0, sigma, o.shape)
    opacity = 1.0 / (1.0 + np.exp(-logit))
    sh_dc = g.sh_dc + rng.normal(0.0, sigma, g.sh_dc.shape)
    sh_rest = g.sh_rest + rng.normal(0.0, sigma, g.sh_rest.shape)
    return _pack(mean, scale, rot, opacity, sh_dc, sh_rest, g.sh_degree)


def lidar_rows(cam: Camera, n_rows: int = 16, keep: float = 0.18, seed: int = 0) -> np.ndarray:
    """Scan-row mask: rows floor((r + 1/2) H / n_rows), pixels kept with probability `keep`.

    Returns ascending linear pixel indices inside the render window.
    """
    rng = _rng(seed)
    rows = np.floor((np.arange(n_rows) + 0.5) * cam.height / n_rows).astype(np.int64)
    xs = np.arange(cam.width)
    pix = []
    for r in rows:
        keepmask = rng.uniform(size=cam.width) < keep
        for x in xs[keepmask]:
            if cam.x0 <= x < cam.x0 + cam.w and cam.y0 <= r < cam.y0 + cam.h:
                pix.append((r - cam.y0) * cam.w + (x - cam.x0))
    return np.unique(np.asarray(pix, dtype=np.int32))


def lidar_beams(cam: Camera, n_beams: int = 32, fov_deg: float = 30.0, keep: float = 0.32, seed: int = 0) -> np.ndarray:
    """Spinning-LiDAR-like mask: one curved image row per beam elevation, columns kept with `keep`."""
    rng = _rng(seed)
    i = np.arange(cam.width, dtype=np.float64)
    pix = []
    for b in range(n_beams):
        e = math.radians(-fov_deg / 2 + fov_deg * b / (n_beams - 1))
        v = np.rint(cam.cy + cam.fy * math.tan(e) * np.sqrt(1.0 + ((i - cam.cx) / cam.fx) ** 2)).astype(np.int64)
        keepmask = rng.uniform(size=cam.width) < keep
        ok = keepmask & (v >= cam.y0) & (v < cam.y0 + cam.h) & (i >= cam.x0) & (i < cam.x0 + cam.w)
        pix.append((v[ok] - cam.y0) * cam.w + (i[ok].astype(np.int64) - cam.x0))
    pix = np.concatenate(pix) if pix else np.zeros(0, np.int64)
    return np.unique(pix).astype(np.int32)


# ---------------------------------------------------------------------------------------------
# Named workloads. Sizes follow the single-view, batched, tracking and serving workloads the
# rasterizer is measured on; every draw is seeded.
# ---------------------------------------------------------------------------------------------

def config_small(seed: int = 0):
    """128x96 pinhole (fx = fy = 100), 2,000 Gaussians in a frustum box at z in [2, 20], SH degree 0."""
    cam = Camera(128, 96, 100.0, 100.0, 63.5, 47.5, np.eye(3), np.zeros(3))
    g = frustum_scene(2000, cam, (2.0, 20.0), sh_degree=0, seed=seed)
    pix = lidar_rows(cam, 16, 0.18, seed=seed + 100)
    return g, cam, pix


def config_street_view(seed: int = 1, n: int = 100_000):
    """640x512, fx = fy = 450 camera at the origin over a ground + facade street of n Gaussians, SH 3."""
    cam = Camera(640, 512, 450.0, 450.0, 319.5, 255.5, np.eye(3), np.zeros(3))
    g = street_scene(n, seed, z_range=(1.0, 60.0), x_half=25.0, n_boxes=12, frac=(0.7, 0.3, 0.0), sh_degree=3)
    pix = lidar_beams(cam, 32, 30.0, 0.32, seed=seed + 100)
    return g, cam, pix


def street_map(n: int = 1_000_000, seed: int = 2, z_range=(-20.0, 220.0), n_boxes: int = 60,
               n_clusters: int = 200) -> Gaussians:
    """Outdoor street map: 50 % ground (|x| < 30), 30 % facades, 20 % vegetation clusters, SH 3."""
    return street_scene(n, seed, z_range=z_range, x_half=30.0, n_boxes=n_boxes, frac=(0.5, 0.3, 0.2),
                        n_clusters=n_clusters, sh_degree=3)


def headline_camera(width: int = 1280, height: int = 720, fx: float = 900.0) -> Camera:
    """1280x720, fx = fy = 900, at z = 10 m on the street axis looking down the street."""
    return look_camera((0.0, 0.0, 10.0), 0.0, 0.0, width, height, fx)


def keyframe_cameras(n_views: int = 8, seed: int = 2):
    """Keyframes along the street with uneven intrinsics (fx in [400, 1100]) and resolutions."""
    rng = _rng(seed + 1000)
    res = [(640, 480), (800, 600), (960, 540), (1024, 768), (1280, 720)]
    cams = []
    for k in range(n_views):
        W, H = res[int(rng.integers(0, len(res)))]
        fx = float(rng.uniform(400.0, 1100.0))
        pos = (float(rng.uniform(-3.0, 3.0)), 0.0, 10.0 + 20.0 * k + float(rng.uniform(-5.0, 5.0)))
        cams.append(look_camera(pos, float(rng.uniform(-20.0, 20.0)), float(rng.uniform(-5.0, 5.0)), W, H, fx))
    return cams


def serving_requests(n_requests: int, seed: int = 4, z_max: float = 1000.0):
    """Mixed-resolution novel views along a 1 km street: 640x360 / 1280x720 / 1920x1080 at 50/35/15 %."""
    rng = _rng(seed + 2000)
    res = [(640, 360), (1280, 720), (1920, 1080)]
    cams = []
    for _ in range(n_requests):
        W, H = res[int(rng.choice(3, p=[0.5, 0.35, 0.15]))]
        pos = (float(rng.uniform(-3.0, 3.0)), 0.0, float(rng.uniform(0.0, z_max)))
        cams.append(look_camera(pos, float(rng.uniform(-30.0, 30.0)), float(rng.uniform(-5.0, 5.0)), W, H, 0.8 * W))
    return cams


def upstream_grads(n_pixels: int, seed: int, channels: int = 3):
    """Random upstream gradients (dL/dC, dL/dD, dL/dO) for checking a backward pass."""
    rng = _rng(seed)
    gc = rng.standard_normal((channels, n_pixels)).astype(np.float32)
    gd = rng.standard_normal(n_pixels).astype(np.float32)
    go = rng.standard_normal(n_pixels).astype(np.float32)
    return gc, gd, go
