"""CPU oracle for the Gaussian-splatting rasterizer — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package. It wraps the FP64 C oracle (gs_oracle.c), the FP32 binning oracle (bins32.c) and
the NumPy brute force (brute.py). Nothing here imports or calls the HIP library.

Arrays cross the boundary as float64 (the oracle's precision) or float32 (binning). Input
parameters are taken as the float32 values the GPU receives and widened exactly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OrCamera(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32),
                ("w", C.c_int32), ("h", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("bg", C.c_double * 3)]


class OrGaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("deg", C.c_int32)] + [
        (k, C.POINTER(C.c_double)) for k in ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")]


class B32Camera(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32),
                ("w", C.c_int32), ("h", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3)]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GS_ORACLE_LIB") or _build.LIB  # the sanitizer test's instrumented build
        if not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        d = C.POINTER(C.c_double)
        i32 = C.POINTER(C.c_int32)
        i64 = C.POINTER(C.c_int64)
        u8 = C.POINTER(C.c_uint8)
        i8 = C.POINTER(C.c_int8)
        u32 = C.POINTER(C.c_uint32)
        f = C.POINTER(C.c_float)
        G, Cm = C.POINTER(OrGaussians), C.POINTER(OrCamera)
        _lib.or_render.argtypes = [G, Cm, C.c_int, C.c_int, C.c_int, C.c_double, d, d, d, d, i32, i64, u8]
        _lib.or_render_pixels.argtypes = [G, Cm, C.c_int64, i32, i32, C.c_double, d, d, d, d, i32, i64, u8]
        _lib.or_contributors.argtypes = [G, Cm, C.c_int, C.c_int, i64, i32, i8]
        _lib.or_replay.argtypes = [G, Cm, i64, i32, i8, i32, d, d, d]
        _lib.or_backward.argtypes = [G, Cm, C.c_int, C.c_int, d, d, d, d, d, d, d, d, d, d, d]
        _lib.or_project.argtypes = [G, Cm, i32, d, d, d, d, d, d, i32]
        _lib.or_project_one.argtypes = [G, Cm, C.c_int64, d]
        _lib.or_sh_basis.argtypes = [C.c_int64, d, C.c_int, d]
        _lib.or_rect_qmin.argtypes = [C.c_double] * 9
        _lib.or_rect_qmin.restype = C.c_double
        _lib.or_lists.argtypes = [G, Cm, C.c_int, C.c_int, i64, i32]
        _lib.or_pair_margins.argtypes = [G, Cm, C.c_int, C.c_int, C.c_int64, i32, i32, i8, d]
        _lib.or_marginal_gaussians.argtypes = [G, Cm, C.c_int, C.c_int, C.c_double, u8]
        _lib.or_set_threads.argtypes = [C.c_int]
        _lib.or_max_threads.restype = C.c_int
        bind_bin32(_lib)
    return _lib


def bind_bin32(handle):
    """Argument types of or32_bin on a loaded library (the oracle's, or a test's own build)."""
    f, i32, i64, u32 = (C.POINTER(t) for t in (C.c_float, C.c_int32, C.c_int64, C.c_uint32))
    handle.or32_bin.argtypes = [C.c_int64, f, f, f, f, C.POINTER(B32Camera), C.c_int, C.c_int, C.c_uint32,
                                C.c_uint32, u32, i32, u32, C.c_int64, u32, u32, u32, i64]
    return handle


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _Keep:
    """Holds the float64 copies alive while the C structs point at them."""

    def __init__(self, g):
        self.arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in
                       (g.mean, g.scale, g.rot, g.opacity, g.sh_dc,
                        g.sh_rest if g.sh_rest.size else np.zeros(1))]
        self.struct = OrGaussians(g.n, g.sh_degree, *[_p(a, C.c_double) for a in self.arrays])


def _cam(cam):
    return OrCamera(cam.width, cam.height, cam.x0, cam.y0, cam.w, cam.h, float(cam.fx), float(cam.fy),
                    float(cam.cx), float(cam.cy), (C.c_double * 9)(*np.asarray(cam.R_cw, np.float64).ravel()),
                    (C.c_double * 3)(*np.asarray(cam.t_cw, np.float64)), (C.c_double * 3)(*cam.bg))


def camera_f32(cam):
    """The float32 camera values the GPU receives, widened back to float64 for the oracle."""
    import dataclasses
    return dataclasses.replace(cam, fx=float(np.float32(cam.fx)), fy=float(np.float32(cam.fy)),
                               cx=float(np.float32(cam.cx)), cy=float(np.float32(cam.cy)),
                               R_cw=np.asarray(cam.R_cw, np.float32).astype(np.float64),
                               t_cw=np.asarray(cam.t_cw, np.float32).astype(np.float64),
                               bg=tuple(float(np.float32(b)) for b in cam.bg))


def render(g, cam, tile=16, cull=True, band=1e-4):
    """FP64 tiled render of the window. Returns dict of planes (window-sized)."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    npx = cam.w * cam.h
    out = dict(color=np.zeros((3, cam.h, cam.w)), depth=np.zeros((cam.h, cam.w)), alpha=np.zeros((cam.h, cam.w)),
               t_final=np.zeros((cam.h, cam.w)), last_id=np.zeros((cam.h, cam.w), np.int32),
               ncontrib=np.zeros((cam.h, cam.w), np.int64), marginal=np.zeros((cam.h, cam.w), np.uint8))
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    rc = L.or_render(C.byref(k.struct), C.byref(cs), tw, th, int(cull), band,
                     _p(out["color"], C.c_double), _p(out["depth"], C.c_double), _p(out["alpha"], C.c_double),
                     _p(out["t_final"], C.c_double), _p(out["last_id"], C.c_int32), _p(out["ncontrib"], C.c_int64),
                     _p(out["marginal"], C.c_uint8))
    assert rc == 0 and npx >= 0
    return out


def render_pixels(g, cam, xs, ys, band=1e-4):
    """Brute-force FP64 values at listed full-image pixel coordinates (no tiles)."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    m = xs.size
    out = dict(color=np.zeros((3, m)), depth=np.zeros(m), alpha=np.zeros(m), t_final=np.zeros(m),
               last_id=np.zeros(m, np.int32), ncontrib=np.zeros(m, np.int64), marginal=np.zeros(m, np.uint8))
    L.or_render_pixels(C.byref(k.struct), C.byref(cs), m, _p(xs, C.c_int32), _p(ys, C.c_int32), band,
                       _p(out["color"], C.c_double), _p(out["depth"], C.c_double), _p(out["alpha"], C.c_double),
                       _p(out["t_final"], C.c_double), _p(out["last_id"], C.c_int32), _p(out["ncontrib"], C.c_int64),
                       _p(out["marginal"], C.c_uint8))
    return out


def project(g, cam):
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    n = g.n
    out = dict(valid=np.zeros(n, np.int32), uv=np.zeros((2, n)), depth=np.zeros(n), conic=np.zeros((3, n)),
               kappa2=np.zeros(n), rgb=np.zeros((3, n)), ext=np.zeros((2, n)), frozen=np.zeros((3, n), np.int32))
    L.or_project(C.byref(k.struct), C.byref(cs), _p(out["valid"], C.c_int32), _p(out["uv"], C.c_double),
                 _p(out["depth"], C.c_double), _p(out["conic"], C.c_double), _p(out["kappa2"], C.c_double),
                 _p(out["rgb"], C.c_double), _p(out["ext"], C.c_double), _p(out["frozen"], C.c_int32))
    return out


def project_one(g, cam, k):
    L = lib()
    kk = _Keep(g)
    cs = _cam(cam)
    out = np.zeros(32)
    L.or_project_one(C.byref(kk.struct), C.byref(cs), int(k), _p(out, C.c_double))
    names = ["valid", "mx", "my", "mz", "u", "v", "s00", "s01", "s11", "a", "b", "c", "kappa2", "hx", "hy", "r", "g",
             "b_", "J00", "J02", "J11", "J12", "S00", "S01", "S02", "S11", "S12", "S22", "clx", "cly", "dist", "o"]
    return dict(zip(names, out))


def sh_basis(dirs, deg=3):
    L = lib()
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], 16))
    L.or_sh_basis(dirs.shape[0], _p(dirs, C.c_double), deg, _p(out, C.c_double))
    return out


def rect_qmin(u, v, a, b, c, xl, xh, yl, yh):
    return lib().or_rect_qmin(u, v, a, b, c, xl, xh, yl, yh)


def backward(g, cam, gC, gD=None, gO=None, tile=16):
    """Gradients of sum(gC*C) + sum(gD*D) + sum(gO*O) w.r.t. parameters and the pose tangent."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    n = g.n
    gC = np.ascontiguousarray(gC, np.float64).reshape(3, cam.h, cam.w)
    gD = None if gD is None else np.ascontiguousarray(gD, np.float64)
    gO = None if gO is None else np.ascontiguousarray(gO, np.float64)
    out = dict(grad2d=np.zeros((10, n)), mean=np.zeros((3, n)), scale=np.zeros((3, n)), rot=np.zeros((4, n)),
               opacity=np.zeros(n), sh_dc=np.zeros((3, n)), sh_rest=np.zeros(g.sh_rest.shape), pose=np.zeros(6))
    rest = out["sh_rest"] if out["sh_rest"].size else np.zeros(1)
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    null = C.POINTER(C.c_double)()
    L.or_backward(C.byref(k.struct), C.byref(cs), tw, th, _p(gC, C.c_double),
                  _p(gD, C.c_double) if gD is not None else null, _p(gO, C.c_double) if gO is not None else null,
                  _p(out["grad2d"], C.c_double), _p(out["mean"], C.c_double), _p(out["scale"], C.c_double),
                  _p(out["rot"], C.c_double), _p(out["opacity"], C.c_double), _p(out["sh_dc"], C.c_double),
                  _p(rest, C.c_double), _p(out["pose"], C.c_double))
    return out


class Frozen:
    """Branch decisions at a base point: contributor lists, alpha clamps, J and SH clamps."""

    def __init__(self, g, cam, tile=16):
        L = lib()
        k = _Keep(g)
        cs = _cam(cam)
        base = render(g, cam, tile=tile, band=0.0)
        self.ncontrib = base["ncontrib"].ravel()
        self.offsets = np.zeros(self.ncontrib.size + 1, np.int64)
        np.cumsum(self.ncontrib, out=self.offsets[1:])
        tot = int(self.offsets[-1])
        self.ids = np.zeros(max(tot, 1), np.int32)
        self.clamped = np.zeros(max(tot, 1), np.int8)
        tw, th = (tile, tile) if np.isscalar(tile) else tile
        L.or_contributors(C.byref(k.struct), C.byref(cs), tw, th, _p(self.offsets, C.c_int64),
                          _p(self.ids, C.c_int32), _p(self.clamped, C.c_int8))
        self.frozen = project(g, cam)["frozen"].copy()
        self.base = base


def replay(g, cam, fz: Frozen):
    """Smooth forward on the frozen branch (for central finite differences)."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    out = dict(color=np.zeros((3, cam.h, cam.w)), depth=np.zeros((cam.h, cam.w)), alpha=np.zeros((cam.h, cam.w)))
    L.or_replay(C.byref(k.struct), C.byref(cs), _p(fz.offsets, C.c_int64), _p(fz.ids, C.c_int32),
                _p(fz.clamped, C.c_int8), _p(fz.frozen, C.c_int32), _p(out["color"], C.c_double),
                _p(out["depth"], C.c_double), _p(out["alpha"], C.c_double))
    return out


def bin32(g, cam, tile=16, tile_base=0, id_base=0, handle=None):
    """FP32 binning: per-Gaussian tile counts, rects, depth keys; sorted pair ids and tile ranges.
    handle: a library exporting or32_bin (bound with bind_bin32); the oracle's own by default."""
    L = lib() if handle is None else handle
    n = g.n
    f = lambda a: np.ascontiguousarray(a, np.float32)
    mean, scale, rot, opac = f(g.mean), f(g.scale), f(g.rot), f(g.opacity)
    bc = B32Camera(cam.width, cam.height, cam.x0, cam.y0, cam.w, cam.h, float(cam.fx), float(cam.fy),
                   float(cam.cx), float(cam.cy), (C.c_float * 9)(*np.asarray(cam.R_cw, np.float32).ravel()),
                   (C.c_float * 3)(*np.asarray(cam.t_cw, np.float32)))
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    T = ((cam.w + tw - 1) // tw) * ((cam.h + th - 1) // th)
    n_tiles = np.zeros(n, np.uint32)
    rect = np.zeros((n, 4), np.int32)
    dkey = np.zeros(n, np.uint32)
    num = np.zeros(1, np.int64)
    tr = np.zeros(2 * T, np.uint32)
    cap = 0  # first call only counts; the second fills the sized arrays
    L.or32_bin(n, _p(mean, C.c_float), _p(scale, C.c_float), _p(rot, C.c_float), _p(opac, C.c_float), C.byref(bc),
               tw, th, tile_base, id_base, _p(n_tiles, C.c_uint32), _p(rect, C.c_int32), _p(dkey, C.c_uint32), cap,
               _p(np.zeros(1, np.uint32), C.c_uint32), None, _p(tr, C.c_uint32), _p(num, C.c_int64))
    P = int(num[0])
    vals = np.zeros(max(P, 1), np.uint32)
    tiles = np.zeros(max(P, 1), np.uint32)
    L.or32_bin(n, _p(mean, C.c_float), _p(scale, C.c_float), _p(rot, C.c_float), _p(opac, C.c_float), C.byref(bc),
               tw, th, tile_base, id_base, _p(n_tiles, C.c_uint32), _p(rect, C.c_int32), _p(dkey, C.c_uint32), P,
               _p(vals, C.c_uint32), _p(tiles, C.c_uint32), _p(tr, C.c_uint32), _p(num, C.c_int64))
    return dict(n_tiles=n_tiles, rect=rect, dkey=dkey, vals=vals[:P], tiles=tiles[:P], tile_range=tr, num_pairs=P)


def lists(g, cam, tile=16):
    """FP64 tile lists (no marginal band): start [T+1] and ids, each tile in (depth, id) order."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    T = ((cam.w + tw - 1) // tw) * ((cam.h + th - 1) // th)
    start = np.zeros(T + 1, np.int64)
    assert L.or_lists(C.byref(k.struct), C.byref(cs), tw, th, _p(start, C.c_int64), None) == 0
    ids = np.zeros(max(int(start[-1]), 1), np.int32)
    assert L.or_lists(C.byref(k.struct), C.byref(cs), tw, th, _p(start, C.c_int64), _p(ids, C.c_int32)) == 0
    return dict(start=start, ids=ids[:int(start[-1])])


def pair_margins(g, cam, gid, tile_ids, tile=16):
    """FP64 decision and relative margin of each queried (Gaussian, window tile) pair."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    gid = np.ascontiguousarray(gid, np.int32)
    tid = np.ascontiguousarray(tile_ids, np.int32)
    listed = np.zeros(gid.size, np.int8)
    margin = np.zeros(gid.size)
    L.or_pair_margins(C.byref(k.struct), C.byref(cs), tw, th, gid.size, _p(gid, C.c_int32), _p(tid, C.c_int32),
                      _p(listed, C.c_int8), _p(margin, C.c_double))
    return listed.astype(bool), margin


def marginal_gaussians(g, cam, tile=16, band=1e-4):
    """Bool [n]: Gaussians taking a decision within the relative band of a threshold (1/255,
    0.99, or the 1e-4 stop) at some pixel of the window."""
    L = lib()
    k = _Keep(g)
    cs = _cam(cam)
    tw, th = (tile, tile) if np.isscalar(tile) else tile
    flag = np.zeros(max(g.n, 1), np.uint8)
    assert L.or_marginal_gaussians(C.byref(k.struct), C.byref(cs), tw, th, band, _p(flag, C.c_uint8)) == 0
    return flag[:g.n].astype(bool)


def set_threads(n: int) -> int:
    """Sets the oracle's OpenMP thread count; returns the previous one."""
    L = lib()
    prev = L.or_max_threads()
    L.or_set_threads(int(n))
    return prev
