"""NumPy FP64 brute-force renderer — TEST INFRASTRUCTURE ONLY, tiny scenes.

A second, independent writing of the forward definition (Sec. "3D Gaussian Splatting
Representation": the projection, eq:alpha and eq:rendered_rgb / _depth / _opacity) with no
tiles and no culling: every pixel composites every Gaussian whose weight reaches 1/255, in
ascending (float32 depth, index) order. It uses matrix algebra where the C oracle writes loops
out, so an error in one is unlikely to repeat in the other. Sized for <= ~100 Gaussians
and a few thousand pixels.
"""
from __future__ import annotations

import math

import numpy as np


def _quat_to_rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    # rotation of the unit quaternion via its action on basis vectors (Hamilton product)
    def rotate(vec):
        qv = np.array([x, y, z])
        t = 2.0 * np.cross(qv, vec)
        return vec + w * t + np.cross(qv, t)
    return np.stack([rotate(e) for e in np.eye(3)], axis=1)


def _sh_values(d, deg):
    x, y, z = d
    s = math.sqrt
    pi = math.pi
    vals = [1 / (2 * s(pi))]
    if deg >= 1:
        c = s(3 / (4 * pi))
        vals += [-c * y, c * z, -c * x]
    if deg >= 2:
        vals += [s(15 / pi) / 2 * x * y, -s(15 / pi) / 2 * y * z, s(5 / pi) / 4 * (3 * z * z - 1),
                 -s(15 / pi) / 2 * x * z, s(15 / pi) / 4 * (x * x - y * y)]
    if deg >= 3:
        vals += [-s(35 / (2 * pi)) / 4 * y * (3 * x * x - y * y), s(105 / pi) / 2 * x * y * z,
                 -s(21 / (2 * pi)) / 4 * y * (5 * z * z - 1), s(7 / pi) / 4 * (5 * z ** 3 - 3 * z),
                 -s(21 / (2 * pi)) / 4 * x * (5 * z * z - 1), s(105 / pi) / 4 * z * (x * x - y * y),
                 -s(35 / (2 * pi)) / 4 * x * (x * x - 3 * y * y)]
    return np.array(vals)


def splat(g, cam):
    """List of dicts, one per Gaussian that survives the validity tests."""
    R, t = np.asarray(cam.R_cw, float), np.asarray(cam.t_cw, float)
    centre = -R.T @ t
    out = []
    for k in range(g.n):
        mu = g.mean[:, k].astype(float)
        mh = R @ mu + t
        d = mh[2]
        if not d > 0.2:
            continue
        Rq = _quat_to_rot(g.rot[:, k].astype(float))
        Sig = Rq @ np.diag(g.scale[:, k].astype(float) ** 2) @ Rq.T
        lx, ly = 1.3 * cam.width / (2 * cam.fx), 1.3 * cam.height / (2 * cam.fy)
        tx, ty = np.clip(mh[0] / d, -lx, lx), np.clip(mh[1] / d, -ly, ly)
        J = np.array([[cam.fx / d, 0, -cam.fx * tx / d], [0, cam.fy / d, -cam.fy * ty / d]])
        S2 = J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2)
        if np.linalg.det(S2) <= 0:
            continue
        o = float(g.opacity[k])
        if o < 1 / 255:
            continue
        view = (mu - centre) / np.linalg.norm(mu - centre)
        Y = _sh_values(view, g.sh_degree)
        coef = np.concatenate([g.sh_dc[:, k][None, :].astype(float),
                               g.sh_rest[:, k].astype(float).reshape(-1, 3)], axis=0) if Y.size > 1 else \
            g.sh_dc[:, k][None, :].astype(float)
        rgb = np.maximum(Y @ coef + 0.5, 0.0)
        # order key (R12): the depth in float32, ((R6 mx + R7 my) + R8 mz) + tz with every
        # operation rounded to float32; the index breaks its ties
        f = np.float32
        m32 = g.mean[:, k].astype(f)
        r32, t32 = np.asarray(cam.R_cw, f), np.asarray(cam.t_cw, f)
        dkey = f(f(f(r32[2, 0] * m32[0]) + f(r32[2, 1] * m32[1])) + f(r32[2, 2] * m32[2])) + t32[2]
        out.append(dict(k=k, d=d, dkey=float(dkey), mu2=np.array([cam.fx * mh[0] / d + cam.cx, cam.fy * mh[1] / d + cam.cy]),
                        Q=np.linalg.inv(S2), o=o, rgb=rgb))
    out.sort(key=lambda s: (s["dkey"], s["k"]))
    return out


def render(g, cam):
    """Window-sized colour [3][h][w], depth, opacity and final transmittance."""
    spl = splat(g, cam)
    h, w = cam.h, cam.w
    C = np.zeros((3, h, w))
    D = np.zeros((h, w))
    O = np.zeros((h, w))
    Tf = np.zeros((h, w))
    for j in range(h):
        for i in range(w):
            rho = np.array([cam.x0 + i, cam.y0 + j], float)
            T, c, dd, oo = 1.0, np.zeros(3), 0.0, 0.0
            for s in spl:
                delta = rho - s["mu2"]
                alpha = min(0.99, s["o"] * math.exp(min(0.0, -0.5 * delta @ s["Q"] @ delta)))
                if alpha < 1 / 255:
                    continue
                if T * (1 - alpha) < 1e-4:
                    break
                c += alpha * T * s["rgb"]
                dd += alpha * T * s["d"]
                oo += alpha * T
                T *= 1 - alpha
            C[:, j, i] = c + T * np.asarray(cam.bg, float)
            D[j, i], O[j, i], Tf[j, i] = dd, oo, T
    return dict(color=C, depth=D, alpha=O, t_final=Tf)
