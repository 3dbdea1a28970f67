"""Pins of the CPU oracle against facts fixed outside it (CPU only).

Each test names what it pins. None of them re-types the oracle's own formula: they use
closed forms of special cases, invariances, a library routine, brute force by an
independent implementation, or central finite differences on a frozen branch.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle.loss import loss_and_grads
from paper_2507_04004_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gauss(means, scales, quats, opac, dc, rest=None, deg=0):
    means = np.asarray(means, np.float64).reshape(-1, 3).T
    n = means.shape[1]
    k = (deg + 1) ** 2 - 1
    rest = np.zeros((3 * k, n)) if rest is None else np.asarray(rest, np.float64)
    return S.Gaussians(means.copy(), np.asarray(scales, np.float64).reshape(-1, 3).T.copy(),
                       np.asarray(quats, np.float64).reshape(-1, 4).T.copy(), np.asarray(opac, np.float64).copy(),
                       np.asarray(dc, np.float64).reshape(-1, 3).T.copy(), rest, deg)


def pinhole(W, H, f, R=None, t=None):
    return S.Camera(W, H, f, f, (W - 1) / 2, (H - 1) / 2, np.eye(3) if R is None else R,
                    np.zeros(3) if t is None else t)


def tiny_scene(seed, n=40, W=48, H=32, deg=0):
    rng = np.random.default_rng(seed)
    cam = S.Camera(W, H, 40.0, 42.0, (W - 1) / 2 + 0.3, (H - 1) / 2 - 0.2, np.eye(3), np.zeros(3))
    z = rng.uniform(2, 8, n)
    mean = np.stack([rng.uniform(-1, 1, n) * z * W / 2 / 40, rng.uniform(-1, 1, n) * z * H / 2 / 42, z])
    scale = np.exp(rng.uniform(-3, -0.5, (3, n)))
    q = rng.standard_normal((4, n))
    opac = 1 / (1 + np.exp(-rng.standard_normal(n) * 2))
    dc = rng.uniform(-1.5, 1.5, (3, n))
    k = (deg + 1) ** 2 - 1
    rest = rng.normal(0, 0.3, (3 * k, n))
    return S.Gaussians(mean, scale, q, opac, dc, rest, deg), cam


def rand_pose(rng, scale=0.3):
    from scipy.spatial.transform import Rotation
    R = Rotation.from_rotvec(rng.normal(0, scale, 3)).as_matrix()
    return R, rng.normal(0, scale, 3)


# --------------------------------------------------------------------------------------------
# P1: one isotropic Gaussian on the optical axis, identity pose: closed forms.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("o", [0.3, 0.8])
def test_single_gaussian_closed_form(o):
    f, z, s = 50.0, 4.0, 0.1
    cam = pinhole(33, 25, f)
    dc = 0.7
    g = gauss([0, 0, z], [s, s, s], [1, 0, 0, 0], [o], [dc, -0.4, 0.2])
    out = oracle.render(g, cam, tile=8, band=0.0)
    ys, xs = np.mgrid[0:cam.h, 0:cam.w]
    r2 = (xs - cam.cx) ** 2 + (ys - cam.cy) ** 2
    sig2 = (f * s / z) ** 2 + 0.3
    raw = o * np.exp(-r2 / (2 * sig2))
    alpha = np.where(raw >= 1 / 255, np.minimum(raw, 0.99), 0.0)
    y0 = 1 / (2 * math.sqrt(math.pi))
    col = np.maximum(np.array([dc, -0.4, 0.2]) * y0 + 0.5, 0)
    np.testing.assert_allclose(out["alpha"], alpha, atol=1e-13)
    np.testing.assert_allclose(out["depth"], z * alpha, atol=1e-12)
    np.testing.assert_allclose(out["t_final"], 1 - alpha, atol=1e-13)
    for ch in range(3):
        np.testing.assert_allclose(out["color"][ch], col[ch] * alpha, atol=1e-13)
    # gradients of L = sum gO * O: d/do, d/dz, and d/ds (sum over the two scale axes that project)
    rng = np.random.default_rng(1)
    gO = rng.standard_normal((cam.h, cam.w))
    gr = oracle.backward(g, cam, np.zeros((3, cam.h, cam.w)), None, gO, tile=8)
    live = (raw >= 1 / 255) & (raw < 0.99)
    e = np.exp(-r2 / (2 * sig2))
    np.testing.assert_allclose(gr["opacity"][0], (gO * e * live).sum(), rtol=1e-10)
    dalpha_dsig2 = raw * r2 / (2 * sig2 ** 2)
    dL_ds = (gO * dalpha_dsig2 * live).sum() * 2 * f ** 2 * s / z ** 2
    np.testing.assert_allclose(gr["scale"][0, 0] + gr["scale"][1, 0], dL_ds, rtol=1e-9)
    assert abs(gr["scale"][2, 0]) < 1e-12 * max(1, abs(dL_ds))
    dL_dz = (gO * dalpha_dsig2 * live).sum() * (-2 * f ** 2 * s ** 2 / z ** 3)
    np.testing.assert_allclose(gr["mean"][2, 0], dL_dz, rtol=1e-9)
    # colour: dL/dDC = sum gC * alpha * Y0
    gC = rng.standard_normal((3, cam.h, cam.w))
    gr2 = oracle.backward(g, cam, gC, None, None, tile=8)
    for ch in range(3):
        want = (gC[ch] * alpha).sum() * y0 if col[ch] > 0 else 0.0
        np.testing.assert_allclose(gr2["sh_dc"][ch, 0], want, rtol=1e-10, atol=1e-14)


# --------------------------------------------------------------------------------------------
# P2 / P3: Jacobian vs numeric derivative of the pinhole map; covariance spectrum; q == -q.
# --------------------------------------------------------------------------------------------
def test_projection_jacobian_and_covariance():
    rng = np.random.default_rng(3)
    cam = pinhole(64, 48, 55.0, *rand_pose(rng, 0.1))
    for trial in range(20):
        m = np.linalg.solve(cam.R_cw, np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 6)]) - cam.t_cw)
        s = np.exp(rng.uniform(-3, -1, 3))
        q = rng.standard_normal(4)
        g = gauss(m, s, q, [0.5], [0, 0, 0])
        p = oracle.project_one(g, cam, 0)
        mh = cam.R_cw @ m + cam.t_cw
        pix = lambda v: np.array([cam.fx * v[0] / v[2] + cam.cx, cam.fy * v[1] / v[2] + cam.cy])
        h = 1e-6
        Jfd = np.stack([(pix(mh + h * e) - pix(mh - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose([p["J00"], p["J02"], p["J11"], p["J12"]],
                                   [Jfd[0, 0], Jfd[0, 2], Jfd[1, 1], Jfd[1, 2]], rtol=1e-7)
        np.testing.assert_allclose([p["u"], p["v"]], pix(mh), rtol=1e-13)
        Sig = np.array([[p["S00"], p["S01"], p["S02"]], [p["S01"], p["S11"], p["S12"]], [p["S02"], p["S12"], p["S22"]]])
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(Sig)), np.sort(s ** 2), rtol=1e-10)
        p2 = oracle.project_one(gauss(m, s, -q * 2.5, [0.5], [0, 0, 0]), cam, 0)
        for key in ("s00", "s01", "s11", "a", "b", "c"):
            np.testing.assert_allclose(p2[key], p[key], rtol=1e-12)
        # isotropic scale: the covariance does not depend on the rotation
        g_iso1 = gauss(m, [0.1] * 3, q, [0.5], [0, 0, 0])
        g_iso2 = gauss(m, [0.1] * 3, rng.standard_normal(4), [0.5], [0, 0, 0])
        a1, a2 = oracle.project_one(g_iso1, cam, 0), oracle.project_one(g_iso2, cam, 0)
        np.testing.assert_allclose([a2["s00"], a2["s01"], a2["s11"]], [a1["s00"], a1["s01"], a1["s11"]],
                                   rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------------------------
# P5: spherical harmonics — orthonormal on the sphere and equal to the library definition.
# --------------------------------------------------------------------------------------------
def test_sh_orthonormal_quadrature():
    nt, nphi = 40, 80
    xg, wg = np.polynomial.legendre.leggauss(nt)  # cos(theta) nodes
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    Y = oracle.sh_basis(dirs, 3)
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-10)


def test_sh_matches_scipy_real_harmonics():
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(5)
    v = rng.standard_normal((50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(v[:, 2])
    phi = np.arctan2(v[:, 1], v[:, 0])
    Y = oracle.sh_basis(v, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            cplx = sph_harm_y(l, abs(m), theta, phi)  # includes the Condon-Shortley phase
            if m > 0:
                want = math.sqrt(2) * cplx.real
            elif m < 0:
                want = math.sqrt(2) * cplx.imag
            else:
                want = cplx.real
            np.testing.assert_allclose(Y[:, l * l + l + m], want, atol=1e-12, err_msg=f"l={l} m={m}")


# --------------------------------------------------------------------------------------------
# P6: worked examples of the alpha clamp, the 1/255 cutoff and the early stop.
# --------------------------------------------------------------------------------------------
def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_worked_examples_constants():
    ex = _golden("compositing_constants.json")
    cam = pinhole(9, 9, 30.0)
    # (a) opacity 1 at the centre pixel: alpha is clamped to its ceiling
    g = gauss([0, 0, 3], [0.05] * 3, [1, 0, 0, 0], [1.0], [0, 0, 0])
    out = oracle.render(g, cam, tile=8, band=0.0)
    assert out["alpha"][4, 4] == ex["alpha_max"]
    # (b) peak weights just below / above 1/255 at the centre pixel
    for factor, contributes in ex["cutoff_cases"]:
        g = gauss([0, 0, 3], [0.05] * 3, [1, 0, 0, 0], [factor / 255.0], [0, 0, 0])
        out = oracle.render(g, cam, tile=8, band=0.0)
        assert (out["alpha"][4, 4] > 0) == contributes
    # (c) a stack of co-centred Gaussians with alpha 0.95: exactly three blend
    st = ex["stack"]
    n = st["n_gaussians"]
    g = gauss([[0, 0, 3 + i] for i in range(n)], [[0.05] * 3] * n, [[1, 0, 0, 0]] * n, [st["alpha"]] * n,
              [[(st["colour"] - 0.5) * 2 * math.sqrt(math.pi)] * 3] * n)
    out = oracle.render(g, cam, tile=8, band=0.0)
    assert out["ncontrib"][4, 4] == st["n_blended"]
    np.testing.assert_allclose(out["t_final"][4, 4], st["t_final"], rtol=1e-12)
    np.testing.assert_allclose(out["alpha"][4, 4], 1 - st["t_final"], rtol=1e-12)
    np.testing.assert_allclose(out["color"][0, 4, 4], st["colour"] * (1 - st["t_final"]), rtol=1e-12)


# --------------------------------------------------------------------------------------------
# P7: transmittance invariants on random scenes.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transmittance_invariants(seed):
    g, cam = tiny_scene(seed, n=60, deg=1)
    out = oracle.render(g, cam, tile=8, band=0.0)
    T = out["t_final"]
    assert np.all(T >= 1e-4) and np.all(T <= 1.0)
    np.testing.assert_allclose(out["alpha"], 1 - T, atol=1e-12)
    has = out["alpha"] > 0
    proj = oracle.project(g, cam)
    dv = proj["depth"][proj["valid"] == 1]
    nd = out["depth"][has] / out["alpha"][has]
    assert np.all(nd >= dv.min() - 1e-9) and np.all(nd <= dv.max() + 1e-9)
    # T decreases strictly along each pixel's contributors (replay of the lists)
    fz = oracle.Frozen(g, cam, tile=8)
    assert np.all(fz.ncontrib[has.ravel()] >= 1)


# --------------------------------------------------------------------------------------------
# P8: tiled C oracle == independent NumPy brute force; P9: tile size / culling invariance.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,deg", [(0, 0), (1, 1), (2, 2), (3, 3)])
def test_tiled_equals_bruteforce(seed, deg):
    g, cam = tiny_scene(seed, n=50, deg=deg)
    if seed == 2:
        R, t = rand_pose(np.random.default_rng(seed), 0.05)
        cam = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R, t, bg=(0.2, 0.1, 0.3))
    if seed == 3:
        cam = cam.window(5, 3, 30, 21)
    ref = brute.render(g, cam)
    out = oracle.render(g, cam, tile=16, band=0.0)
    for key in ("color", "depth", "alpha", "t_final"):
        np.testing.assert_allclose(out[key], ref[key], atol=1e-12, err_msg=key)


def test_tile_size_and_cull_invariance():
    g, cam = tiny_scene(7, n=80, W=70, H=45, deg=2)
    base = oracle.render(g, cam, tile=16, cull=True, band=0.0)
    for tile, cull in [(8, True), (32, True), (16, False), ((8, 32), True), ((32, 8), False)]:
        out = oracle.render(g, cam, tile=tile, cull=cull, band=0.0)
        for key in ("color", "depth", "alpha", "t_final"):
            assert np.array_equal(out[key], base[key]), (tile, cull, key)


def test_render_pixels_equals_tiled():
    g, cam = tiny_scene(11, n=70, deg=3)
    out = oracle.render(g, cam, tile=16, band=0.0)
    ys, xs = np.mgrid[0:cam.h, 0:cam.w]
    px = oracle.render_pixels(g, cam, xs.ravel(), ys.ravel(), band=0.0)
    np.testing.assert_array_equal(px["color"].reshape(3, cam.h, cam.w), out["color"])
    np.testing.assert_array_equal(px["last_id"].reshape(cam.h, cam.w), out["last_id"])


def test_tile_cull_min_is_exact():
    """The facing-edge minimum equals a dense brute-force minimum over the rectangle."""
    rng = np.random.default_rng(9)
    for _ in range(300):
        A = rng.standard_normal((2, 2))
        Sg = A @ A.T + 0.05 * np.eye(2)
        Q = np.linalg.inv(Sg)
        u, v = rng.uniform(-20, 40, 2)
        xl, yl = rng.uniform(0, 15, 2)
        xh, yh = xl + rng.uniform(0, 15), yl + rng.uniform(0, 15)
        got = oracle.rect_qmin(u, v, Q[0, 0], Q[0, 1], Q[1, 1], xl, xh, yl, yh)
        X, Y = np.meshgrid(np.linspace(xl, xh, 301), np.linspace(yl, yh, 301))
        dx, dy = X - u, Y - v
        q = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
        assert got <= q.min() + 1e-9
        # grid spacing bounds how far above the true minimum the grid can be
        step = max((xh - xl), (yh - yl)) / 300
        assert q.min() - got <= 2 * np.linalg.norm(Q) * (np.hypot(xh - u, yh - v) + np.hypot(xl - u, yl - v) + 1) * step + 1e-9


# --------------------------------------------------------------------------------------------
# P11 / P13: analytic backward == central finite differences on the frozen branch.
# --------------------------------------------------------------------------------------------
def _functional(out, gC, gD, gO):
    return (gC * out["color"]).sum() + (gD * out["depth"]).sum() + (gO * out["alpha"]).sum()


def _perturb(g, field, comp, k, h):
    g2 = S.Gaussians(*(np.array(a, np.float64, copy=True) for a in
                       (g.mean, g.scale, g.rot, g.opacity, g.sh_dc, g.sh_rest)), g.sh_degree)
    arr = getattr(g2, field)
    if arr.ndim == 1:
        arr[k] += h
    else:
        arr[comp, k] += h
    return g2


def _se3_exp(xi):
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-12:
        R, V = np.eye(3) + K, np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K
        V = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * K @ K
    return R, V @ rho


def _cam_left(cam, xi):
    dR, dt = _se3_exp(xi)
    return S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, dR @ cam.R_cw, dR @ cam.t_cw + dt,
                    cam.x0, cam.y0, cam.w, cam.h, cam.bg)


@pytest.mark.parametrize("which", ["all", "rgb", "depth", "opacity"])
@pytest.mark.parametrize("seed", [21, 22])
def test_backward_matches_frozen_fd(which, seed):
    g, cam = tiny_scene(seed, n=30, W=40, H=30, deg=3)
    R, t = rand_pose(np.random.default_rng(seed), 0.05)
    cam = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R, t, bg=(0.1, 0.2, 0.3))
    rng = np.random.default_rng(seed + 100)
    gC = rng.standard_normal((3, cam.h, cam.w)) * (which in ("all", "rgb"))
    gD = rng.standard_normal((cam.h, cam.w)) * (which in ("all", "depth"))
    gO = rng.standard_normal((cam.h, cam.w)) * (which in ("all", "opacity"))
    an = oracle.backward(g, cam, gC, gD, gO, tile=8)
    fz = oracle.Frozen(g, cam, tile=8)
    f0 = _functional(oracle.replay(g, cam, fz), gC, gD, gO)
    np.testing.assert_allclose(f0, _functional(fz.base, gC, gD, gO), rtol=1e-12)
    h = 1e-6
    proj = oracle.project(g, cam)
    live = np.nonzero(np.abs(an["grad2d"]).sum(0) > 0)[0]
    assert live.size >= 5
    checks = []
    for k in live[:6]:
        for field, ncomp in (("mean", 3), ("scale", 3), ("rot", 4), ("opacity", 1), ("sh_dc", 3), ("sh_rest", 45)):
            comps = range(ncomp) if ncomp <= 4 else rng.choice(ncomp, 4, replace=False)
            for comp in comps:
                fp = _functional(oracle.replay(_perturb(g, field, comp, k, h), cam, fz), gC, gD, gO)
                fm = _functional(oracle.replay(_perturb(g, field, comp, k, -h), cam, fz), gC, gD, gO)
                got = an[field][k] if field == "opacity" else an[field][comp, k]
                checks.append((field, (fp - fm) / (2 * h), got))
    for i in range(6):
        xi = np.zeros(6)
        xi[i] = h
        fp = _functional(oracle.replay(g, _cam_left(cam, xi), fz), gC, gD, gO)
        fm = _functional(oracle.replay(g, _cam_left(cam, -xi), fz), gC, gD, gO)
        checks.append(("pose", (fp - fm) / (2 * h), an["pose"][i]))
    scale = {f: max(abs(c[2]) for c in checks if c[0] == f) for f in set(c[0] for c in checks)}
    for field, fd, got in checks:
        assert abs(fd - got) <= 1e-6 * max(abs(got), 1e-3 * scale[field]) + 2e-8, (field, fd, got)
    assert proj["valid"].sum() > 0


def test_pose_translation_identity():
    """d L / d rho == R sum_k d L / d mu_k exactly (translating the camera moves every mean)."""
    g, cam = tiny_scene(31, n=60, deg=3)
    R, t = rand_pose(np.random.default_rng(31), 0.2)
    cam = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R, t)
    rng = np.random.default_rng(32)
    an = oracle.backward(g, cam, rng.standard_normal((3, cam.h, cam.w)), rng.standard_normal((cam.h, cam.w)),
                         rng.standard_normal((cam.h, cam.w)))
    np.testing.assert_allclose(an["pose"][:3], R @ an["mean"].sum(1), rtol=1e-10, atol=1e-12)


def test_rigid_motion_equivariance():
    """Moving world and camera together leaves images and the camera-frame pose gradient unchanged."""
    from scipy.spatial.transform import Rotation
    g, cam = tiny_scene(41, n=60, deg=0)
    rng = np.random.default_rng(41)
    Rg = Rotation.from_rotvec(rng.normal(0, 0.5, 3))
    tg = rng.normal(0, 2, 3)
    mean2 = Rg.as_matrix() @ g.mean + tg[:, None]
    qg = Rg.as_quat()  # (x, y, z, w)
    rot2 = np.empty_like(g.rot)
    for k in range(g.n):
        qk = Rotation.from_quat(np.r_[g.rot[1:, k], g.rot[0, k]])
        xyzw = (Rg * qk).as_quat()
        rot2[:, k] = np.r_[xyzw[3], xyzw[:3]]
    g2 = S.Gaussians(mean2, g.scale, rot2, g.opacity, g.sh_dc, g.sh_rest, 0)
    Rc = cam.R_cw @ Rg.as_matrix().T
    cam2 = S.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, Rc, cam.t_cw - Rc @ tg)
    a, b = oracle.render(g, cam, band=0.0), oracle.render(g2, cam2, band=0.0)
    for key in ("color", "depth", "alpha"):
        np.testing.assert_allclose(b[key], a[key], atol=1e-10)
    gC = rng.standard_normal((3, cam.h, cam.w))
    ga, gb = oracle.backward(g, cam, gC), oracle.backward(g2, cam2, gC)
    np.testing.assert_allclose(gb["pose"], ga["pose"], rtol=1e-7, atol=1e-9)
    assert qg.shape == (4,)


def test_loss_gradient_matches_fd():
    rng = np.random.default_rng(51)
    h, w = 6, 7
    C = rng.uniform(0, 1, (3, h, w))
    T = rng.uniform(0, 1, (3, h, w))
    D = rng.uniform(1, 5, (h, w))
    O = rng.uniform(0.2, 1, (h, w))
    O[0, 0] = 0.0
    pix = np.array([0, 3, 10, 20, 33])
    ds = rng.uniform(1, 6, pix.size)
    L1, Ld, gC, gD, gO = loss_and_grads(C, D, O, T, pix, ds, gamma=0.7)
    eps = 1e-7
    for arr, grad in ((C, gC), (D, gD), (O, gO)):
        for idx in [np.unravel_index(i, arr.shape) for i in rng.choice(arr.size, 8, replace=False)] + \
                   ([np.unravel_index(p, arr.shape) for p in pix[1:]] if arr.ndim == 2 else []):
            a1 = arr.copy(); a1[idx] += eps
            a2 = arr.copy(); a2[idx] -= eps
            args = {id(C): (a1, D, O), id(D): (C, a1, O), id(O): (C, D, a1)}[id(arr)]
            args2 = {id(C): (a2, D, O), id(D): (C, a2, O), id(O): (C, D, a2)}[id(arr)]
            fp = sum(loss_and_grads(*args, T, pix, ds, 0.7)[:2])
            fm = sum(loss_and_grads(*args2, T, pix, ds, 0.7)[:2])
            np.testing.assert_allclose((fp - fm) / (2 * eps), grad[idx], atol=1e-6)
    assert Ld > 0 and L1 > 0
