"""Pins of the FP64 D-SSIM oracle (no GPU): identical images, the closed form for constant
images away from the border, central differences of the gradient, the window's separability
and the symmetry of SSIM."""
import numpy as np
import torch

from oracle import ssim as O


def test_identical_images_give_zero_and_zero_gradient():
    x = np.random.default_rng(0).uniform(size=(3, 20, 23))
    loss, g = O.dssim(x, x, weight=0.7)
    assert abs(loss) < 1e-15
    assert np.abs(g).max() < 1e-12


def test_constant_images_closed_form():
    # away from the border the window sees only the constants: no variance, so
    # SSIM = (2 a b + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.8
    x = torch.full((1, 24, 24), a, dtype=torch.float64)
    y = torch.full((1, 24, 24), b, dtype=torch.float64)
    s = O.ssim_map(x, y)[0, 5:-5, 5:-5]
    expect = (2 * a * b + O.C1) / (a * a + b * b + O.C1)
    assert torch.allclose(s, torch.full_like(s, expect), rtol=0, atol=1e-12)


def test_gradient_against_central_differences():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(2, 14, 17))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    _, g = O.dssim(x, y, weight=0.5)
    h = 1e-6
    for c, i, j in [(0, 0, 0), (1, 7, 8), (0, 13, 16), (1, 3, 12), (0, 10, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (O.dssim(xp, y, 0.5)[0] - O.dssim(xm, y, 0.5)[0]) / (2 * h)
        assert abs(fd - g[c, i, j]) <= 1e-7 * max(1.0, abs(g[c, i, j])), (c, i, j, fd, g[c, i, j])


def test_window_is_normalised_and_separable():
    w = O.window2d()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    r = np.arange(11) - 5
    g1 = np.exp(-r ** 2 / (2 * O.SIGMA ** 2))
    g1 /= g1.sum()
    assert np.abs(np.outer(g1, g1) - w).max() < 1e-16


def test_ssim_is_symmetric():
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.uniform(size=(3, 16, 16)))
    y = torch.tensor(rng.uniform(size=(3, 16, 16)))
    assert torch.allclose(O.ssim_map(x, y), O.ssim_map(y, x), rtol=0, atol=1e-15)
