"""Pins of the FP64 sparse Adam oracle (no GPU): closed forms of the first steps, untouched
Gaussians outside the visible set, the all-visible case against torch's Adam, and the
activation chain rule against central differences."""
import math

import numpy as np
import torch

from oracle import adam as A


def _group(n, k=3, act=A.ACT_NONE, lr=1e-2, seed=0):
    rng = np.random.default_rng(seed)
    return {"param": rng.normal(size=(k, n)), "exp_avg": np.zeros((k, n)), "exp_avg_sq": np.zeros((k, n)),
            "grad": rng.normal(size=(k, n)), "act": act, "lr": lr}


def test_first_step_closed_form():
    # from zero moments the bias-corrected ratio is g / |g|: every element moves by lr against sign(g)
    g = _group(50)
    p0, grad = g["param"].copy(), g["grad"].copy()
    A.sparse_adam_step(g, np.ones(50, bool), step=1, eps=1e-15)
    np.testing.assert_allclose(g["param"], p0 - 1e-2 * grad / (np.abs(grad) + 1e-15), rtol=0, atol=1e-15)
    np.testing.assert_allclose(g["exp_avg"], 0.1 * grad, rtol=1e-15)
    np.testing.assert_allclose(g["exp_avg_sq"], 1e-3 * grad * grad, rtol=1e-12)


def test_shared_step_counter_closed_form():
    # a Gaussian first reached at step 2 starts from zero moments but is corrected with t = 2:
    # m^ = g / (1 + b1), v^ = g^2 / (1 + b2), so it moves by lr sqrt(1 + b2) / (1 + b1) against sign(g)
    g = _group(40, seed=1)
    vis1 = np.zeros(40, bool)
    vis1[:20] = True
    A.sparse_adam_step(g, vis1, step=1)
    p1 = g["param"].copy()
    assert np.array_equal(g["exp_avg"][:, 20:], np.zeros((3, 20)))
    A.sparse_adam_step(g, np.ones(40, bool), step=2)
    late = slice(20, 40)
    expect = p1[:, late] - 1e-2 * math.sqrt(1.999) / 1.9 * np.sign(g["grad"][:, late])
    np.testing.assert_allclose(g["param"][:, late], expect, rtol=0, atol=1e-13)


def test_invisible_gaussians_untouched():
    g = _group(64, seed=2)
    g["exp_avg"][:] = 0.3
    g["exp_avg_sq"][:] = 0.7
    before = {k: g[k].copy() for k in ("param", "exp_avg", "exp_avg_sq")}
    n_tiles = np.zeros((2, 64), np.uint32)
    n_tiles[0, ::3] = 4
    n_tiles[1, 1::5] = 1
    vis = A.visible_mask(n_tiles)
    assert vis.sum() == len(set(range(0, 64, 3)) | set(range(1, 64, 5)))
    A.sparse_adam_step(g, vis, step=3)
    for k, b in before.items():
        assert np.array_equal(g[k][:, ~vis], b[:, ~vis]), k
        assert not np.any(g[k][:, vis] == b[:, vis]), k


def test_all_visible_equals_torch_adam():
    n, steps = 33, 5
    g = _group(n, k=4, lr=3e-3, seed=3)
    p = torch.tensor(g["param"].copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-15)
    rng = np.random.default_rng(4)
    for t in range(1, steps + 1):
        grad = rng.normal(size=(4, n))
        g["grad"] = grad
        A.sparse_adam_step(g, np.ones(n, bool), step=t)
        p.grad = torch.tensor(grad)
        opt.step()
    np.testing.assert_allclose(g["param"], p.detach().numpy(), rtol=0, atol=1e-13)


def test_activation_chain_rule_against_central_differences():
    rng = np.random.default_rng(5)
    raw = rng.normal(size=(2, 7))
    up = rng.normal(size=(2, 7))  # gradient w.r.t. the activated value
    h = 1e-6
    for act in (A.ACT_EXP, A.ACT_SIGMOID):
        fd = (A.activate(raw + h, act) - A.activate(raw - h, act)) / (2 * h) * up
        np.testing.assert_allclose(A.raw_grad(raw, up, act), fd, rtol=1e-8, atol=1e-12)
    assert np.array_equal(A.raw_grad(raw, up, A.ACT_NONE), up)
    # the activated values the renderer reads: exp and the logistic function
    assert abs(A.activate(np.array([0.0]), A.ACT_SIGMOID)[0] - 0.5) < 1e-16
    assert abs(A.activate(np.array([math.log(2.0)]), A.ACT_EXP)[0] - 2.0) < 1e-15
