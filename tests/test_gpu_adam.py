"""Sparse Adam (needs an MI355X): gs_adam_sparse against the float64 oracle over several steps,
with a ragged Gaussian count, two views of visibility and every parameter group; Gaussians no
view reached must stay bit for bit. Edge cases: nothing reached, everything reached (no
visibility list), SH degree 0 (an empty group) and a single Gaussian.

Tolerances from the arithmetic: a step changes a parameter by at most ~3 lr (the moment ratio
is bounded by (1 - b1) / sqrt(1 - b2)); the float32 kernel rounds the moments, the ratio and the
parameter once each per step, so after S steps a parameter is within ~S (ulp(p) + 1e-6 lr) of
the float64 oracle started from the same float32 values: rtol 2e-6 and atol 1e-6 cover S = 3.
Moments carry the gradient's float32 transform through exp / logistic (a few ulp): rtol 1e-5,
and where the first moment cancels, a few ulp of its terms (2e-6 of the group's largest).
"""
import numpy as np
import pytest
import torch

from oracle import adam as OA
from paper_2507_04004_amd import _native as N
from paper_2507_04004_amd.adam import SparseAdam
from paper_2507_04004_amd.raster import GaussianMap, ParamGrads

pytestmark = pytest.mark.gpu
DEV = "cuda"
F32 = lambda x: float(np.float32(x))
GROUPS = [("mean", OA.ACT_NONE), ("scale", OA.ACT_EXP), ("rot", OA.ACT_NONE), ("opacity", OA.ACT_SIGMOID),
          ("sh_dc", OA.ACT_NONE), ("sh_rest", OA.ACT_NONE)]


def _map(n, deg, seed):
    rng = np.random.default_rng(seed)
    k_rest = 3 * ((deg + 1) ** 2 - 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)
    return GaussianMap(t(rng.normal(0, 5, (3, n))), t(np.exp(rng.normal(-3, 0.5, (3, n)))),
                       t(rng.normal(size=(4, n))), t(rng.uniform(0.02, 0.98, (1, n))[0]),
                       t(rng.normal(0, 0.3, (3, n))), t(rng.normal(0, 0.1, (k_rest, n))), deg)


def _grads(gm, seed):
    rng = np.random.default_rng(seed)
    t = lambda x: torch.from_numpy(rng.normal(0, 1e-2, tuple(x.shape)).astype(np.float32)).to(DEV)
    return ParamGrads(t(gm.mean), t(gm.scale), t(gm.rot), t(gm.opacity), t(gm.sh_dc), t(gm.sh_rest),
                      torch.zeros(6, device=DEV))


def _oracle_state(opt):
    st = []
    for (raw, act_out, name, act, lr), m, v in zip(opt.groups, opt.exp_avg, opt.exp_avg_sq):
        st.append({"param": raw.double().cpu().numpy().reshape(-1, opt.gm.n),
                   "exp_avg": m.double().cpu().numpy().reshape(-1, opt.gm.n),
                   "exp_avg_sq": v.double().cpu().numpy().reshape(-1, opt.gm.n), "act": act, "lr": F32(lr),
                   "name": name})
    return st


def _run(n, deg, steps, vis_fn, seed=0):
    gm = _map(n, deg, seed)
    opt = SparseAdam(gm, lr={"mean": 1e-3, "scale": 5e-3, "rot": 1e-3, "opacity": 5e-2, "sh_dc": 2.5e-3,
                             "sh_rest": 1.25e-4})
    ref = _oracle_state(opt)
    init = [g["param"].copy() for g in ref]
    rng = np.random.default_rng(seed + 1)
    for s in range(1, steps + 1):
        counts = vis_fn(rng, n)
        grads = _grads(gm, seed + 10 * s)
        vis_t = None if counts is None else torch.from_numpy(counts.astype(np.int32)).to(DEV)
        opt.step(grads, vis_t)
        visible = np.ones(n, bool) if counts is None else OA.visible_mask(counts)
        for g, (_, _, name, _, _) in zip(ref, opt.groups):
            g["grad"] = getattr(grads, name).double().cpu().numpy().reshape(-1, n)
            # the float32 values the kernel receives, widened exactly
            g["act_value"] = OA.sparse_adam_step(g, visible, s, beta1=F32(0.9), beta2=F32(0.999), eps=F32(1e-15))
    torch.cuda.synchronize()
    return gm, opt, ref, init


def _compare(opt, ref, touched):
    for (raw, act_out, name, act, lr), m, v, g in zip(opt.groups, opt.exp_avg, opt.exp_avg_sq, ref):
        if raw.numel() == 0:
            continue
        n = opt.gm.n
        p = raw.double().cpu().numpy().reshape(-1, n)
        np.testing.assert_allclose(p, g["param"], rtol=2e-6, atol=1e-6, err_msg=name)
        # the first moment cancels where the gradient changes sign: its error is a few ulp of the
        # terms added, bounded through the largest moment of the group
        np.testing.assert_allclose(m.double().cpu().numpy().reshape(-1, n), g["exp_avg"], rtol=1e-5,
                                   atol=2e-6 * np.abs(g["exp_avg"]).max(), err_msg=name)
        np.testing.assert_allclose(v.double().cpu().numpy().reshape(-1, n), g["exp_avg_sq"], rtol=1e-5,
                                   atol=2e-6 * np.abs(g["exp_avg_sq"]).max(), err_msg=name)
        if act_out is not None and touched.any():
            a = act_out.double().cpu().numpy().reshape(-1, n)[:, touched]
            np.testing.assert_allclose(a, g["act_value"][:, touched], rtol=1e-5, err_msg=name)


def _two_views(rng, n):
    counts = np.zeros((2, n), np.uint32)
    counts[0, : n // 3] = rng.integers(0, 3, n // 3)          # a block of the map, partly culled
    idx = rng.choice(n, n // 5, replace=False)
    counts[1, idx] = 1 + rng.integers(0, 4, idx.size)          # scattered Gaussians
    return counts


def test_sparse_adam_matches_oracle_over_steps():
    n = 100_003
    print(f"[adam] n={n} deg=3 steps=3", flush=True)
    gm, opt, ref, init = _run(n, 3, 3, _two_views)
    rng = np.random.default_rng(1)
    touched = np.zeros(n, bool)
    for s in range(3):
        touched |= OA.visible_mask(_two_views(rng, n))
    assert 0.2 * n < touched.sum() < 0.8 * n
    _compare(opt, ref, touched)
    for (raw, _, name, _, _), p0 in zip(opt.groups, init):
        if raw.numel():
            p = raw.double().cpu().numpy().reshape(-1, n)
            assert np.array_equal(p[:, ~touched], p0[:, ~touched]), name  # never reached: bit for bit


def test_sparse_adam_edge_cases():
    # nothing reached: every plane unchanged, moments stay zero
    gm, opt, ref, init = _run(1000, 3, 2, lambda rng, n: np.zeros((1, n), np.uint32))
    for (raw, _, name, _, _), p0, m in zip(opt.groups, init, opt.exp_avg):
        assert np.array_equal(raw.double().cpu().numpy().reshape(-1, 1000), p0), name
        assert not m.any(), name
    # everything reached (no visibility list), SH degree 0 (empty group), ragged sizes, n = 1
    for n, deg in ((1, 0), (65, 0), (4097, 1)):
        print(f"[adam] all reached n={n} deg={deg}", flush=True)
        gm, opt, ref, init = _run(n, deg, 2, lambda rng, n: None, seed=n)
        _compare(opt, ref, np.ones(n, bool))
