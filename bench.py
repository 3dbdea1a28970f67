#!/usr/bin/env python3
"""Headline benchmark: fwd+bwd views/s and render Mpix/s at 1280x720 with a 1M-Gaussian map.

Workload: a seeded synthetic street map of 1,000,000 Gaussians (50 % ground plane, 30 % box
facades, 20 % vegetation clusters; SH degree 3; float32) viewed by one 1280x720 pinhole
(fx = fy = 900) 10 m down the street, with a 32-beam LiDAR mask (~2 % of pixels). Targets
come from a copy of the map perturbed by N(0, 0.01^2) noise, rendered once by the same GPU
path before timing.

One step = the whole hot path on one view with inputs resident in HBM: projection + SH (a1),
binning with the alpha-max cull and the (tile, depth) sort (a2), compositing (a3) with the
sparse-LiDAR depth term (a6), the RGB L1 loss, and the backward to every parameter and the
pose (a4, a5). The backward writes every gradient element (overwrite mode), so the step needs
no clearing pass.

Besides the headline figure the line carries the roofline of the dominant kernel, the two
small configurations, the batched 8-keyframe pass, the sparse Adam step over the reached
Gaussians (`sparse_adam`), map expansion at the headline keyframe (`expansion`), the
photometric tracking loop on a 2M-Gaussian map (`tracking`), novel-view serving, and the
float64 CPU oracle as a baseline.

Prints ONE JSON line. `value` is fwd+bwd views/s on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X's published fp32 vector peak (256 CUs x 2.4 GHz, counting two-wide packed fp32
# instructions), the roofline's peak. The ceiling of single-issue fp32 FMAs, 256 CUs x 64 lanes x
# 2 flops x 2.4 GHz = 78.6 TFLOP/s, is reported beside it: this build compiles with packed fp32
# instructions turned off.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
# Algorithmic work per unit: bytes for the memory-bound stages (N Gaussians, V visible, P
# pairs, T tiles); flops per alpha evaluation for compositing. The backward count is 80 flops
# per evaluation E_b (E_b = sum over pixels of last + 1): the derivative of one alpha-blended
# Gaussian at one pixel (transmittance rebuilt by division, colour / depth / opacity terms, the
# conic, centre and opacity terms). The forward count is 28 flops per evaluation E_f.
BYTES_PRE_PER_N, BYTES_PRE_PER_V = 44 + 64 + 8, 192
BYTES_BIN_PER_N, BYTES_BIN_PER_V, BYTES_BIN_PER_P, BYTES_BIN_PER_T = 4, 64, 4, 8
BYTES_PREBWD_PER_N, BYTES_PREBWD_PER_V = 12 + 44 + 236 + 8, 192 + 48
FLOPS_FWD_EVAL = 28
FLOPS_BWD_EVAL = 80
# the tighter count of the operations each evaluation and contribution cannot avoid (14 per
# evaluation: offset, quadratic, exponent, clamp, compare; 57 more per contribution), reported
# as a second figure
FLOPS_MIN_EVAL, FLOPS_MIN_FWD_CONTRIB, FLOPS_MIN_BWD_CONTRIB = 14, 13, 57


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the HIP sources; counter readings are valid only for the sources they came from."""
    import hashlib
    d = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2507_04004_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(src, name), "rb") as fh:
                d.update(name.encode() + b"\0" + fh.read())
    return d.hexdigest()


def measured_traffic(kernel: str, tile: int, bd: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter readings (FETCH_SIZE
    and WRITE_SIZE, each scaled by what the counter reads for a plain copy of known size), or
    None when the readings are missing or were taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != kernel_source_digest():
        return None
    k = rec.get("kernels", {}).get(f"{kernel}/{tile}x{tile}/{bd}")
    return None if k is None else int(k["bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--tile", type=int, default=8)
    ap.add_argument("--blend-depth", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=5, help="oracle views timed for the CPU baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the 8-keyframe batched measurement")
    ap.add_argument("--no-small", action="store_true", help="skip the two small single-view configurations")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-adam", action="store_true", help="skip the sparse Adam measurement")
    ap.add_argument("--no-tracking", action="store_true", help="skip the photometric tracking measurement")
    ap.add_argument("--no-expansion", action="store_true", help="skip the map expansion measurement")
    ap.add_argument("--no-autograd", action="store_true", help="skip timing the autograd function (GSRender)")
    ap.add_argument("--no-c4", action="store_true", help="skip the 2M-Gaussian differentiation measurement")
    ap.add_argument("--tracking-only", action="store_true",
                    help="run only the photometric tracking measurement (for profiling it alone)")
    ap.add_argument("--tracking-frames", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (reference point for HBM byte counters)")
    return ap.parse_args()


def lidar_targets(frame, pix):
    """LiDAR depths D/O of a rendered target at the mask pixels (hits with O = 0 dropped)."""
    D = frame.depth.flatten().cpu().numpy()
    O = frame.alpha.flatten().cpu().numpy()
    keep = O[pix] > 0
    pix = pix[keep].astype(np.int32)
    return pix, (D[pix] / O[pix]).astype(np.float32)


def timed(torch, fn, reps, warmup):
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev)


def measure_small_configs(R, N, torch, S, tile, bd, dev, reps=50):
    """The two plain single-view configurations beside the headline view: 2,000 Gaussians at
    128x96 (SH 0, 16-row LiDAR mask) and 100k Gaussians at 640x512 (SH 3, 32-beam mask), each
    one full fwd + L1/LiDAR loss + bwd step with inputs resident."""
    from paper_2507_04004_amd.step import PlainStep
    out = {}
    for name, (g, cam, pix) in (("small_2k_128x96", S.config_small(0)), ("street_100k_640x512", S.config_street_view(1))):
        gp = S.perturb(g, 0.01, seed=3)
        tgt = PlainStep(R.GaussianMap.from_numpy(gp, dev), cam, pix,
                        torch.zeros(3, cam.h, cam.w, device=dev), np.zeros(pix.size, np.float32), tile, bd, dev)
        tgt.forward()
        torch.cuda.synchronize()
        target = tgt.frame.color.clone()
        hits, ds = lidar_targets(tgt.frame, pix)
        del tgt
        st = PlainStep(R.GaussianMap.from_numpy(g, dev), cam, hits, target, ds, tile, bd, dev)
        ms = timed(torch, st.step, reps, 5)
        out[name] = {"gaussians": int(g.n), "pixels": int(cam.w * cam.h), "ms_per_step": round(ms, 4),
                     "views_s": round(1e3 / ms, 1)}
        del st
    return out


def measure_batched(R, N, torch, S, g, gm, tile, bd, dev, reps=20):
    """8 keyframes of the same map (uneven intrinsics and resolutions) per optimisation pass:
    one graph-captured fwd+bwd batch (tile size and chunk length from the autotuner) against 8
    sequential plain fwd+bwd calls on the same stream."""
    from paper_2507_04004_amd.autotune import SCHEDULE_NAMES, autotune_config
    from paper_2507_04004_amd.batch import BatchPlan, ViewSlot
    from paper_2507_04004_amd.step import PlainStep
    cams = S.keyframe_cameras(8, seed=2)
    total_px = sum(c.w * c.h for c in cams)
    gp = R.GaussianMap.from_numpy(S.perturb(g, 0.01, seed=3), dev)
    # targets and LiDAR depths from the perturbed map (untimed)
    cap = 8 << 20
    while True:
        tplan = BatchPlan(gm.n, gm.sh_degree, 8, total_px, tile, bd, cap, dev)
        tslots = [ViewSlot.make(c, dev) for c in cams]
        tplan.run(gp, tslots, fwd=True)
        need = tplan.num_pairs()
        tplan.close()
        if need <= cap:
            break
        cap = int(need * 1.25)
    del gp
    cap = int(need * 1.25) + 4096
    targets = [s.frame.color.clone() for s in tslots]
    lidars = []
    for k, (c, sl) in enumerate(zip(cams, tslots)):
        pix, ds = lidar_targets(sl.frame, S.lidar_beams(c, 32, 30.0, 0.32, seed=200 + k))
        lidars.append((pix, ds))
    del tslots
    # the autotuner's whole search: nine tile shapes x chunk lengths 32-256, and the bucketed
    # backward at 8x8 and 16x16
    tuned = autotune_config(gm, cams, backward=True, capacity=cap, reps=3, warmup=1, device=dev, targets=targets)
    tile_b, bd_b, sched_b, timings = tuned["tile"], tuned["blend_depth"], tuned["schedule"], tuned["timings"]
    plan = BatchPlan(gm.n, gm.sh_degree, 8, total_px, tile_b, bd_b, cap, dev)
    slots = [ViewSlot.make(c, dev, backward=True, target=targets[k],
                           lidar=R.LidarHits(torch.from_numpy(lidars[k][0]).to(dev),
                                             torch.from_numpy(lidars[k][1]).to(dev), weight=1.0))
             for k, c in enumerate(cams)]
    grads = R.ParamGrads.empty(gm)
    run = lambda: plan.run(gm, slots, fwd=True, bwd=True, grads=grads, graph=True, overwrite=True, schedule=sched_b)
    ms_b = timed(torch, run, reps, 3)
    assert plan.num_pairs() <= plan.capacity
    plan.close()
    seq = [PlainStep(gm, c, lidars[k][0], targets[k], lidars[k][1], tile, bd, dev)
           for k, c in enumerate(cams)]

    def run_seq():
        for st in seq:
            st.step()
    ms_s = timed(torch, run_seq, reps, 3)
    del seq
    return {"views": 8, "pixels": total_px, "tile": list(R.tile_wh(tile_b)), "blend_depth": bd_b,
            "bwd_schedule": SCHEDULE_NAMES[sched_b],
            "autotune_ms": {k: round(v, 4) for k, v in timings.items()},
            "batched_graph_ms": round(ms_b, 4), "batched_views_s": round(8e3 / ms_b, 2),
            "sequential_plain_ms": round(ms_s, 4), "sequential_views_s": round(8e3 / ms_s, 2),
            "speedup": round(ms_s / ms_b, 3)}


def measure_serving(R, torch, S, tile, bd, dev, n_req, log):
    """Novel-view serving from a resident 3M-Gaussian map of a 1 km street: Poisson arrivals at
    0.5 / 0.8 / 1.0 / 1.2 x the one-at-a-time capacity, 640x360 / 1280x720 / 1920x1080 at
    50/35/15 %, RGB + depth forward; arrival-to-completion latency, batched (up to 16 views
    per launch) against one-at-a-time FIFO."""
    import numpy as np
    from paper_2507_04004_amd.serve import RenderServer, poisson_arrivals, simulate
    log("[bench] serving: generating the 3M-Gaussian 1 km map")
    g5 = S.street_map(3_000_000, seed=4, z_range=(-20.0, 1020.0), n_boxes=260, n_clusters=860)
    gm5 = R.GaussianMap.from_numpy(g5, dev)
    del g5
    server = RenderServer(gm5, max_batch=16, memory_budget=8 << 30, tile=tile, blend_depth=bd, device=dev)
    cams = S.serving_requests(n_req, seed=4)
    # warm-up, then the one-at-a-time capacity on back-to-back requests
    simulate(server, cams[:48], np.zeros(48), batched=True)
    simulate(server, cams[:48], np.zeros(48), batched=False)
    m = min(n_req, 300)
    st = simulate(server, cams[:m], np.zeros(m), batched=False)
    cap_rate = m / (st["busy_frac"] * st["wall_s"])
    out = {"map_gaussians": gm5.n, "requests_per_rate": n_req, "fifo_capacity_req_s": round(cap_rate, 1), "rates": []}
    for f in (0.5, 0.8, 1.0, 1.2):
        arr = poisson_arrivals(n_req, f * cap_rate, seed=int(f * 100))
        b = simulate(server, cams, arr, batched=True)
        o = simulate(server, cams, arr, batched=False)
        out["rates"].append({"load": f, "rate_req_s": round(f * cap_rate, 1),
                             "batched": {k: round(b[k], 3) for k in ("p50_ms", "p99_ms", "mpix_per_s")},
                             "fifo": {k: round(o[k], 3) for k in ("p50_ms", "p99_ms", "mpix_per_s")}})
        log(f"[bench] serving load {f}: batched {out['rates'][-1]['batched']} fifo {out['rates'][-1]['fifo']}")
    server.close()
    return out


def measure_sparse_adam(R, torch, S, ps, tile, dev, reps=20):
    """Sparse Adam (gs_adam_sparse) on the 1M map with the benchmark's last gradients: over the
    Gaussians the headline view reached, those a centred 256x192 window reached, and all of them.
    Algorithmic bytes per updated Gaussian: 16 B read and 12 B written per parameter plane (param,
    both moments, gradient) plus the 4 renderer planes written back (scale, opacity), and the
    tile counts read per Gaussian and view."""
    from paper_2507_04004_amd.adam import SparseAdam
    opt = SparseAdam(ps.gm)
    n = ps.n
    planes = sum(raw.numel() // n for raw, *_ in opt.groups)
    win = S.headline_camera().window(512, 264, 256, 192)
    spl_w = R.preprocess(ps.gs, R.camera_struct(win), tile, dev)
    cases = (("headline_view", ps.spl.n_tiles.view(1, -1)), ("window_256x192", spl_w.n_tiles.view(1, -1)),
             ("all", None))
    out = {"gaussians": n, "planes": planes}
    for name, vis in cases:
        for _ in range(3):
            opt.step(ps.grads, vis)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            opt.step(ps.grads, vis)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        reached = n if vis is None else int((vis > 0).any(0).sum().item())
        nbytes = reached * (planes * 28 + 4 * 4) + (0 if vis is None else 4 * n * vis.shape[0])
        out[name] = {"reached": reached, "ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def measure_tracking(R, torch, S, tile, bd, dev, n=2_000_000, frames=10):
    """Photometric tracking (camera factor option 2): N_t = 30 pose iterations per frame, map
    frozen, on a 2M-Gaussian street map at 1280x720. Each frame starts from the true pose moved
    by a seeded left perturbation (N(0, 3 cm) per translation axis, N(0, 0.003 rad) per rotation
    axis) and refines it against the image rendered at the true pose (rendered once, untimed),
    with the library's default step sizes; the median start and end pose errors over the
    frames are reported. Timed: `frames` calls of the captured loop, no host
    synchronisation between them. Also the D-SSIM kernels alone on a 3x720x1280 image pair,
    against HBM: algorithmic bytes per value 20 in the forward (two images read, three
    derivative maps written) and 28 in the backward (three maps and two images read, dL/dC
    read and written)."""
    import numpy as np
    from paper_2507_04004_amd import track as T
    g = S.street_map(n, seed=6)
    cam = S.headline_camera()
    gm = R.GaussianMap.from_numpy(g, dev)
    cs = R.camera_struct(cam)
    spl = R.preprocess(gm.struct(), cs, tile, dev)
    bins = R.bin_sort_fit(spl, gm.n, cs, tile, dev)
    fr = R.render_fwd(spl, gm.n, bins, cs, bd, dev)
    target = fr.color.clone()
    del spl, bins, fr
    rng = np.random.default_rng(8)
    starts = []
    for _ in range(frames):
        starts.append(R.camera_left_update(cs, np.r_[rng.normal(0, 0.03, 3), rng.normal(0, 0.003, 3)]))
    trk = T.PoseTracker(gm, cam.w * cam.h, tile=tile, blend_depth=bd, device=dev)
    out = {"n_gaussians": gm.n, "width": cam.w, "height": cam.h, "iters": T.DEFAULTS["iters"], "frames": frames}
    for graph in (True, False):
        trk.track(starts[0], target, graph=graph, check=True)  # capture / warm up, pair check
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for st in starts:
            trk.track(st, target, graph=graph, check=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / frames
        key = "graph" if graph else "eager"
        out[key] = {"ms_per_frame": round(ms, 3), "frames_s": round(1e3 / ms, 2),
                    "iters_s": round(1e3 * T.DEFAULTS["iters"] / ms, 1)}
    true_pose = np.r_[np.asarray(cs.R_cw[:]), np.asarray(cs.t_cw[:])]

    def err(pose):
        d = T.pose_residual(true_pose, pose)
        return [float(np.linalg.norm(d[:3])), float(np.linalg.norm(d[3:]))]
    e0, e1, pairs, losses = [], [], 0, []
    for st in starts:  # every frame once more with its trace (untimed)
        res = trk.track(st, target, graph=True, trace=True, check=True)
        tr = res.trace.double().cpu().numpy()
        e0.append(err(tr[0, :12]))
        e1.append(err(res.pose.double().cpu().numpy()))
        losses.append((float(tr[0, 18] + tr[0, 19]), float(tr[-1, 18] + tr[-1, 19])))
        pairs = max(pairs, res.pairs)
    e0, e1, losses = np.array(e0), np.array(e1), np.array(losses)
    out["pairs_max"] = pairs
    out["step_sizes"] = {"rho_m": T.DEFAULTS["lr_rho"], "phi_rad": T.DEFAULTS["lr_phi"]}
    out["loss_first_last_median"] = [round(float(np.median(losses[:, 0])), 5), round(float(np.median(losses[:, 1])), 5)]
    out["pose_error_m_rad_median"] = {"start": [round(float(np.median(e0[:, 0])), 5), round(float(np.median(e0[:, 1])), 6)],
                                      "end": [round(float(np.median(e1[:, 0])), 5), round(float(np.median(e1[:, 1])), 6)],
                                      "end_max": [round(float(e1[:, 0].max()), 5), round(float(e1[:, 1].max()), 6)]}
    trk.close()
    # D-SSIM kernels alone
    x = target.contiguous()
    y = torch.roll(target, shifts=(3, 5), dims=(1, 2)).contiguous()
    dC = torch.zeros_like(x)
    loss = torch.empty(1, device=dev)
    scratch = torch.empty(R.N.lib().gs_dssim_scratch_bytes(3, cam.h, cam.w), dtype=torch.uint8, device=dev)
    for _ in range(3):
        R.loss_dssim(x, y, 0.5, dC, loss, scratch)
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        R.loss_dssim(x, y, 0.5, dC, loss, scratch)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 48 * x.numel()
    out["dssim"] = {"values": x.numel(), "ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                    "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del gm, target, x, y, dC, scratch
    torch.cuda.empty_cache()
    return out


def measure_expansion(R, N, torch, S, ps, dev, n_pts=1_000_000, reps=10):
    """Map expansion at the headline keyframe: 1M colourised points (the means of a second street
    map, seeded, with random colours) tested against the rendered opacity of the headline view
    (O < 0.99), and the 1M-Gaussian map grown by the selected points. Algorithmic bytes: the
    selection reads 12 B of position per point and 4 B of opacity per point inside the window;
    the write copies the existing map (236 B per Gaussian, read and written) and writes 236 B per
    new Gaussian from 24 B of point data."""
    import numpy as np
    gp = S.street_map(n_pts, seed=11)
    rng = np.random.default_rng(12)
    xyz = torch.from_numpy(np.ascontiguousarray(gp.mean, np.float32)).to(dev)
    rgb = torch.from_numpy(rng.uniform(0, 1, (3, n_pts)).astype(np.float32)).to(dev)
    del gp
    pts = N.Points(n_pts, R._p(xyz), R._p(rgb))
    scratch = torch.empty(N.lib().gs_expand_scratch_bytes(n_pts), dtype=torch.uint8, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    alpha = ps.frame.alpha
    st = R._stream()

    def select():
        N.check(N.lib().gs_expand_select(C.byref(pts), C.byref(ps.cs), R._p(alpha), 0.99, R._p(count),
                                         R._p(scratch), scratch.numel(), st), "gs_expand_select")
    select()
    added = int(count.item())
    gm = ps.gm
    m = gm.n + added
    e = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
    new = R.GaussianMap(e(3, m), e(3, m), e(4, m), e(m), e(3, m), e(45, m), 3)
    out = N.GaussiansOut(m, 3, R._p(new.mean), R._p(new.scale), R._p(new.rot), R._p(new.opacity), R._p(new.sh_dc),
                         R._p(new.sh_rest))
    old = gm.struct()

    def write():
        N.check(N.lib().gs_expand_write(C.byref(pts), C.byref(ps.cs), C.byref(old), added, R._p(scratch),
                                        scratch.numel(), C.byref(out), st), "gs_expand_write")

    def timed_ms(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    t_sel, t_wr = timed_ms(select), timed_ms(write)
    # points whose pixel falls inside the window (the opacity gathers), counted on the host
    Rm = np.asarray(ps.cs.R_cw[:], np.float64).reshape(3, 3)
    pc = Rm @ xyz.double().cpu().numpy() + np.asarray(ps.cs.t_cw[:], np.float64)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = ps.cs.fx * pc[0] / pc[2] + ps.cs.cx
        v = ps.cs.fy * pc[1] / pc[2] + ps.cs.cy
    inwin = int(((pc[2] > 0.2) & (u > -0.5) & (u < ps.cs.w - 0.5) & (v > -0.5) & (v < ps.cs.h - 0.5)).sum())
    b_sel = 12 * n_pts + 4 * inwin
    b_wr = 2 * 236 * gm.n + (236 + 24) * added
    res = {"points": n_pts, "in_window": inwin, "added": added, "map_before": gm.n,
           "select": {"ms": round(t_sel, 4), "GB/s": round(b_sel / (t_sel * 1e-3) / 1e9, 1),
                      "frac_hbm": round(b_sel / (t_sel * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "points_s": round(n_pts / (t_sel * 1e-3), 0)},
           "write": {"ms": round(t_wr, 4), "GB/s": round(b_wr / (t_wr * 1e-3) / 1e9, 1),
                     "frac_hbm": round(b_wr / (t_wr * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    del new, xyz, rgb, scratch
    torch.cuda.empty_cache()
    return res


def measure_autograd(R, torch, S, g, cam, pix, ds, target_color, tile, bd, dev, calls=200, warmup=20):
    """The differentiable form users call: GSRender forward (with the LiDAR term), the RGB L1
    loss in torch, and the backward to every parameter and the pose tangent (a device tensor
    at zero), one call after another; per-call latency from events around each call."""
    gm = R.GaussianMap.from_numpy(g, dev)
    params = [gm.mean, gm.scale, gm.rot, gm.opacity, gm.sh_dc, gm.sh_rest]
    for t in params:
        t.requires_grad_(True)
    xi = torch.zeros(6, device=dev, requires_grad=True)
    lidar = R.LidarHits(torch.from_numpy(pix).to(dev), torch.from_numpy(ds).to(dev), weight=1.0)
    settings = R.RenderSettings(cam, tile=tile, blend_depth=bd, lidar=lidar)

    def call():
        for t in params:
            t.grad = None
        xi.grad = None
        color, _, _, lloss = R.render(settings, gm, xi)
        loss = (color - target_color).abs().mean() + lloss
        loss.backward()

    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    settings.check()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        call()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    settings.check()  # no call overflowed its pair capacity
    lat = sorted(a.elapsed_time(b) for a, b in ev)
    pct = lambda xs, q: xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]
    return {"calls": calls, "p50_ms": round(pct(lat, 0.5), 4), "p99_ms": round(pct(lat, 0.99), 4),
            "views_s": round(1e3 / pct(lat, 0.5), 2), "wall_ms_per_call": round(wall / calls * 1e3, 4),
            "tile": tile, "blend_depth": bd, "pair_capacity": settings.capacity}


def se3_left(cam, xi):
    """Camera with pose Exp(xi) T_cw (closed-form SE(3) exponential; xi = (rho, phi))."""
    import dataclasses
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = float(np.linalg.norm(phi))
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-12:
        dR, V = np.eye(3) + K, np.eye(3) + 0.5 * K
    else:
        dR = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K
        V = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K
    return dataclasses.replace(cam, R_cw=dR @ cam.R_cw, t_cw=dR @ cam.t_cw + V @ rho)


def measure_c4(R, torch, S, tile, bd, dev, reps=20):
    """Differentiation at map size: a frozen 2M-Gaussian street map, one 1280x720 view, the L1 +
    LiDAR loss against the render from a pose moved by Exp(delta), delta ~ N(0, 0.01^2) per
    axis, and the backward to every parameter and the pose tangent; plus the memory the
    forward leaves for the backward against per-fragment state. (Its gradients are compared
    with the float64 oracle and finite differences by the GPU tests, not here.)"""
    from paper_2507_04004_amd.step import PlainStep
    g = S.street_map(2_000_000, seed=3)
    cam = S.headline_camera()
    gm = R.GaussianMap.from_numpy(g, dev)
    delta = np.random.default_rng(3).normal(0.0, 0.01, 6)
    pix = S.lidar_beams(cam, 32, 30.0, 0.32, seed=103)
    tgt = PlainStep(gm, se3_left(cam, delta), np.zeros(0, np.int32), torch.zeros(3, cam.h, cam.w, device=dev),
                    np.zeros(0, np.float32), tile, bd, dev)
    tgt.forward()
    torch.cuda.synchronize()
    target = tgt.frame.color.clone()
    hits, ds = lidar_targets(tgt.frame, pix)
    del tgt
    ps = PlainStep(gm, cam, hits, target, ds, tile, bd, dev)
    ms = timed(torch, ps.step, reps, 3)
    assert not ps.overflowed()
    kept = R.kept_bytes(ps.spl, ps.bins, ps.frame, ps.cs, bd)
    cnt = R.Frame.empty(cam.h, cam.w, dev, count=True)
    R.render_fwd(ps.spl, ps.n, ps.bins, ps.cs, bd, dev, out=cnt)
    torch.cuda.synchronize()
    frags = int(cnt.n_contrib.long().sum().item())
    pose = ps.grads.pose.cpu().numpy().tolist()
    res = {"gaussians": int(g.n), "width": cam.w, "height": cam.h, "lidar_hits": int(hits.size),
           "fwd_bwd_ms": round(ms, 4), "views_s": round(1e3 / ms, 1),
           "pose_grad": [round(v, 8) for v in pose],
           "kept_MB": {k: round(v / 1e6, 2) for k, v in kept.items()},
           "per_fragment_MB": round(8 * frags / 1e6, 1), "fragments": frags}
    del ps, cnt, gm
    torch.cuda.empty_cache()
    return res


def host_cpu():
    """CPU model, logical CPUs, physical cores (distinct (package, core) pairs) and the CPUs this
    process may run on."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "physical_cores": len(cores) or None,
            "cpus_allowed": allowed}


def cpu_baseline(g, cam, gC_np, repeats, single_thread=True):
    """The FP64 oracle (as it stands) on the host: full-view fwd + bwd of the same workload at the
    OpenMP thread count the process gets (median of `repeats` views) and at one thread (one view:
    ~13 s of host work, which keeps the whole baseline within ~30 s)."""
    import oracle
    oc = oracle.camera_f32(cam)

    def one():
        t0 = time.perf_counter()
        oracle.render(g, oc, tile=16, band=0.0)
        oracle.backward(g, oc, gC_np)
        return time.perf_counter() - t0

    threads = oracle.lib().or_max_threads()
    t = statistics.median(one() for _ in range(repeats))
    res = {"value": round(1.0 / t, 4), "unit": "views/s", "cores": threads, "kind": "oracle",
           "sample": f"one full 1280x720 fwd+bwd view of the 1M-Gaussian map in float64 at {threads} OpenMP threads "
                     f"(median of {repeats} views, {t:.2f} s each; upstream dL/dC = sign residual of the L1 loss)",
           "host": host_cpu()}
    if single_thread:
        prev = oracle.set_threads(1)
        t1 = one()
        oracle.set_threads(prev)
        res["single_thread"] = {"value": round(1.0 / t1, 4), "unit": "views/s", "s_per_view": round(t1, 2),
                                "views": 1, "speedup_all_threads": round(t1 / t, 2)}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2507_04004_amd import _native as N
    from paper_2507_04004_amd import raster as R
    from paper_2507_04004_amd import scenes as S
    from paper_2507_04004_amd.step import PlainStep

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    dev = "cuda:0"
    if args.tracking_only:
        log("[bench] photometric tracking only")
        print(json.dumps({"tracking": measure_tracking(R, torch, S, args.tile, args.blend_depth, dev,
                                                       frames=args.tracking_frames)}), flush=True)
        return
    log("[bench] generating the 1M-Gaussian street map")
    g = S.street_map(args.n, seed=2)
    cam = S.headline_camera()
    pix = S.lidar_beams(cam, 32, 30.0, 0.32, seed=102)

    # Targets: a perturbed copy rendered once by the same GPU path (untimed).
    log("[bench] rendering targets")
    gp = S.perturb(g, 0.01, seed=3)
    tgt = PlainStep(R.GaussianMap.from_numpy(gp, dev), cam, pix, torch.zeros(3, cam.h, cam.w, device=dev),
                    np.zeros(pix.size, np.float32), args.tile, args.blend_depth, dev)
    tgt.forward()
    torch.cuda.synchronize()
    target_color = tgt.frame.color.clone()
    D = tgt.frame.depth.flatten().cpu().numpy()
    O = tgt.frame.alpha.flatten().cpu().numpy()
    keep = O[pix] > 0
    pix = pix[keep].astype(np.int32)
    ds = (D[pix] / O[pix]).astype(np.float32)
    del tgt
    torch.cuda.empty_cache()

    if args.copy_calibration:
        src = torch.ones(64 << 20, device=dev)  # 256 MiB read, 256 MiB written
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log("[bench] building the step")
    gm = R.GaussianMap.from_numpy(g, dev)
    ps = PlainStep(gm, cam, pix, target_color, ds, args.tile, args.blend_depth, dev)
    for _ in range(args.warmup):
        ps.step()
    torch.cuda.synchronize()

    # ---- timed fwd+bwd steps; the dominant kernel (the compositing backward) is bracketed by
    # library events on its stream inside the timed region --------------------------------------
    L = N.lib()
    N.check(L.gs_profile_enable(1 << N.GS_STAGE_BLEND_BWD, max(args.steps, 1)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ps.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot, cnt = C.c_double(), C.c_int32()
    N.check(L.gs_profile_read(N.GS_STAGE_BLEND_BWD, C.byref(tot), C.byref(cnt)))
    dom_ms = tot.value / max(cnt.value, 1)
    L.gs_profile_disable()
    # per-stage breakdown from a separate pass with every stage bracketed (untimed)
    stage_reps = 10
    N.check(L.gs_profile_enable(0x1F, stage_reps))
    for _ in range(stage_reps):
        ps.step()
    torch.cuda.synchronize()
    stage_ms = {}
    names = {N.GS_STAGE_PREPROCESS: "preprocess", N.GS_STAGE_BIN_SORT: "bin_sort",
             N.GS_STAGE_BLEND_FWD: "blend_fwd", N.GS_STAGE_BLEND_BWD: "blend_bwd",
             N.GS_STAGE_PREPROCESS_BWD: "preprocess_bwd"}
    for sid, name in names.items():
        tot, cnt = C.c_double(), C.c_int32()
        N.check(L.gs_profile_read(sid, C.byref(tot), C.byref(cnt)))
        stage_ms[name] = tot.value / max(cnt.value, 1)
    L.gs_profile_disable()
    log(f"[bench] {args.steps} steps in {wall:.3f} s; compositing backward {dom_ms:.4f} ms; stage ms {stage_ms}")

    # ---- latency over many calls, and render-only throughput ----------------------------------
    lat = []
    n_lat = args.latency_calls
    evl = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    for i in range(n_lat):
        evl[i][0].record()
        ps.step()
        evl[i][1].record()
    torch.cuda.synchronize()
    lat = sorted(a.elapsed_time(b) for a, b in evl)
    evr = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    for i in range(n_lat):
        evr[i][0].record()
        ps.forward()
        evr[i][1].record()
    torch.cuda.synchronize()
    rlat = sorted(a.elapsed_time(b) for a, b in evr)
    pct = lambda xs, q: xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]

    # ---- the two compositing-backward schedules on the same step (stage events) ---------------
    sched_ms = {}
    for name, sc in (("chunks", N.GS_BWD_CHUNKS), ("buckets", N.GS_BWD_BUCKETS)):
        if sc == N.GS_BWD_BUCKETS and args.tile == 32:
            continue
        ps.s_grads.schedule = sc
        for _ in range(2):
            ps.step()
        N.check(L.gs_profile_enable(1 << N.GS_STAGE_BLEND_BWD, 10))
        for _ in range(10):
            ps.step()
        tot, cnt = C.c_double(), C.c_int32()
        N.check(L.gs_profile_read(N.GS_STAGE_BLEND_BWD, C.byref(tot), C.byref(cnt)))
        L.gs_profile_disable()
        sched_ms[name] = round(tot.value / max(cnt.value, 1), 4)
    ps.s_grads.schedule = N.GS_BWD_CHUNKS
    log(f"[bench] compositing backward by schedule (ms): {sched_ms}")

    # ---- counts for the roofline (untimed) -----------------------------------------------------
    P = ps.bins.pairs()
    assert P <= ps.capacity, "pair capacity overflow during timing"
    cnt_frame = R.Frame.empty(cam.h, cam.w, dev, count=True)
    R.render_fwd(ps.spl, ps.n, ps.bins, ps.cs, args.blend_depth, dev, out=cnt_frame)
    torch.cuda.synchronize()
    # evaluations: the forward count takes every splat of a tile's list for every pixel of the
    # tile (an upper bound: pixels stop early, and the forward skips the later chunks of a tile
    # whose pixels have all stopped); the backward walks each pixel's list from its last
    # contributor to the front
    tr = ps.bins.tile_range.view(-1, 2).long()
    lens = (tr[:, 1] - tr[:, 0]).cpu().numpy()
    tx, ty = (cam.w + args.tile - 1) // args.tile, (cam.h + args.tile - 1) // args.tile
    pw = np.minimum(args.tile, cam.w - np.arange(tx) * args.tile)
    ph = np.minimum(args.tile, cam.h - np.arange(ty) * args.tile)
    E_f = int((lens.reshape(ty, tx) * np.outer(ph, pw)).sum())
    E_b = int((cnt_frame.last.long() + 1).sum().item())
    C_n = int(cnt_frame.n_contrib.long().sum().item())
    V = int((ps.spl.n_tiles > 0).sum().item())
    work = {
        "preprocess": ("hbm", BYTES_PRE_PER_N * ps.n + BYTES_PRE_PER_V * V),
        "bin_sort": ("hbm", BYTES_BIN_PER_N * ps.n + BYTES_BIN_PER_V * V + BYTES_BIN_PER_P * P
                     + BYTES_BIN_PER_T * tx * ty),
        "preprocess_bwd": ("hbm", BYTES_PREBWD_PER_N * ps.n + BYTES_PREBWD_PER_V * V),
        "blend_fwd": ("alu", FLOPS_FWD_EVAL * E_f),
        "blend_bwd": ("alu", FLOPS_BWD_EVAL * E_b),
    }
    # dominant kernel: the compositing backward, one launch per step (its stage events bracket
    # exactly that launch on the library's stream)
    dom = "blend_bwd"
    bound, amount = work[dom]
    t_s = dom_ms * 1e-3  # measured in the timed region
    achieved, peak, unit = amount / t_s / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
    tight = FLOPS_MIN_EVAL * E_b + FLOPS_MIN_BWD_CONTRIB * C_n
    roofline = {"bound": bound, "kernel": "k_blend_bwd_chunk", "achieved": round(achieved, 3), "peak": peak,
                "unit": unit, "frac": round(achieved / peak, 5),
                "traffic": measured_traffic("k_blend_bwd_chunk", args.tile, args.blend_depth),
                "avg_launch_ms": round(dom_ms, 4), "flops_per_launch": amount,
                "flop_count": f"{FLOPS_BWD_EVAL} per backward evaluation x E_b {E_b}",
                "frac_of_single_issue_fp32": round(achieved / FP32_NONPACKED_TFLOPS, 5),
                "tight_count": {"flops_per_launch": tight, "TFLOP/s": round(tight / t_s / 1e12, 3),
                                "frac": round(tight / t_s / 1e12 / peak, 5)}}
    per_stage = {}
    for k, (b, amt) in work.items():
        ts = stage_ms[k] * 1e-3
        if ts <= 0:
            continue
        if b == "hbm":
            per_stage[k] = {"ms": round(stage_ms[k], 4), "GB/s": round(amt / ts / 1e9, 1),
                            "frac_hbm": round(amt / ts / 1e9 / HBM_PEAK_GBS, 4)}
        else:
            per_stage[k] = {"ms": round(stage_ms[k], 4), "TFLOP/s": round(amt / ts / 1e12, 3),
                            "frac_fp32": round(amt / ts / 1e12 / FP32_PEAK_TFLOPS, 4)}

    ms_per_step = wall * 1e3 / args.steps
    out = {
        "metric": "fwd+bwd views/s at 1280x720, 1M Gaussians",
        "value": round(1e3 / ms_per_step, 3),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M-Gaussian street map (SH3), one 1280x720 view, fx=900, 32-beam LiDAR; "
                               "fwd + L1/LiDAR loss + bwd to all parameters and the pose",
                   "n_gaussians": ps.n, "width": cam.w, "height": cam.h, "tile": args.tile,
                   "blend_depth": args.blend_depth, "visible": V, "pairs": P, "evals_fwd": E_f, "evals_bwd": E_b,
                   "contributions": C_n, "lidar_hits": int(pix.size)},
        "render_mpix_s": round(cam.w * cam.h / (statistics.median(rlat) * 1e-3) / 1e6, 2),
        "latency_ms": {"fwd_bwd_p50": round(pct(lat, 0.5), 4), "fwd_bwd_p99": round(pct(lat, 0.99), 4),
                       "render_p50": round(pct(rlat, 0.5), 4), "render_p99": round(pct(rlat, 0.99), 4),
                       "calls": n_lat},
        "stages": per_stage,
        "bwd_schedule_ms": sched_ms,
        "roofline": roofline,
    }
    if not args.no_autograd:
        log("[bench] autograd function")
        out["autograd"] = measure_autograd(R, torch, S, g, cam, pix, ds, target_color, args.tile, args.blend_depth,
                                           dev, calls=args.latency_calls)
        log(f"[bench] autograd {out['autograd']}")
    gC_cpu = None
    if not args.no_cpu_baseline:
        gC_cpu = np.sign(ps.frame.color.cpu().numpy().astype(np.float64) - target_color.cpu().numpy()) / ps.nval
    if not args.no_small:
        log("[bench] small configurations")
        out["small_configs"] = measure_small_configs(R, N, torch, S, args.tile, args.blend_depth, dev)
    if not args.no_batched:
        log("[bench] batched keyframes")
        out["batched"] = measure_batched(R, N, torch, S, g, gm, args.tile, args.blend_depth, dev)
        log(f"[bench] batched {out['batched']}")
    if not args.no_adam:
        log("[bench] sparse Adam")
        out["sparse_adam"] = measure_sparse_adam(R, torch, S, ps, args.tile, dev)
        log(f"[bench] sparse Adam {out['sparse_adam']}")
    if not args.no_expansion:
        log("[bench] map expansion")
        out["expansion"] = measure_expansion(R, N, torch, S, ps, dev)
        log(f"[bench] expansion {out['expansion']}")
    if not args.no_c4:
        log("[bench] differentiation at 2M Gaussians")
        out["c4"] = measure_c4(R, torch, S, args.tile, args.blend_depth, dev)
        log(f"[bench] c4 {out['c4']}")
    if not args.no_tracking:
        log("[bench] photometric tracking")
        out["tracking"] = measure_tracking(R, torch, S, args.tile, args.blend_depth, dev, frames=args.tracking_frames)
        log(f"[bench] tracking {out['tracking']}")
    if not args.no_serving:
        del ps
        torch.cuda.empty_cache()
        out["serving"] = measure_serving(R, torch, S, args.tile, args.blend_depth, dev, args.serve_requests, log)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(g, cam, gC_cpu, args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
