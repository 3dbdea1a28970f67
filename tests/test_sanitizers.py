"""Sanitizer builds (CPU only): the oracle and the host side of the C ABI run under
AddressSanitizer and UndefinedBehaviorSanitizer, any report fatal.

- oracle: gs_oracle.c and bins32.c built with -fsanitize=address,undefined; a child process
  preloading gcc's runtimes renders, differentiates, bins (float32 and float64 lists, pair
  margins, marginal flags) and replays small, windowed, street and empty scenes, and must
  give the plain build's results;
- C ABI host code: api.hip's host pass built with the same sanitizers (device code
  unchanged) and linked with the other objects; a child process preloading clang's runtime
  runs the host argument-check tests of test_abi.py against it.
Integer results (tile lists, last contributors, flags) must agree bit for bit; floating-point
ones within 1e-10 relative (the OpenMP backward sums in a run-dependent order).
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, code=None, args=None, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable] + (["-c", code] if code is not None else args)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    text = r.stdout + r.stderr
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]
    return text


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import build as OB
    lib = OB.build_sanitized(str(tmp_path / "gs_oracle_san.so"))
    pre = " ".join(subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
                   for n in ("libasan.so", "libubsan.so"))
    code = textwrap.dedent(f"""
        import os, sys, numpy as np
        sys.path.insert(0, {ROOT!r})
        import oracle
        from paper_2507_04004_amd import scenes as S
        out = {{}}
        def run(tag, g, cam, tile):
            r = oracle.render(g, cam, tile=tile)
            gC = np.random.default_rng(1).standard_normal((3, cam.h, cam.w))
            b = oracle.backward(g, cam, gC, np.ones((cam.h, cam.w)), np.ones((cam.h, cam.w)), tile=tile)
            b32 = oracle.bin32(g, cam, tile=tile)
            L = oracle.lists(g, cam, tile)
            fz = oracle.Frozen(g, cam, tile=tile)
            rp = oracle.replay(g, cam, fz)
            mg = oracle.marginal_gaussians(g, cam, tile=tile)
            px = oracle.render_pixels(g, cam, np.array([0, cam.w - 1]), np.array([0, cam.h - 1]))
            n = max(g.n, 1)
            ids = b32["vals"][: min(50, b32["vals"].size)].astype(np.int64)
            tl = b32["tiles"][: ids.size].astype(np.int64) if "tiles" in b32 else np.zeros_like(ids)
            pm = oracle.pair_margins(g, cam, ids, tl, tile=tile) if ids.size else (np.zeros(0), np.zeros(0))
            out[tag] = [r["color"], r["depth"], r["last_id"], b["mean"], b["pose"], b32["vals"], L["ids"],
                        rp["color"], mg, px["color"], pm[1]]
        g, cam, _ = S.config_small(0)
        cam = oracle.camera_f32(cam)
        run("small8", g, cam, 8)
        run("window16", g, cam.window(5, 3, 70, 50), 16)
        gs = S.street_scene(3000, 5, z_range=(1.0, 30.0), x_half=10.0, n_boxes=4, frac=(0.6, 0.3, 0.1),
                            n_clusters=8, sh_degree=3)
        W, H = 77, 53
        cs = oracle.camera_f32(S.Camera(W, H, 0.7 * W, 0.7 * W, (W - 1) / 2, (H - 1) / 2, np.eye(3), np.zeros(3)))
        run("street32", gs, cs, 32)
        run("empty", S.frustum_scene(0, cam, (2.0, 5.0), sh_degree=0, seed=1), cam, 16)
        np.savez(sys.argv[1] if len(sys.argv) > 1 else os.environ["OUT_NPZ"],
                 **{{f"{{k}}_{{i}}": np.asarray(v) for k, vs in out.items() for i, v in enumerate(vs)}})
        print("oracle under sanitizers: ok")
    """)
    san = str(tmp_path / "san.npz")
    plain = str(tmp_path / "plain.npz")
    text = _run({"LD_PRELOAD": pre, "GS_ORACLE_LIB": lib, "OUT_NPZ": san}, code=code)
    assert "oracle under sanitizers: ok" in text
    _run({"OUT_NPZ": plain}, code=code)
    import numpy as np
    a, b = np.load(san), np.load(plain)
    assert sorted(a.files) == sorted(b.files) and len(a.files) > 40
    for k in a.files:
        if np.issubdtype(a[k].dtype, np.floating):
            # the backward sums over OpenMP threads in a run-dependent order
            np.testing.assert_allclose(a[k], b[k], rtol=1e-10, atol=1e-12 * max(1.0, np.abs(b[k]).max(initial=0)),
                                       err_msg=k)
        else:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_abi_host_checks_under_asan_ubsan(tmp_path):
    from paper_2507_04004_amd import build as PB
    lib = PB.build_host_sanitized(str(tmp_path / "libgs_san.so"))
    rt = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        import glob
        rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))[-1]
    text = _run({"LD_PRELOAD": rt, "GS_LIB_PATH": lib},
                args=["-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py",
                      "-k", "argument or errors or rejects or exports or scratch or camera_left_update"])
    assert " passed" in text and "failed" not in text, text[-3000:]
