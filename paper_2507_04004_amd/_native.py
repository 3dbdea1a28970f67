"""ctypes view of the C ABI in include/gs.h (argument marshalling only).

The library is loaded from the package's _lib/ directory (or from GS_LIB_PATH, which the
sanitizer test sets to an instrumented build of the same sources). There is no fallback: if
the HIP library is missing, loading raises, so nothing silently runs elsewhere.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GS_LIB_PATH") or os.path.join(_HERE, "_lib", "libgs.so")

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_HIP, GS_ERR_UNSUPPORTED, GS_ERR_CAPACITY = 0, 1, 2, 3, 4
GS_MAX_VIEWS = 16
GS_FWD, GS_BWD, GS_GRAPH = 1, 2, 4
GS_PLAN_FWD_ONLY = 1

fp = C.POINTER(C.c_float)
vp = C.c_void_p


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32),
                ("w", C.c_int32), ("h", C.c_int32), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("R_cw", C.c_float * 9), ("t_cw", C.c_float * 3), ("bg", C.c_float * 3)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32)] + [
        (k, vp) for k in ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")]


class Projected(C.Structure):
    _fields_ = [(k, vp) for k in ("card", "n_tiles", "dkey", "pose")]


class Bins(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("capacity", C.c_int64), ("vals", vp),
                ("tile_range", vp), ("num_pairs", vp), ("scratch", vp), ("scratch_bytes", C.c_size_t)]


class Image(C.Structure):
    _fields_ = [(k, vp) for k in ("color", "depth", "alpha", "t_final", "last", "n_contrib", "state")] + [
        ("state_bytes", C.c_size_t)]


class Lidar(C.Structure):
    _fields_ = [("m", C.c_int32), ("pix", vp), ("depth_target", vp), ("weight", C.c_float), ("loss_out", vp),
                ("grad_scale", vp)]


class Grads(C.Structure):
    _fields_ = [(k, vp) for k in ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest", "pose", "scratch")] + [
        ("scratch_bytes", C.c_size_t), ("overwrite", C.c_int32), ("schedule", C.c_int32)]


GS_BWD_CHUNKS, GS_BWD_BUCKETS = 0, 1


class View(C.Structure):
    _fields_ = [("cam", Camera), ("out", Image), ("dL_dC", vp), ("dL_dD", vp), ("dL_dO", vp), ("lidar", Lidar),
                ("target", vp), ("rgb_weight", C.c_float), ("rgb_loss_out", vp), ("pose_grad", vp)]


GS_ACT_NONE, GS_ACT_EXP, GS_ACT_SIGMOID = 0, 1, 2
GS_ADAM_MAX_GROUPS = 8


class AdamGroup(C.Structure):
    _fields_ = [("param", vp), ("exp_avg", vp), ("exp_avg_sq", vp), ("grad", vp), ("act_out", vp),
                ("k", C.c_int32), ("act", C.c_int32), ("lr", C.c_float)]


class Adam(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_groups", C.c_int32), ("n_views", C.c_int32), ("visible", vp),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("bias1", C.c_float),
                ("bias2", C.c_float), ("group", AdamGroup * GS_ADAM_MAX_GROUPS)]


class TrackParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("l1_weight", C.c_float), ("ssim_weight", C.c_float), ("lr_rho", C.c_float),
                ("lr_phi", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("flags", C.c_uint32)]


TRACK_TRACE_STRIDE = 20


class Points(C.Structure):
    _fields_ = [("n", C.c_int64), ("xyz", vp), ("rgb", vp)]


class GaussiansOut(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32)] + [
        (k, vp) for k in ("mean", "scale", "rot", "opacity", "sh_dc", "sh_rest")]


class GSError(RuntimeError):
    pass


_lib = None

EXPORTS = ["gs_preprocess", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd", "gs_render_bwd_noalloc",
           "gs_render_batch", "gs_loss_l1",
           "gs_adam_sparse", "gs_loss_dssim", "gs_dssim_scratch_bytes", "gs_track_plan_create",
           "gs_track_plan_destroy", "gs_track_capacity", "gs_track_pose", "gs_track_required_pairs",
           "gs_pose_residual", "gs_pose_left_update", "gs_expand_scratch_bytes", "gs_expand_select", "gs_expand_write",
           "gs_bins_scratch_bytes", "gs_image_state_bytes", "gs_grads_scratch_bytes", "gs_batch_plan_create", "gs_batch_plan_bytes", "gs_batch_plan_destroy",
           "gs_batch_num_pairs", "gs_batch_capacity", "gs_camera_left_update", "gs_last_error",
           "gs_profile_enable", "gs_profile_read", "gs_profile_disable"]
GS_STAGE_PREPROCESS, GS_STAGE_BIN_SORT, GS_STAGE_BLEND_FWD, GS_STAGE_BLEND_BWD, GS_STAGE_PREPROCESS_BWD = range(5)


def lib():
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GSError(f"HIP library not built: {LIB_PATH} (run paper_2507_04004_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.gs_preprocess.argtypes = [P(Gaussians), P(Camera), C.c_int32, C.c_int32, P(Projected), vp]
    L.gs_bin_sort.argtypes = [P(Projected), C.c_int64, P(Camera), P(Bins), vp]
    L.gs_render_fwd.argtypes = [P(Projected), C.c_int64, P(Bins), P(Camera), C.c_int32, P(Lidar), P(Image), vp]
    L.gs_render_bwd.argtypes = [P(Gaussians), P(Camera), P(Projected), P(Bins), P(Image), vp, vp, vp, P(Lidar),
                                C.c_int32, P(Grads), vp]
    L.gs_render_bwd_noalloc.argtypes = L.gs_render_bwd.argtypes
    L.gs_loss_l1.argtypes = [vp, vp, C.c_int64, C.c_float, vp, vp, vp]
    L.gs_adam_sparse.argtypes = [P(Adam), vp]
    L.gs_dssim_scratch_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    L.gs_dssim_scratch_bytes.restype = C.c_size_t
    L.gs_loss_dssim.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float, vp, vp, vp, C.c_size_t, vp]
    L.gs_bins_scratch_bytes.argtypes = [C.c_int64, C.c_int64, C.c_int64]
    L.gs_bins_scratch_bytes.restype = C.c_size_t
    L.gs_image_state_bytes.argtypes = [C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32]
    L.gs_image_state_bytes.restype = C.c_size_t
    L.gs_grads_scratch_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int64]
    L.gs_grads_scratch_bytes.restype = C.c_size_t
    L.gs_batch_plan_create.argtypes = [P(vp), C.c_int64, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                       C.c_int32, C.c_int64, C.c_uint32]
    L.gs_batch_plan_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_int64, C.c_uint32]
    L.gs_batch_plan_bytes.restype = C.c_size_t
    L.gs_batch_plan_destroy.argtypes = [vp]
    L.gs_batch_plan_destroy.restype = None
    L.gs_render_batch.argtypes = [vp, P(Gaussians), C.c_int32, P(View), C.c_uint32, P(Grads), vp]
    L.gs_batch_num_pairs.argtypes = [vp, P(C.c_int64), vp]
    L.gs_batch_capacity.argtypes = [vp]
    L.gs_batch_capacity.restype = C.c_int64
    L.gs_camera_left_update.argtypes = [P(Camera), P(C.c_float * 6), P(Camera)]
    L.gs_pose_left_update.argtypes = [P(Camera), vp, vp, vp]
    L.gs_track_plan_create.argtypes = [P(vp), C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int64]
    L.gs_track_plan_destroy.argtypes = [vp]
    L.gs_track_plan_destroy.restype = None
    L.gs_track_capacity.argtypes = [vp]
    L.gs_track_capacity.restype = C.c_int64
    L.gs_track_pose.argtypes = [vp, P(Gaussians), P(Camera), vp, P(TrackParams), vp, vp, vp]
    L.gs_track_required_pairs.argtypes = [vp, P(C.c_int64), vp]
    L.gs_pose_residual.argtypes = [P(C.c_float * 12), P(C.c_float * 12), P(C.c_double * 6)]
    L.gs_expand_scratch_bytes.argtypes = [C.c_int64]
    L.gs_expand_scratch_bytes.restype = C.c_size_t
    L.gs_expand_select.argtypes = [P(Points), P(Camera), vp, C.c_float, vp, vp, C.c_size_t, vp]
    L.gs_expand_write.argtypes = [P(Points), P(Camera), P(Gaussians), C.c_int64, vp, C.c_size_t, P(GaussiansOut), vp]
    L.gs_profile_enable.argtypes = [C.c_uint32, C.c_int32]
    L.gs_profile_read.argtypes = [C.c_int32, P(C.c_double), P(C.c_int32)]
    L.gs_profile_disable.argtypes = []
    L.gs_profile_disable.restype = None
    L.gs_last_error.argtypes = []
    L.gs_last_error.restype = C.c_char_p
    _lib = L
    return L


def check(rc: int, what: str = "") -> None:
    if rc != GS_OK:
        msg = lib().gs_last_error().decode(errors="replace")
        raise GSError(f"{what} failed (code {rc}): {msg}")
