// Host-side declarations of the stage launchers (one per translation unit).
#pragma once

#include "gs_device.hpp"

namespace gs {

struct MapTable {
  float *gD[kMaxViews];
  float *gO[kMaxViews];
};
struct MapSrc {
  const float *gD[kMaxViews];
  const float *gO[kMaxViews];
  int64_t npx[kMaxViews];
};

// Optional event pairs around one stage's launches (see gs_profile_enable).
void profile_begin(int stage, hipStream_t st);
void profile_end(int stage, hipStream_t st);

hipError_t launch_preprocess(const ViewTable &vt, const gs_gaussians &g, const gs_projected &p, hipStream_t st);
hipError_t launch_preprocess_bwd(const ViewTable &vt, const gs_gaussians &g, const gs_projected &p, const float *g2,
                                 float4 *gdir,
                                 const gs_grads &out, float *const *pose_out, float *pose_partial, hipStream_t st);
int64_t preprocess_bwd_blocks(int64_t n);

size_t bin_scratch_bytes(int64_t n, int64_t cap);
hipError_t launch_bin_sort(const ViewTable &vt, const gs_projected &p, int64_t n, int64_t cap, uint32_t *vals,
                           uint32_t *tile_range, int64_t *num_pairs, void *scratch, hipStream_t st);
hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);

size_t blend_state_bytes(int64_t total_tiles, int64_t cap, int tw, int th, int bd);
hipError_t launch_blend_fwd(int bd, const ViewTable &vt, const ImgTable &it, const gs_projected &p,
                            const uint32_t *vals, const uint32_t *range, void *state, int64_t cap, hipStream_t st);
hipError_t launch_blend_bwd(int bd, const ViewTable &vt, const ImgTable &it, const GradTable &gtab,
                            const gs_projected &p, const uint32_t *vals, const uint32_t *range, void *state,
                            int64_t cap, float *g2, hipStream_t st, int schedule = GS_BWD_CHUNKS);
hipError_t launch_lidar_loss(const LidarTable &lt, const ImgTable &it, int max_m, hipStream_t st);
// grad2d (n floats) zeroed, the views' dense gradient maps set (max_npx 0: none), the LiDAR
// term's gradient added to them.
hipError_t launch_bwd_prep(float *g2, int64_t n, const MapSrc &src, const MapTable &dst, int n_views, int64_t max_npx,
                           const LidarTable &lt, const ImgTable &it, int max_m, hipStream_t st);
hipError_t launch_loss_l1(const float *c, const float *t, int64_t n, float weight, float *dldc, float *loss,
                          hipStream_t st);

// Sparse Adam: the validated gs_adam with the bias terms folded (step_size = lr / bias1).
struct AdamGroupDev {
  float *param, *exp_avg, *exp_avg_sq;
  const float *grad;
  float *act_out;
  int32_t k, act;
  float step_size;
};
struct AdamArgs {
  int64_t n;
  int32_t n_groups, n_views;
  const uint32_t *visible;
  float beta1, beta2, eps, sqrt_bias2;
  AdamGroupDev group[GS_ADAM_MAX_GROUPS];
};
hipError_t launch_adam_sparse(const AdamArgs &a, hipStream_t st);

size_t dssim_scratch_bytes(int c, int h, int w);
size_t dssim_scratch_bound(int64_t pixels);  // three channels, any window of at most `pixels`
hipError_t launch_dssim(const float *x, const float *y, int c, int h, int w, float weight, float *dldc, float *loss,
                        float *scratch, hipStream_t st);

// Tracking loop state in device memory: float64 master pose and Adam moments, the float32
// pose the projection kernels read (R 9, t 3, centre 3, pad), and the per-iteration
// gradient and loss terms written by the backward and the loss kernels.
struct TrackState {
  double R[9], t[3];
  double m[6], v[6];
  int64_t max_pairs;  // largest pair count seen over the iterations
  float pose[16];
  float grad[6];
  float loss[2];  // L1 term, D-SSIM term
};
struct TrackPose {
  double R[9], t[3];
};
struct TrackStepArgs {
  double lr[6];
  double beta1, beta2, eps, bias1, bias2;  // bias = 1 - beta^k
  int32_t k;
};
// Map initialization / expansion.
struct ExpandArgs {
  const float *xyz, *rgb;  // [3][n]
  int64_t n;
  float R[9], t[3];
  float fx, fy, cx, cy;
  int32_t x0, y0, w, h;
  const float *opacity;  // window plane, or null (initialization: no mask)
  float tau;
};
struct ExpandOut {
  int64_t n, n_old, added;
  int32_t k_rest;
  float *mean, *scale, *rot, *opacity, *sh_dc, *sh_rest;
};
constexpr int kMaxPlanes = 59;  // 3 + 3 + 4 + 1 + 3 + 45
struct PlaneCopy {
  const float *src[kMaxPlanes];  // null when there is no existing map
  float *dst[kMaxPlanes];
  int64_t plane[kMaxPlanes];  // plane index within its group
  float fill[kMaxPlanes];     // value of the new Gaussians on a constant plane
  int32_t constant[kMaxPlanes];
};
int64_t expand_blocks(int64_t n);
size_t expand_scratch_bytes(int64_t n);
hipError_t launch_expand_select(const ExpandArgs &a, void *scratch, int64_t *total, hipStream_t st);
hipError_t launch_expand_write(const ExpandArgs &a, const void *scratch, const ExpandOut &o, const PlaneCopy &pc,
                               int n_planes, hipStream_t st);

constexpr int kTrackTraceStride = 20;  // pose (12), gradient (6), L1 term, D-SSIM term
hipError_t launch_track_init(TrackState *s, const TrackPose &p0, hipStream_t st);
hipError_t launch_pose_left_update(const TrackPose &p0, const float *xi, float *pose, hipStream_t st);
hipError_t launch_track_step(TrackState *s, const TrackStepArgs &a, const int64_t *num_pairs, float *trace,
                             float *pose_out, hipStream_t st);

}  // namespace gs
