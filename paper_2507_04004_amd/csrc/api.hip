// C ABI of the rasterizer (declared in include/gs.h): argument checks, view tables,
// scratch layout, stage sequencing, and the batched plan with hipGraph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gs_internal.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char *where) {
  return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define GS_TRY_HIP(expr, where)                 \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// The kernels are built for gfx950 only: the current device's architecture is checked once per
// device before the first launch of an entry point (GS_ERR_UNSUPPORTED on any other).
int check_device() {
  constexpr int kMaxDevices = 64;
  static std::atomic<int> state[kMaxDevices];  // 0 unknown, 1 gfx950, 2 other
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  int s = (dev >= 0 && dev < kMaxDevices) ? state[dev].load(std::memory_order_relaxed) : 0;
  if (s == 0) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    s = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    if (dev >= 0 && dev < kMaxDevices) state[dev].store(s, std::memory_order_relaxed);
  }
  if (s != 1) return fail(GS_ERR_UNSUPPORTED, "device %d is not gfx950 (the only target this library is built for)", dev);
  return GS_OK;
}

#define GS_CHECK_DEVICE()            \
  do {                               \
    const int rc_ = check_device();  \
    if (rc_ != GS_OK) return rc_;    \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

bool side_ok(int s) { return s == 8 || s == 16 || s == 32; }
bool tile_ok(int tw, int th) { return side_ok(tw) && side_ok(th); }
bool depth_ok(int bd) { return bd == 32 || bd == 64 || bd == 128 || bd == 256; }

int check_camera(const gs_camera *c) {
  if (!c) return fail(GS_ERR_INVALID_ARG, "camera is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(GS_ERR_INVALID_ARG, "image size must be positive");
  if (c->w <= 0 || c->h <= 0) return fail(GS_ERR_INVALID_ARG, "render window must be non-empty");
  if (c->x0 < 0 || c->y0 < 0 || (int64_t)c->x0 + c->w > c->width || (int64_t)c->y0 + c->h > c->height)
    return fail(GS_ERR_INVALID_ARG, "render window (%d,%d,%d,%d) outside the %dx%d image", c->x0, c->y0, c->w, c->h,
                c->width, c->height);
  if (!(c->fx > 0.f) || !(c->fy > 0.f) || !std::isfinite(c->fx) || !std::isfinite(c->fy) ||
      !std::isfinite(c->cx) || !std::isfinite(c->cy))
    return fail(GS_ERR_INVALID_ARG, "intrinsics must be finite with fx, fy > 0");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->R_cw[i])) return fail(GS_ERR_INVALID_ARG, "rotation is not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->t_cw[i]) || !std::isfinite(c->bg[i]))
      return fail(GS_ERR_INVALID_ARG, "translation / background is not finite");
  if ((int64_t)c->width > 32767 * 8 || (int64_t)c->height > 32767 * 8)
    return fail(GS_ERR_INVALID_ARG, "image too large for int16 tile rectangles");
  return GS_OK;
}

int check_gaussians(const gs_gaussians *g) {
  if (!g) return fail(GS_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n < 0) return fail(GS_ERR_INVALID_ARG, "n < 0");
  if (g->sh_degree < 0 || g->sh_degree > 3) return fail(GS_ERR_INVALID_ARG, "sh_degree must be in 0..3");
  if (g->n > 0 && (!g->mean || !g->scale || !g->rot || !g->opacity || !g->sh_dc))
    return fail(GS_ERR_INVALID_ARG, "a parameter plane is NULL");
  if (g->n > 0 && g->sh_degree > 0 && !g->sh_rest) return fail(GS_ERR_INVALID_ARG, "sh_rest is NULL at degree > 0");
  if (g->n >= ((int64_t)1 << 30)) return fail(GS_ERR_INVALID_ARG, "n too large (at most 2^30 - 1 Gaussians)");
  return GS_OK;
}

// Record arrays may be NULL only when there are no records.
int check_projected(const gs_projected *p, int64_t n) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "projected records are NULL");
  if (n > 0 && (!p->card || !p->n_tiles || !p->dkey))
    return fail(GS_ERR_INVALID_ARG, "projected record pointer is NULL");
  if (n > 0 && (reinterpret_cast<uintptr_t>(p->card) & 63u))
    return fail(GS_ERR_INVALID_ARG, "splat cards must be 64-byte aligned");
  return GS_OK;
}

// Host view description: the camera plus the derived tile grid.
void make_view(const gs_camera &c, int tw, int th, uint32_t tile_base, uint32_t pix_base, gs::ViewCam &v) {
  v.fx = c.fx; v.fy = c.fy; v.cx = c.cx; v.cy = c.cy;
  for (int i = 0; i < 9; ++i) v.R[i] = c.R_cw[i];
  for (int i = 0; i < 3; ++i) v.t[i] = c.t_cw[i];
  for (int i = 0; i < 3; ++i) {
    // camera centre -R^T t, in float64 then rounded once
    double s = 0.0;
    for (int j = 0; j < 3; ++j) s += (double)c.R_cw[3 * j + i] * (double)c.t_cw[j];
    v.cw[i] = (float)(-s);
    v.bg[i] = c.bg[i];
  }
  v.W = c.width; v.H = c.height; v.x0 = c.x0; v.y0 = c.y0; v.w = c.w; v.h = c.h;
  v.tiles_x = (c.w + tw - 1) / tw;
  v.tiles_y = (c.h + th - 1) / th;
  v.tile_base = tile_base;
  v.pix_base = pix_base;
}

int make_table(const gs_camera *cams, int nv, int64_t n, int deg, int tw, int th, gs::ViewTable &vt) {
  std::memset(&vt, 0, sizeof vt);
  vt.n_views = nv;
  vt.tile_w = tw;
  vt.tile_h = th;
  vt.sh_degree = deg;
  vt.n = n;
  uint64_t tb = 0, pb = 0;
  for (int i = 0; i < nv; ++i) {
    int rc = check_camera(&cams[i]);
    if (rc) return rc;
    make_view(cams[i], tw, th, (uint32_t)tb, (uint32_t)pb, vt.v[i]);
    tb += (uint64_t)vt.v[i].tiles_x * vt.v[i].tiles_y;
    pb += (uint64_t)cams[i].w * cams[i].h;
  }
  if (tb > 0x7FFFFFFFull || pb > 0x7FFFFFFFull) return fail(GS_ERR_INVALID_ARG, "too many tiles or pixels");
  vt.total_tiles = (uint32_t)tb;
  return GS_OK;
}

// Backward scratch layout: grad2d [E][12] | pose partials [blocks][V][6] | gD, gO maps [pixels]
// | view-direction gradients [E] (float4).
struct GradScratch {
  float *g2, *pose_partial, *mapD, *mapO;
  float4 *gdir;
};

size_t grads_scratch_bytes_impl(int64_t n, int nv, int64_t pixels) {
  const int64_t E = std::max<int64_t>(n * nv, 1);
  size_t s = a256(sizeof(float) * 12 * E);
  s += a256(sizeof(float) * 6 * nv * std::max<int64_t>(gs::preprocess_bwd_blocks(n), 1));
  s += 2 * a256(sizeof(float) * std::max<int64_t>(pixels, 1));
  s += a256(sizeof(float4) * E);
  return s;
}

GradScratch carve_grads(void *base, int64_t n, int nv, int64_t pixels) {
  char *p = (char *)base;
  const int64_t E = std::max<int64_t>(n * nv, 1);
  GradScratch s;
  s.g2 = (float *)p;
  p += a256(sizeof(float) * 12 * E);
  s.pose_partial = (float *)p;
  p += a256(sizeof(float) * 6 * nv * std::max<int64_t>(gs::preprocess_bwd_blocks(n), 1));
  s.mapD = (float *)p;
  p += a256(sizeof(float) * std::max<int64_t>(pixels, 1));
  s.mapO = (float *)p;
  p += a256(sizeof(float) * std::max<int64_t>(pixels, 1));
  s.gdir = (float4 *)p;
  return s;
}

struct ViewIO {
  gs_image img;
  const float *dC, *dD, *dO;
  gs_lidar lidar;
  float *pose;
};

// The backward of all views of one table: dense gradient maps (user planes + LiDAR term),
// blend backward into grad2d, then the chain rule to parameters and poses.
int enqueue_backward(const gs::ViewTable &vt, const gs_gaussians &g, const gs_projected &p, const uint32_t *vals,
                     const uint32_t *range, void *state, int64_t cap, const ViewIO *io, int bd, const gs_grads &out,
                     const GradScratch &s, hipStream_t st) {
  const int nv = vt.n_views;
  gs::ImgTable it{};
  gs::GradTable gtab{};
  gs::LidarTable lt{};
  gs::MapSrc src{};
  gs::MapTable dst{};
  lt.n_views = nv;
  int max_m = 0;
  int64_t max_npx = 0;
  bool any_map = false;
  for (int i = 0; i < nv; ++i) {
    it.v[i] = {io[i].img.color, io[i].img.depth, io[i].img.alpha, io[i].img.t_final, io[i].img.last,
               io[i].img.n_contrib};
    const int64_t npx = (int64_t)vt.v[i].w * vt.v[i].h;
    const bool has_lidar = io[i].lidar.m > 0;
    const bool need_map = has_lidar || io[i].dD || io[i].dO;
    gtab.v[i].gC = io[i].dC;
    if (need_map) {
      any_map = true;
      dst.gD[i] = s.mapD + vt.v[i].pix_base;
      dst.gO[i] = s.mapO + vt.v[i].pix_base;
      src.gD[i] = io[i].dD;
      src.gO[i] = io[i].dO;
      src.npx[i] = npx;
      gtab.v[i].gD = dst.gD[i];
      gtab.v[i].gO = dst.gO[i];
      max_npx = std::max(max_npx, npx);
    }
    if (has_lidar) {
      lt.v[i] = {io[i].lidar.pix, io[i].lidar.depth_target, io[i].lidar.grad_scale, io[i].lidar.loss_out,
                 io[i].lidar.weight, io[i].lidar.m, (int32_t)npx};
      max_m = std::max(max_m, io[i].lidar.m);
    }
  }
  GS_TRY_HIP(gs::launch_bwd_prep(s.g2, 12 * vt.n * nv, src, dst, nv, any_map ? max_npx : 0, lt, it, max_m, st),
             "grad2d and gradient maps");
  gs::profile_begin(GS_STAGE_BLEND_BWD, st);
  GS_TRY_HIP(gs::launch_blend_bwd(bd, vt, it, gtab, p, vals, range, state, cap, s.g2, st, out.schedule),
             "blend backward");
  gs::profile_end(GS_STAGE_BLEND_BWD, st);
  float *pose_out[gs::kMaxViews] = {};
  for (int i = 0; i < nv; ++i) pose_out[i] = io[i].pose;
  gs::profile_begin(GS_STAGE_PREPROCESS_BWD, st);
  GS_TRY_HIP(gs::launch_preprocess_bwd(vt, g, p, s.g2, s.gdir, out, pose_out, s.pose_partial, st),
             "preprocess backward");
  gs::profile_end(GS_STAGE_PREPROCESS_BWD, st);
  return GS_OK;
}

int check_schedule(int32_t schedule, int tile_w, int tile_h) {
  if (schedule != GS_BWD_CHUNKS && schedule != GS_BWD_BUCKETS)
    return fail(GS_ERR_INVALID_ARG, "unknown backward schedule %d", schedule);
  if (schedule == GS_BWD_BUCKETS && tile_w * tile_h > 256)
    return fail(GS_ERR_UNSUPPORTED, "the bucketed backward runs on tiles of at most 256 pixels");
  return GS_OK;
}

int check_lidar(const gs_lidar *l, int64_t npx) {
  if (!l || l->m == 0) return GS_OK;
  if (l->m < 0) return fail(GS_ERR_INVALID_ARG, "lidar m < 0");
  if (!l->pix || !l->depth_target) return fail(GS_ERR_INVALID_ARG, "lidar arrays are NULL");
  if (!std::isfinite(l->weight)) return fail(GS_ERR_INVALID_ARG, "lidar weight is not finite");
  (void)npx;
  return GS_OK;
}

int check_image(const gs_image *im) {
  if (!im || !im->color || !im->depth || !im->alpha || !im->t_final || !im->last)
    return fail(GS_ERR_INVALID_ARG, "image plane is NULL");
  return GS_OK;
}

int check_state(const gs_image *im, int64_t cap, int64_t tiles, int tw, int th, int bd) {
  const size_t need = gs::blend_state_bytes(tiles, cap, tw, th, bd);
  if (!im->state || im->state_bytes < need)
    return fail(GS_ERR_INVALID_ARG, "image state too small: %zu < %zu", im->state ? im->state_bytes : (size_t)0, need);
  return GS_OK;
}

struct StageProfile {
  std::vector<hipEvent_t> begin, end;
  int used = 0;
  bool open = false;
};
thread_local uint32_t g_prof_mask = 0;
thread_local StageProfile g_prof[GS_NUM_STAGES];

}  // namespace

namespace gs {
void profile_begin(int stage, hipStream_t st) {
  if (!(g_prof_mask & (1u << stage))) return;
  StageProfile &p = g_prof[stage];
  if (p.used >= (int)p.begin.size()) return;
  (void)hipEventRecord(p.begin[p.used], st);
  p.open = true;
}
void profile_end(int stage, hipStream_t st) {
  if (!(g_prof_mask & (1u << stage))) return;
  StageProfile &p = g_prof[stage];
  if (!p.open) return;
  (void)hipEventRecord(p.end[p.used], st);
  p.used++;
  p.open = false;
}
}  // namespace gs

extern "C" {

const char *gs_last_error(void) { return g_err; }

void gs_profile_disable(void) {
  for (auto &p : g_prof) {
    for (auto e : p.begin) (void)hipEventDestroy(e);
    for (auto e : p.end) (void)hipEventDestroy(e);
    p = StageProfile();
  }
  g_prof_mask = 0;
}

int gs_profile_enable(uint32_t stage_mask, int32_t max_records) {
  if (max_records <= 0 || max_records > 1000000) return fail(GS_ERR_INVALID_ARG, "max_records out of range");
  gs_profile_disable();
  for (int s = 0; s < GS_NUM_STAGES; ++s) {
    if (!(stage_mask & (1u << s))) continue;
    StageProfile &p = g_prof[s];
    p.begin.resize(max_records);
    p.end.resize(max_records);
    for (int i = 0; i < max_records; ++i) {
      GS_TRY_HIP(hipEventCreate(&p.begin[i]), "event create");
      GS_TRY_HIP(hipEventCreate(&p.end[i]), "event create");
    }
  }
  g_prof_mask = stage_mask;
  return GS_OK;
}

int gs_profile_read(int32_t stage, double *total_ms, int32_t *count) {
  if (stage < 0 || stage >= GS_NUM_STAGES || !total_ms || !count) return fail(GS_ERR_INVALID_ARG, "bad argument");
  StageProfile &p = g_prof[stage];
  double tot = 0.0;
  for (int i = 0; i < p.used; ++i) {
    GS_TRY_HIP(hipEventSynchronize(p.end[i]), "event sync");
    float ms = 0.f;
    GS_TRY_HIP(hipEventElapsedTime(&ms, p.begin[i], p.end[i]), "event elapsed");
    tot += ms;
  }
  *total_ms = tot;
  *count = p.used;
  p.used = 0;
  return GS_OK;
}

size_t gs_bins_scratch_bytes(int64_t n, int64_t capacity, int64_t num_tiles) {
  (void)num_tiles;
  return gs::bin_scratch_bytes(std::max<int64_t>(n, 0), std::max<int64_t>(capacity, 0));
}

size_t gs_image_state_bytes(int64_t capacity, int64_t num_tiles, int32_t tile_w, int32_t tile_h, int32_t blend_depth) {
  if (capacity < 0 || num_tiles < 0 || !tile_ok(tile_w, tile_h) || !depth_ok(blend_depth)) return 0;
  return gs::blend_state_bytes(num_tiles, capacity, tile_w, tile_h, blend_depth);
}

size_t gs_grads_scratch_bytes(int64_t n, int32_t n_views, int64_t total_window_pixels) {
  return grads_scratch_bytes_impl(std::max<int64_t>(n, 0), std::max(n_views, 1), std::max<int64_t>(total_window_pixels, 0));
}

int gs_preprocess(const gs_gaussians *g, const gs_camera *cam, int32_t tile_w, int32_t tile_h, gs_projected *out,
                  gs_stream_t stream) {
  int rc;
  if ((rc = check_gaussians(g)) || (rc = check_camera(cam)) || (rc = check_projected(out, g->n))) return rc;
  if (!tile_ok(tile_w, tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  gs::ViewTable vt;
  if ((rc = make_table(cam, 1, g->n, g->sh_degree, tile_w, tile_h, vt))) return rc;
  vt.pose_dev = out->pose;
  gs::profile_begin(GS_STAGE_PREPROCESS, (hipStream_t)stream);
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_preprocess(vt, *g, *out, (hipStream_t)stream), "preprocess");
  gs::profile_end(GS_STAGE_PREPROCESS, (hipStream_t)stream);
  return GS_OK;
}

int gs_bin_sort(const gs_projected *proj, int64_t n, const gs_camera *cam, gs_bins *io, gs_stream_t stream) {
  int rc;
  if ((rc = check_projected(proj, n)) || (rc = check_camera(cam))) return rc;
  if (!io || !io->vals || !io->tile_range || !io->num_pairs || !io->scratch)
    return fail(GS_ERR_INVALID_ARG, "bins pointer is NULL");
  if (n < 0 || io->capacity < 0) return fail(GS_ERR_INVALID_ARG, "negative size");
  if (!tile_ok(io->tile_w, io->tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  if (io->capacity > 0xFFFFFFFFll) return fail(GS_ERR_INVALID_ARG, "capacity too large");
  gs::ViewTable vt;
  if ((rc = make_table(cam, 1, n, 0, io->tile_w, io->tile_h, vt))) return rc;
  if (io->scratch_bytes < gs::bin_scratch_bytes(n, io->capacity))
    return fail(GS_ERR_INVALID_ARG, "bins scratch too small: %zu < %zu", io->scratch_bytes,
                gs::bin_scratch_bytes(n, io->capacity));
  gs::profile_begin(GS_STAGE_BIN_SORT, (hipStream_t)stream);
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_bin_sort(vt, *proj, n, io->capacity, io->vals, io->tile_range, io->num_pairs, io->scratch,
                                 (hipStream_t)stream),
             "bin/sort");
  gs::profile_end(GS_STAGE_BIN_SORT, (hipStream_t)stream);
  return GS_OK;
}

int gs_render_fwd(const gs_projected *proj, int64_t n, const gs_bins *bins, const gs_camera *cam, int32_t blend_depth,
                  const gs_lidar *lidar, gs_image *out, gs_stream_t stream) {
  int rc;
  if ((rc = check_projected(proj, n)) || (rc = check_camera(cam)) || (rc = check_image(out))) return rc;
  if (!bins || !bins->vals || !bins->tile_range) return fail(GS_ERR_INVALID_ARG, "bins pointer is NULL");
  if (!tile_ok(bins->tile_w, bins->tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  if (!depth_ok(blend_depth)) return fail(GS_ERR_INVALID_ARG, "blend_depth must be 32, 64, 128 or 256");
  if ((rc = check_lidar(lidar, (int64_t)cam->w * cam->h))) return rc;
  if (lidar && lidar->m > 0 && !lidar->loss_out) return fail(GS_ERR_INVALID_ARG, "lidar loss_out is NULL");
  gs::ViewTable vt;
  if ((rc = make_table(cam, 1, n, 0, bins->tile_w, bins->tile_h, vt))) return rc;
  if ((rc = check_state(out, bins->capacity, vt.total_tiles, bins->tile_w, bins->tile_h, blend_depth))) return rc;
  gs::ImgTable it{};
  it.v[0] = {out->color, out->depth, out->alpha, out->t_final, out->last, out->n_contrib};
  hipStream_t st = (hipStream_t)stream;
  gs::profile_begin(GS_STAGE_BLEND_FWD, st);
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_blend_fwd(blend_depth, vt, it, *proj, bins->vals, bins->tile_range, out->state,
                                  bins->capacity, st),
             "blend forward");
  gs::profile_end(GS_STAGE_BLEND_FWD, st);
  if (lidar && lidar->m > 0) {
    gs::LidarTable lt{};
    lt.n_views = 1;
    lt.v[0] = {lidar->pix, lidar->depth_target, lidar->grad_scale, lidar->loss_out, lidar->weight, lidar->m, (int32_t)((int64_t)cam->w * cam->h)};
    GS_TRY_HIP(gs::launch_lidar_loss(lt, it, lidar->m, st), "lidar loss");
  }
  return GS_OK;
}

}  // extern "C"

namespace {

// Checks shared by gs_render_bwd and gs_render_bwd_noalloc (everything except the scratch),
// and the view table of the call.
int check_bwd(const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj, const gs_bins *bins,
              const gs_image *fwd, const float *dL_dC, const gs_lidar *lidar, int32_t blend_depth,
              const gs_grads *out, gs::ViewTable &vt) {
  int rc;
  if ((rc = check_gaussians(g)) || (rc = check_camera(cam)) || (rc = check_projected(proj, g->n)) ||
      (rc = check_image(fwd)))
    return rc;
  if (!bins || !bins->vals || !bins->tile_range) return fail(GS_ERR_INVALID_ARG, "bins pointer is NULL");
  if (!tile_ok(bins->tile_w, bins->tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  if (!depth_ok(blend_depth)) return fail(GS_ERR_INVALID_ARG, "blend_depth must be 32, 64, 128 or 256");
  if (!dL_dC) return fail(GS_ERR_INVALID_ARG, "dL_dC is NULL");
  if (!out) return fail(GS_ERR_INVALID_ARG, "grads is NULL");
  if (out->sh_dc && g->sh_degree > 0 && !out->sh_rest) return fail(GS_ERR_INVALID_ARG, "grads.sh_rest is NULL");
  if ((rc = check_schedule(out->schedule, bins->tile_w, bins->tile_h))) return rc;
  if ((rc = check_lidar(lidar, (int64_t)cam->w * cam->h))) return rc;
  if ((rc = make_table(cam, 1, g->n, g->sh_degree, bins->tile_w, bins->tile_h, vt))) return rc;
  vt.pose_dev = proj->pose;
  return check_state(fwd, bins->capacity, vt.total_tiles, bins->tile_w, bins->tile_h, blend_depth);
}

int run_bwd(const gs::ViewTable &vt, const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj,
            const gs_bins *bins, const gs_image *fwd, const float *dL_dC, const float *dL_dD, const float *dL_dO,
            const gs_lidar *lidar, int32_t blend_depth, const gs_grads *out, void *scratch_base, hipStream_t st) {
  ViewIO io{};
  io.img = *fwd;
  io.dC = dL_dC;
  io.dD = dL_dD;
  io.dO = dL_dO;
  if (lidar) io.lidar = *lidar;
  io.pose = out->pose;
  const GradScratch s = carve_grads(scratch_base, g->n, 1, (int64_t)cam->w * cam->h);
  return enqueue_backward(vt, *g, *proj, bins->vals, bins->tile_range, fwd->state, bins->capacity, &io, blend_depth,
                          *out, s, st);
}

}  // namespace

// The backward scratch of gs_render_bwd_noalloc: one array per device, held by the loaded code
// object until the process ends. Host code never names it: its device address is resolved
// once per device (noalloc_scratch) and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
std::atomic<void *> g_noalloc_ptr[kNoAllocDevices];

// Device address of the scratch array on the current device.
int noalloc_scratch(void **out) {
  int dev = 0;
  GS_TRY_HIP(hipGetDevice(&dev), "current device");
  if (dev < 0 || dev >= kNoAllocDevices) return fail(GS_ERR_UNSUPPORTED, "device index %d out of range", dev);
  void *p = g_noalloc_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    p = g_noalloc_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      GS_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the no-allocation scratch");
      if (!p) return fail(GS_ERR_HIP, "address of the no-allocation scratch is NULL");
      g_noalloc_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return GS_OK;
}

}  // namespace

extern "C" {

int gs_render_bwd(const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj, const gs_bins *bins,
                  const gs_image *fwd, const float *dL_dC, const float *dL_dD, const float *dL_dO, const gs_lidar *lidar,
                  int32_t blend_depth, gs_grads *out, gs_stream_t stream) {
  gs::ViewTable vt;
  int rc;
  if ((rc = check_bwd(g, cam, proj, bins, fwd, dL_dC, lidar, blend_depth, out, vt))) return rc;
  if (!out->scratch) return fail(GS_ERR_INVALID_ARG, "grads scratch is NULL");
  const size_t need = grads_scratch_bytes_impl(g->n, 1, (int64_t)cam->w * cam->h);
  if (out->scratch_bytes < need)
    return fail(GS_ERR_INVALID_ARG, "grads scratch too small: %zu < %zu", out->scratch_bytes, need);
  GS_CHECK_DEVICE();
  return run_bwd(vt, g, cam, proj, bins, fwd, dL_dC, dL_dD, dL_dO, lidar, blend_depth, out, out->scratch,
                 (hipStream_t)stream);
}

int gs_render_bwd_noalloc(const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj, const gs_bins *bins,
                          const gs_image *fwd, const float *dL_dC, const float *dL_dD, const float *dL_dO,
                          const gs_lidar *lidar, int32_t blend_depth, gs_grads *out, gs_stream_t stream) {
  gs::ViewTable vt;
  int rc;
  if ((rc = check_bwd(g, cam, proj, bins, fwd, dL_dC, lidar, blend_depth, out, vt))) return rc;
  const size_t need = grads_scratch_bytes_impl(g->n, 1, (int64_t)cam->w * cam->h);
  if (need > (size_t)GS_NOALLOC_SCRATCH_BYTES)
    return fail(GS_ERR_INVALID_ARG,
                "backward scratch of %zu bytes (%lld Gaussians, %lld pixels) exceeds the no-allocation limit of %zu",
                need, (long long)g->n, (long long)cam->w * cam->h, (size_t)GS_NOALLOC_SCRATCH_BYTES);
  GS_CHECK_DEVICE();
  void *base = nullptr;
  if ((rc = noalloc_scratch(&base))) return rc;
  return run_bwd(vt, g, cam, proj, bins, fwd, dL_dC, dL_dD, dL_dO, lidar, blend_depth, out, base,
                 (hipStream_t)stream);
}

int gs_camera_left_update(const gs_camera *in, const float xi[6], gs_camera *out) {
  if (!in || !xi || !out) return fail(GS_ERR_INVALID_ARG, "NULL argument");
  const double rho[3] = {xi[0], xi[1], xi[2]}, phi[3] = {xi[3], xi[4], xi[5]};
  const double th = std::sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  // Rodrigues: R = I + A K + B K^2, V = I + B K + C K^2 (series near zero)
  double A, B, Cc;
  if (th < 1e-4) {
    A = 1.0 - th * th / 6.0;
    B = 0.5 - th * th / 24.0;
    Cc = 1.0 / 6.0 - th * th / 120.0;
  } else {
    A = std::sin(th) / th;
    B = (1.0 - std::cos(th)) / (th * th);
    Cc = (th - std::sin(th)) / (th * th * th);
  }
  double dR[9], V[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    dR[i] = I + A * K[i] + B * K2[i];
    V[i] = I + B * K[i] + Cc * K2[i];
  }
  gs_camera o = *in;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += dR[3 * i + l] * (double)in->R_cw[3 * l + j];
      o.R_cw[3 * i + j] = (float)s;
    }
    double s = 0.0;
    for (int l = 0; l < 3; ++l) s += dR[3 * i + l] * (double)in->t_cw[l] + V[3 * i + l] * rho[l];
    o.t_cw[i] = (float)s;
  }
  *out = o;
  return GS_OK;
}

int gs_pose_left_update(const gs_camera *cam, const float *xi, float *pose_out, gs_stream_t stream) {
  int rc;
  if ((rc = check_camera(cam))) return rc;
  if (!xi || !pose_out) return fail(GS_ERR_INVALID_ARG, "NULL argument");
  gs::TrackPose p0;
  for (int i = 0; i < 9; ++i) p0.R[i] = cam->R_cw[i];
  for (int i = 0; i < 3; ++i) p0.t[i] = cam->t_cw[i];
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_pose_left_update(p0, xi, pose_out, (hipStream_t)stream), "pose update");
  return GS_OK;
}

size_t gs_dssim_scratch_bytes(int32_t channels, int32_t h, int32_t w) {
  if (channels < 0 || h < 0 || w < 0) return 0;
  return gs::dssim_scratch_bytes(channels, h, w);
}

int gs_loss_dssim(const float *color, const float *target, int32_t channels, int32_t h, int32_t w, float weight,
                  float *dL_dC, float *loss_out, void *scratch, size_t scratch_bytes, gs_stream_t stream) {
  if (channels < 0 || h < 0 || w < 0) return fail(GS_ERR_INVALID_ARG, "image size must be non-negative");
  if ((int64_t)channels * h * w >= (int64_t(1) << 31) || channels > 64 || h > 32768 || w > 32768)
    return fail(GS_ERR_INVALID_ARG, "image too large (at most 64 channels of 32768 x 32768, 2^31 values)");
  const int64_t n = (int64_t)channels * h * w;
  if (n > 0 && (!color || !target)) return fail(GS_ERR_INVALID_ARG, "color / target is NULL");
  if (!std::isfinite(weight)) return fail(GS_ERR_INVALID_ARG, "weight is not finite");
  if (n > 0 && (!scratch || scratch_bytes < gs::dssim_scratch_bytes(channels, h, w)))
    return fail(GS_ERR_INVALID_ARG, "scratch must hold gs_dssim_scratch_bytes bytes");
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_dssim(color, target, channels, h, w, weight, dL_dC, loss_out, (float *)scratch,
                              (hipStream_t)stream),
             "d-ssim");
  return GS_OK;
}

int gs_adam_sparse(const gs_adam *a, gs_stream_t stream) {
  if (!a) return fail(GS_ERR_INVALID_ARG, "adam arguments are NULL");
  if (a->n < 0 || a->n >= (int64_t(1) << 30)) return fail(GS_ERR_INVALID_ARG, "n must be in [0, 2^30)");
  if (a->n_groups < 0 || a->n_groups > GS_ADAM_MAX_GROUPS)
    return fail(GS_ERR_INVALID_ARG, "n_groups must be in [0, %d]", GS_ADAM_MAX_GROUPS);
  if (a->visible && (a->n_views < 1 || a->n_views > GS_MAX_VIEWS))
    return fail(GS_ERR_INVALID_ARG, "n_views must be in [1, %d]", GS_MAX_VIEWS);
  if (!(a->beta1 >= 0.f && a->beta1 < 1.f) || !(a->beta2 >= 0.f && a->beta2 < 1.f))
    return fail(GS_ERR_INVALID_ARG, "betas must be in [0, 1)");
  if (!(a->eps >= 0.f) || !std::isfinite(a->eps)) return fail(GS_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (!(a->bias1 > 0.f && a->bias1 <= 1.f) || !(a->bias2 > 0.f && a->bias2 <= 1.f))
    return fail(GS_ERR_INVALID_ARG, "bias terms must be in (0, 1]");
  gs::AdamArgs d{};
  d.n = a->n;
  d.n_groups = a->n_groups;
  d.n_views = a->visible ? a->n_views : 0;
  d.visible = a->visible;
  d.beta1 = a->beta1;
  d.beta2 = a->beta2;
  d.eps = a->eps;
  d.sqrt_bias2 = (float)std::sqrt((double)a->bias2);
  for (int i = 0; i < a->n_groups; ++i) {
    const gs_adam_group &G = a->group[i];
    if (G.k < 0) return fail(GS_ERR_INVALID_ARG, "group %d: k < 0", i);
    if (G.act != GS_ACT_NONE && G.act != GS_ACT_EXP && G.act != GS_ACT_SIGMOID)
      return fail(GS_ERR_INVALID_ARG, "group %d: unknown activation %d", i, G.act);
    if (G.k > 0 && a->n > 0 && (!G.param || !G.exp_avg || !G.exp_avg_sq || !G.grad))
      return fail(GS_ERR_INVALID_ARG, "group %d: a plane is NULL", i);
    if (!std::isfinite(G.lr)) return fail(GS_ERR_INVALID_ARG, "group %d: lr is not finite", i);
    d.group[i] = gs::AdamGroupDev{G.param, G.exp_avg, G.exp_avg_sq, G.grad,
                                  G.act == GS_ACT_NONE ? nullptr : G.act_out, G.k, G.act,
                                  (float)((double)G.lr / (double)a->bias1)};
  }
  if (a->n == 0 || a->n_groups == 0) return GS_OK;  // nothing to launch
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_adam_sparse(d, (hipStream_t)stream), "sparse adam");
  return GS_OK;
}

int gs_loss_l1(const float *color, const float *target, int64_t n_values, float weight, float *dL_dC, float *loss_out,
               gs_stream_t stream) {
  if (n_values < 0) return fail(GS_ERR_INVALID_ARG, "n_values < 0");
  if (n_values > 0 && (!color || !target)) return fail(GS_ERR_INVALID_ARG, "color / target is NULL");
  if (!std::isfinite(weight)) return fail(GS_ERR_INVALID_ARG, "weight is not finite");
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_loss_l1(color, target, n_values, weight, dL_dC, loss_out, (hipStream_t)stream), "l1 loss");
  return GS_OK;
}

}  // extern "C"

// =============================================================================================
// Batched plan: one launch per stage over all views, optional hipGraph replay.
// =============================================================================================
struct gs_batch_plan {
  int64_t n = 0;
  int32_t deg = 0, max_views = 0, tw = 16, th = 16, bd = 256;
  int64_t max_pixels = 0, cap = 0, max_tiles = 0;
  bool fwd_only = false;
  // owned device memory
  void *block = nullptr;
  gs_projected proj{};
  uint32_t *vals = nullptr, *tile_range = nullptr;
  int64_t *num_pairs = nullptr;
  void *bin_scratch = nullptr;
  void *grad_scratch = nullptr;
  float *dC = nullptr;  // fused L1 gradient planes, concatenated over views
  void *blend_state = nullptr;
  // graph: captured on the plan's own stream (capture is not allowed on the legacy null
  // stream), launched on the caller's stream
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> signature;
};

namespace {

size_t plan_bytes(const gs_batch_plan &p, size_t *offs) {
  const int64_t E = std::max<int64_t>(p.n * p.max_views, 1);
  size_t o = 0;
  auto put = [&](int i, size_t bytes) {
    offs[i] = o;
    o += a256(bytes);
  };
  put(0, 64 * E);                                      // splat cards
  put(1, 4 * E);                                       // n_tiles
  put(2, 4 * E);                                       // dkey
  put(3, 4 * std::max<int64_t>(p.cap, 1));             // vals
  put(4, 8 * std::max<int64_t>(p.max_tiles, 1));       // tile ranges
  put(5, 16);                                          // num_pairs
  put(6, gs::bin_scratch_bytes(E, p.cap));             // bin scratch
  put(7, p.fwd_only ? 0 : grads_scratch_bytes_impl(p.n, p.max_views, p.max_pixels));
  put(8, p.fwd_only ? 0 : 12 * std::max<int64_t>(p.max_pixels, 1));  // dC planes
  put(9, gs::blend_state_bytes(p.max_tiles, p.cap, p.tw, p.th, p.bd));
  return o;
}

int enqueue_batch(gs_batch_plan *p, const gs_gaussians *g, int nv, const gs_view *views, uint32_t mode,
                  gs_grads *grads, hipStream_t st) {
  std::vector<gs_camera> cams(nv);
  for (int i = 0; i < nv; ++i) cams[i] = views[i].cam;
  gs::ViewTable vt;
  int rc = make_table(cams.data(), nv, g->n, g->sh_degree, p->tw, p->th, vt);
  if (rc) return rc;
  if ((int64_t)vt.total_tiles > p->max_tiles) return fail(GS_ERR_INVALID_ARG, "views need more tiles than the plan holds");
  int64_t pixels = 0;
  for (int i = 0; i < nv; ++i) pixels += (int64_t)cams[i].w * cams[i].h;
  if (pixels > p->max_pixels) return fail(GS_ERR_INVALID_ARG, "views exceed the plan's pixel budget");
  const int64_t E = g->n * nv;
  gs::ImgTable it{};
  for (int i = 0; i < nv; ++i) {
    const gs_image &im = views[i].out;
    it.v[i] = {im.color, im.depth, im.alpha, im.t_final, im.last, im.n_contrib};
  }
  if (mode & GS_FWD) {
    gs::profile_begin(GS_STAGE_PREPROCESS, st);
    GS_TRY_HIP(gs::launch_preprocess(vt, *g, p->proj, st), "batch preprocess");
    gs::profile_end(GS_STAGE_PREPROCESS, st);
    gs::profile_begin(GS_STAGE_BIN_SORT, st);
    GS_TRY_HIP(gs::launch_bin_sort(vt, p->proj, E, p->cap, p->vals, p->tile_range, p->num_pairs, p->bin_scratch, st),
               "batch bin/sort");
    gs::profile_end(GS_STAGE_BIN_SORT, st);
    gs::profile_begin(GS_STAGE_BLEND_FWD, st);
    GS_TRY_HIP(gs::launch_blend_fwd(p->bd, vt, it, p->proj, p->vals, p->tile_range, p->blend_state, p->cap, st),
               "batch blend forward");
    gs::profile_end(GS_STAGE_BLEND_FWD, st);
    gs::LidarTable lt{};
    lt.n_views = nv;
    int max_m = 0;
    for (int i = 0; i < nv; ++i) {
      const gs_lidar &l = views[i].lidar;
      if (l.m > 0 && l.loss_out) {
        lt.v[i] = {l.pix, l.depth_target, l.grad_scale, l.loss_out, l.weight, l.m, cams[i].w * cams[i].h};
        max_m = std::max(max_m, l.m);
      }
    }
    if (max_m > 0) GS_TRY_HIP(gs::launch_lidar_loss(lt, it, max_m, st), "batch lidar loss");
  }
  if (mode & GS_BWD) {
    std::vector<ViewIO> io(nv);
    for (int i = 0; i < nv; ++i) {
      const gs_view &v = views[i];
      io[i].img = v.out;
      io[i].dC = v.dL_dC;
      if (v.target) {
        float *dc = p->dC + 3 * (int64_t)vt.v[i].pix_base;
        const int64_t nval = 3 * (int64_t)v.cam.w * v.cam.h;
        GS_TRY_HIP(gs::launch_loss_l1(v.out.color, v.target, nval, v.rgb_weight, dc, v.rgb_loss_out, st),
                   "batch l1 loss");
        io[i].dC = dc;
      }
      io[i].dD = v.dL_dD;
      io[i].dO = v.dL_dO;
      io[i].lidar = v.lidar;
      io[i].pose = v.pose_grad;
    }
    gs_grads gg{};
    if (grads) gg = *grads;
    GradScratch s = carve_grads(p->grad_scratch, g->n, nv, p->max_pixels);
    rc = enqueue_backward(vt, *g, p->proj, p->vals, p->tile_range, p->blend_state, p->cap, io.data(), p->bd, gg, s,
                          st);
    if (rc) return rc;
  }
  return GS_OK;
}

int check_views(const gs_batch_plan *p, const gs_gaussians *g, int nv, const gs_view *views, uint32_t mode,
                const gs_grads *grads) {
  int rc;
  if ((rc = check_gaussians(g))) return rc;
  if (g->n > p->n) return fail(GS_ERR_INVALID_ARG, "map has more Gaussians than the plan");
  if (g->sh_degree > p->deg) return fail(GS_ERR_INVALID_ARG, "SH degree above the plan's");
  if (nv <= 0 || nv > p->max_views) return fail(GS_ERR_INVALID_ARG, "n_views must be in 1..%d", p->max_views);
  if (!views) return fail(GS_ERR_INVALID_ARG, "views is NULL");
  if (!(mode & (GS_FWD | GS_BWD))) return fail(GS_ERR_INVALID_ARG, "mode needs GS_FWD and/or GS_BWD");
  if ((mode & GS_BWD) && p->fwd_only) return fail(GS_ERR_INVALID_ARG, "the plan was created forward-only");
  for (int i = 0; i < nv; ++i) {
    if ((rc = check_camera(&views[i].cam)) || (rc = check_image(&views[i].out))) return rc;
    if ((rc = check_lidar(&views[i].lidar, (int64_t)views[i].cam.w * views[i].cam.h))) return rc;
    if ((mode & GS_BWD) && !views[i].dL_dC && !views[i].target)
      return fail(GS_ERR_INVALID_ARG, "view %d has neither dL_dC nor a target", i);
  }
  if ((mode & GS_BWD) && grads && grads->sh_dc && g->sh_degree > 0 && !grads->sh_rest)
    return fail(GS_ERR_INVALID_ARG, "grads.sh_rest is NULL");
  if ((mode & GS_BWD) && grads && (rc = check_schedule(grads->schedule, p->tw, p->th))) return rc;
  return GS_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Arguments of a batch plan, checked; fills the plan's sizes.
int plan_args(int64_t n, int32_t sh_degree, int32_t n_views, int64_t max_total_pixels, int32_t tile_w, int32_t tile_h,
              int32_t blend_depth, int64_t capacity, uint32_t flags, gs_batch_plan &p) {
  if (n < 0 || n > 0x7FFFFFFF || sh_degree < 0 || sh_degree > 3) return fail(GS_ERR_INVALID_ARG, "bad n or degree");
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARG, "n_views must be in 1..%d", GS_MAX_VIEWS);
  if (n * n_views > 0xFFFFFFFFll) return fail(GS_ERR_INVALID_ARG, "n * n_views too large");
  if (!tile_ok(tile_w, tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  if (!depth_ok(blend_depth)) return fail(GS_ERR_INVALID_ARG, "blend_depth must be 32, 64, 128 or 256");
  if (max_total_pixels <= 0 || capacity <= 0 || capacity > 0xFFFFFFFFll)
    return fail(GS_ERR_INVALID_ARG, "bad pixel budget or capacity");
  if (flags & ~(uint32_t)GS_PLAN_FWD_ONLY) return fail(GS_ERR_INVALID_ARG, "unknown plan flags 0x%x", flags);
  p.n = n;
  p.deg = sh_degree;
  p.max_views = n_views;
  p.max_pixels = max_total_pixels;
  p.tw = tile_w;
  p.th = tile_h;
  p.bd = blend_depth;
  p.cap = capacity;
  p.fwd_only = (flags & GS_PLAN_FWD_ONLY) != 0;
  // every view adds at most one partial tile row and column beyond pixels / tile area
  p.max_tiles = max_total_pixels / ((int64_t)tile_w * tile_h) + (int64_t)n_views * (32768 / tile_w + 32768 / tile_h + 1);
  return GS_OK;
}

}  // namespace

extern "C" {

size_t gs_batch_plan_bytes(int64_t n, int32_t sh_degree, int32_t n_views, int64_t max_total_pixels, int32_t tile_w,
                           int32_t tile_h, int32_t blend_depth, int64_t capacity, uint32_t flags) {
  gs_batch_plan p;
  if (plan_args(n, sh_degree, n_views, max_total_pixels, tile_w, tile_h, blend_depth, capacity, flags, p)) return 0;
  size_t offs[10];
  return plan_bytes(p, offs);
}

int gs_batch_plan_create(gs_batch_plan **out, int64_t n, int32_t sh_degree, int32_t n_views, int64_t max_total_pixels,
                         int32_t tile_w, int32_t tile_h, int32_t blend_depth, int64_t capacity, uint32_t flags) {
  if (!out) return fail(GS_ERR_INVALID_ARG, "plan out-pointer is NULL");
  *out = nullptr;
  gs_batch_plan args;
  int rc;
  if ((rc = plan_args(n, sh_degree, n_views, max_total_pixels, tile_w, tile_h, blend_depth, capacity, flags, args)))
    return rc;
  GS_CHECK_DEVICE();
  gs_batch_plan *p = new gs_batch_plan(args);
  size_t offs[10];
  const size_t bytes = plan_bytes(*p, offs);
  hipError_t e = hipMalloc(&p->block, bytes);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "plan allocation");
  }
  char *b = (char *)p->block;
  p->proj.card = (float *)(b + offs[0]);
  p->proj.n_tiles = (uint32_t *)(b + offs[1]);
  p->proj.dkey = (uint32_t *)(b + offs[2]);
  p->vals = (uint32_t *)(b + offs[3]);
  p->tile_range = (uint32_t *)(b + offs[4]);
  p->num_pairs = (int64_t *)(b + offs[5]);
  p->bin_scratch = b + offs[6];
  p->grad_scratch = b + offs[7];
  p->dC = (float *)(b + offs[8]);
  p->blend_state = b + offs[9];
  *out = p;
  return GS_OK;
}

void gs_batch_plan_destroy(gs_batch_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->block) (void)hipFree(p->block);
  delete p;
}

int gs_batch_num_pairs(const gs_batch_plan *p, int64_t *required, gs_stream_t stream) {
  if (!p || !required) return fail(GS_ERR_INVALID_ARG, "NULL argument");
  GS_TRY_HIP(hipMemcpyAsync(required, p->num_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, (hipStream_t)stream),
             "copy pair count");
  GS_TRY_HIP(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
  return GS_OK;
}
int64_t gs_batch_capacity(const gs_batch_plan *p) { return p ? p->cap : 0; }

int gs_render_batch(gs_batch_plan *p, const gs_gaussians *g, int32_t n_views, const gs_view *views, uint32_t mode,
                    gs_grads *grads, gs_stream_t stream) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "plan is NULL");
  int rc = check_views(p, g, n_views, views, mode, grads);
  if (rc) return rc;
  GS_CHECK_DEVICE();
  hipStream_t st = (hipStream_t)stream;
  if (!(mode & GS_GRAPH)) return enqueue_batch(p, g, n_views, views, mode, grads, st);
  // The captured graph bakes every argument in; replay only while they are unchanged.
  std::vector<unsigned char> sig;
  auto add = [&](const void *src, size_t bytes) {
    const unsigned char *c = (const unsigned char *)src;
    sig.insert(sig.end(), c, c + bytes);
  };
  add(g, sizeof *g);
  add(&n_views, sizeof n_views);
  add(&mode, sizeof mode);
  add(views, sizeof(gs_view) * n_views);
  gs_grads gz{};
  add(grads ? grads : &gz, sizeof(gs_grads));

  if (!p->exec || sig != p->signature) {
    if (p->exec) {
      (void)hipGraphExecDestroy(p->exec);
      p->exec = nullptr;
    }
    if (p->graph) {
      (void)hipGraphDestroy(p->graph);
      p->graph = nullptr;
    }
    if (!p->capture_stream)
      GS_TRY_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "capture stream");
    hipStream_t cs = p->capture_stream;
    GS_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    rc = enqueue_batch(p, g, n_views, views, mode & ~GS_GRAPH, grads, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "graph instantiate");
    }
    p->graph = graph;
    p->signature.swap(sig);
  }
  GS_TRY_HIP(hipGraphLaunch(p->exec, st), "graph launch");
  return GS_OK;
}

}  // extern "C"

// =============================================================================================
// Tracking plan: the photometric pose loop (eq:tracking_loss) on one view, map frozen.
// =============================================================================================
struct gs_track_plan {
  int64_t n = 0;
  int32_t deg = 0, tw = 16, th = 16, bd = 256;
  int64_t max_pixels = 0, cap = 0, max_tiles = 0;
  void *block = nullptr;
  gs_projected proj{};
  uint32_t *vals = nullptr, *tile_range = nullptr;
  int64_t *num_pairs = nullptr;
  void *bin_scratch = nullptr, *grad_scratch = nullptr, *blend_state = nullptr;
  float *dC = nullptr, *color = nullptr, *depth = nullptr, *alpha = nullptr, *t_final = nullptr;
  int32_t *last = nullptr;
  float *ssim_scratch = nullptr;
  gs::TrackState *state = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> signature;
};

namespace {

size_t track_bytes(const gs_track_plan &p, size_t *offs) {
  const int64_t n = std::max<int64_t>(p.n, 1), px = std::max<int64_t>(p.max_pixels, 1);
  size_t o = 0;
  auto put = [&](int i, size_t bytes) {
    offs[i] = o;
    o += a256(bytes);
  };
  put(0, 64 * n);                                   // splat cards
  put(1, 4 * n);                                    // n_tiles
  put(2, 4 * n);                                    // dkey
  put(3, 4 * std::max<int64_t>(p.cap, 1));          // vals
  put(4, 8 * std::max<int64_t>(p.max_tiles, 1));    // tile ranges
  put(5, 16);                                       // num_pairs
  put(6, gs::bin_scratch_bytes(n, p.cap));          // bin scratch
  put(7, grads_scratch_bytes_impl(p.n, 1, px));     // backward scratch
  put(8, gs::blend_state_bytes(p.max_tiles, p.cap, p.tw, p.th, p.bd));
  put(9, 12 * px);                                  // dL/dC
  put(10, 12 * px);                                 // colour
  put(11, 4 * px);                                  // depth
  put(12, 4 * px);                                  // opacity
  put(13, 4 * px);                                  // final transmittance
  put(14, 4 * px);                                  // last contributor
  put(15, gs::dssim_scratch_bound(px));             // D-SSIM derivative maps and partial sums
  put(16, sizeof(gs::TrackState));
  return o;
}

int check_track_params(const gs_track_params *q) {
  if (!q) return fail(GS_ERR_INVALID_ARG, "tracking parameters are NULL");
  if (q->iters < 1 || q->iters > 1000) return fail(GS_ERR_INVALID_ARG, "iters must be in [1, 1000]");
  const float f[] = {q->l1_weight, q->ssim_weight, q->lr_rho, q->lr_phi};
  for (float v : f)
    if (!std::isfinite(v) || v < 0.f) return fail(GS_ERR_INVALID_ARG, "weights and step sizes must be finite, >= 0");
  if (!(q->beta1 >= 0.f && q->beta1 < 1.f) || !(q->beta2 >= 0.f && q->beta2 < 1.f))
    return fail(GS_ERR_INVALID_ARG, "betas must be in [0, 1)");
  if (!(q->eps > 0.f) || !std::isfinite(q->eps)) return fail(GS_ERR_INVALID_ARG, "eps must be finite and > 0");
  if (q->flags & ~(uint32_t)GS_GRAPH) return fail(GS_ERR_INVALID_ARG, "unknown flags");
  return GS_OK;
}

// The iterations (everything after the state set-up), enqueued on `st`.
int enqueue_track(gs_track_plan *p, const gs_gaussians *g, const gs_camera *cam, const float *target,
                  const gs_track_params *q, float *pose_out, float *trace, hipStream_t st) {
  gs::ViewTable vt;
  int rc = make_table(cam, 1, g->n, g->sh_degree, p->tw, p->th, vt);
  if (rc) return rc;
  vt.pose_dev = p->state->pose;
  const int h = cam->h, w = cam->w;
  const int64_t px = (int64_t)w * h;
  if (gs::dssim_scratch_bytes(3, h, w) > gs::dssim_scratch_bound(p->max_pixels))
    return fail(GS_ERR_INVALID_ARG, "d-ssim scratch");
  gs::ImgTable it{};
  it.v[0] = {p->color, p->depth, p->alpha, p->t_final, p->last, nullptr};
  gs_image img{p->color, p->depth, p->alpha, p->t_final, p->last, nullptr, p->blend_state, 0};
  ViewIO io{};
  io.img = img;
  io.dC = p->dC;
  io.pose = p->state->grad;
  gs_grads none{};
  none.overwrite = 1;
  const GradScratch s = carve_grads(p->grad_scratch, g->n, 1, px);
  gs::TrackStepArgs a{};
  for (int i = 0; i < 3; ++i) {
    a.lr[i] = q->lr_rho;
    a.lr[3 + i] = q->lr_phi;
  }
  a.beta1 = q->beta1;
  a.beta2 = q->beta2;
  a.eps = q->eps;
  for (int k = 1; k <= q->iters; ++k) {
    gs::profile_begin(GS_STAGE_PREPROCESS, st);
    GS_TRY_HIP(gs::launch_preprocess(vt, *g, p->proj, st), "track preprocess");
    gs::profile_end(GS_STAGE_PREPROCESS, st);
    gs::profile_begin(GS_STAGE_BIN_SORT, st);
    GS_TRY_HIP(gs::launch_bin_sort(vt, p->proj, g->n, p->cap, p->vals, p->tile_range, p->num_pairs, p->bin_scratch,
                                   st),
               "track bin/sort");
    gs::profile_end(GS_STAGE_BIN_SORT, st);
    gs::profile_begin(GS_STAGE_BLEND_FWD, st);
    GS_TRY_HIP(gs::launch_blend_fwd(p->bd, vt, it, p->proj, p->vals, p->tile_range, p->blend_state, p->cap, st),
               "track blend forward");
    gs::profile_end(GS_STAGE_BLEND_FWD, st);
    GS_TRY_HIP(gs::launch_loss_l1(p->color, target, 3 * px, q->l1_weight, p->dC, &p->state->loss[0], st),
               "track l1 loss");
    GS_TRY_HIP(gs::launch_dssim(p->color, target, 3, h, w, q->ssim_weight, p->dC, &p->state->loss[1], p->ssim_scratch,
                                st),
               "track d-ssim");
    rc = enqueue_backward(vt, *g, p->proj, p->vals, p->tile_range, p->blend_state, p->cap, &io, p->bd, none, s, st);
    if (rc) return rc;
    a.k = k;
    a.bias1 = 1.0 - std::pow((double)q->beta1, k);
    a.bias2 = 1.0 - std::pow((double)q->beta2, k);
    GS_TRY_HIP(gs::launch_track_step(p->state, a, p->num_pairs, trace, k == q->iters ? pose_out : nullptr, st),
               "track pose step");
  }
  return GS_OK;
}

// SE(3) logarithm (inverse of the closed-form exponential) for rotation angles below pi.
void se3_log(const double R[9], const double t[3], double xi[6]) {
  const double c = std::min(1.0, std::max(-1.0, (R[0] + R[4] + R[8] - 1.0) / 2.0));
  const double th = std::acos(c);
  const double w[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};  // vee(R - R^T)
  const double f = th < 1e-5 ? 0.5 + th * th / 12.0 : th / (2.0 * std::sin(th));
  const double phi[3] = {f * w[0], f * w[1], f * w[2]};
  const double P[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
  const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], tn = std::sqrt(t2);
  // V^-1 = I - P/2 + D P^2
  const double D = tn < 1e-5 ? 1.0 / 12.0 + t2 / 720.0
                             : (1.0 - tn * std::sin(tn) / (2.0 * (1.0 - std::cos(tn)))) / t2;
  for (int i = 0; i < 3; ++i) {
    double s = t[i];
    for (int l = 0; l < 3; ++l) {
      double p2 = 0.0;
      for (int m = 0; m < 3; ++m) p2 += P[3 * i + m] * P[3 * m + l];
      s += (-0.5 * P[3 * i + l] + D * p2) * t[l];
    }
    xi[i] = s;
    xi[3 + i] = phi[i];
  }
}

}  // namespace

extern "C" {

int gs_track_plan_create(gs_track_plan **out, int64_t n, int32_t sh_degree, int64_t max_pixels, int32_t tile_w,
                         int32_t tile_h, int32_t blend_depth, int64_t capacity) {
  if (!out) return fail(GS_ERR_INVALID_ARG, "plan out-pointer is NULL");
  *out = nullptr;
  if (n < 0 || n > 0x7FFFFFFF || sh_degree < 0 || sh_degree > 3) return fail(GS_ERR_INVALID_ARG, "bad n or degree");
  if (!tile_ok(tile_w, tile_h)) return fail(GS_ERR_INVALID_ARG, "tile sides must be 8, 16 or 32");
  if (!depth_ok(blend_depth)) return fail(GS_ERR_INVALID_ARG, "blend_depth must be 32, 64, 128 or 256");
  if (max_pixels <= 0 || max_pixels > 0x7FFFFFFF || capacity <= 0 || capacity > 0xFFFFFFFFll)
    return fail(GS_ERR_INVALID_ARG, "bad pixel budget or capacity");
  GS_CHECK_DEVICE();
  gs_track_plan *p = new gs_track_plan();
  p->n = n;
  p->deg = sh_degree;
  p->tw = tile_w;
  p->th = tile_h;
  p->bd = blend_depth;
  p->max_pixels = max_pixels;
  p->cap = capacity;
  p->max_tiles = max_pixels / ((int64_t)tile_w * tile_h) + (32768 / tile_w + 32768 / tile_h + 1);
  size_t offs[17];
  const size_t bytes = track_bytes(*p, offs);
  hipError_t e = hipMalloc(&p->block, bytes);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "tracking plan allocation");
  }
  char *b = (char *)p->block;
  p->proj.card = (float *)(b + offs[0]);
  p->proj.n_tiles = (uint32_t *)(b + offs[1]);
  p->proj.dkey = (uint32_t *)(b + offs[2]);
  p->vals = (uint32_t *)(b + offs[3]);
  p->tile_range = (uint32_t *)(b + offs[4]);
  p->num_pairs = (int64_t *)(b + offs[5]);
  p->bin_scratch = b + offs[6];
  p->grad_scratch = b + offs[7];
  p->blend_state = b + offs[8];
  p->dC = (float *)(b + offs[9]);
  p->color = (float *)(b + offs[10]);
  p->depth = (float *)(b + offs[11]);
  p->alpha = (float *)(b + offs[12]);
  p->t_final = (float *)(b + offs[13]);
  p->last = (int32_t *)(b + offs[14]);
  p->ssim_scratch = (float *)(b + offs[15]);
  p->state = (gs::TrackState *)(b + offs[16]);
  *out = p;
  return GS_OK;
}

void gs_track_plan_destroy(gs_track_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->block) (void)hipFree(p->block);
  delete p;
}

int64_t gs_track_capacity(const gs_track_plan *p) { return p ? p->cap : 0; }

int gs_track_required_pairs(const gs_track_plan *p, int64_t *required, gs_stream_t stream) {
  if (!p || !required) return fail(GS_ERR_INVALID_ARG, "NULL argument");
  GS_TRY_HIP(hipMemcpyAsync(required, &p->state->max_pairs, sizeof(int64_t), hipMemcpyDeviceToHost,
                            (hipStream_t)stream),
             "copy pair count");
  GS_TRY_HIP(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
  return GS_OK;
}

int gs_track_pose(gs_track_plan *p, const gs_gaussians *g, const gs_camera *cam, const float *target,
                  const gs_track_params *q, float *pose_out, float *trace, gs_stream_t stream) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "plan is NULL");
  int rc;
  if ((rc = check_gaussians(g)) || (rc = check_camera(cam)) || (rc = check_track_params(q))) return rc;
  if (g->n > p->n) return fail(GS_ERR_INVALID_ARG, "map has more Gaussians than the plan");
  if (g->sh_degree > p->deg) return fail(GS_ERR_INVALID_ARG, "SH degree above the plan's");
  if ((int64_t)cam->w * cam->h > p->max_pixels) return fail(GS_ERR_INVALID_ARG, "window exceeds the plan's pixels");
  if (cam->w > 32768 || cam->h > 32768) return fail(GS_ERR_INVALID_ARG, "window above 32768 pixels a side");
  if ((int64_t)((cam->w + p->tw - 1) / p->tw) * ((cam->h + p->th - 1) / p->th) > p->max_tiles)
    return fail(GS_ERR_INVALID_ARG, "window needs more tiles than the plan holds");
  if (!target || !pose_out) return fail(GS_ERR_INVALID_ARG, "target / pose_out is NULL");
  GS_CHECK_DEVICE();
  hipStream_t st = (hipStream_t)stream;
  gs::TrackPose p0;
  for (int i = 0; i < 9; ++i) p0.R[i] = cam->R_cw[i];
  for (int i = 0; i < 3; ++i) p0.t[i] = cam->t_cw[i];
  GS_TRY_HIP(gs::launch_track_init(p->state, p0, st), "track init");
  if (!(q->flags & GS_GRAPH)) return enqueue_track(p, g, cam, target, q, pose_out, trace, st);
  // The graph bakes in every argument but the starting pose, which the init above sets.
  gs_camera key = *cam;
  std::memset(key.R_cw, 0, sizeof key.R_cw);
  std::memset(key.t_cw, 0, sizeof key.t_cw);
  std::vector<unsigned char> sig;
  auto add = [&](const void *src, size_t bytes) {
    const unsigned char *c = (const unsigned char *)src;
    sig.insert(sig.end(), c, c + bytes);
  };
  add(g, sizeof *g);
  add(&key, sizeof key);
  add(&target, sizeof target);
  add(q, sizeof *q);
  add(&pose_out, sizeof pose_out);
  add(&trace, sizeof trace);
  if (!p->exec || sig != p->signature) {
    if (p->exec) {
      (void)hipGraphExecDestroy(p->exec);
      p->exec = nullptr;
    }
    if (p->graph) {
      (void)hipGraphDestroy(p->graph);
      p->graph = nullptr;
    }
    if (!p->capture_stream)
      GS_TRY_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "capture stream");
    hipStream_t cs = p->capture_stream;
    GS_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    rc = enqueue_track(p, g, cam, target, q, pose_out, trace, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "graph instantiate");
    }
    p->graph = graph;
    p->signature.swap(sig);
  }
  GS_TRY_HIP(hipGraphLaunch(p->exec, st), "graph launch");
  return GS_OK;
}

int gs_pose_residual(const float pred_cw[12], const float refined_cw[12], double r[6]) {
  if (!pred_cw || !refined_cw || !r) return fail(GS_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(pred_cw[i]) || !std::isfinite(refined_cw[i]))
      return fail(GS_ERR_INVALID_ARG, "pose is not finite");
  // camera-to-world T_wc = T_cw^-1, so T_wc(t) T~_wc^-1 = T_cw(t)^-1 T~_cw:
  //   R = Rp^T Rr,  t = Rp^T (tr - tp)
  const float *Rp = pred_cw, *tp = pred_cw + 9, *Rr = refined_cw, *tr = refined_cw + 9;
  double R[9], t[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += (double)Rp[3 * l + i] * (double)Rr[3 * l + j];
      R[3 * i + j] = s;
    }
    double s = 0.0;
    for (int l = 0; l < 3; ++l) s += (double)Rp[3 * l + i] * ((double)tr[l] - (double)tp[l]);
    t[i] = s;
  }
  se3_log(R, t, r);
  return GS_OK;
}

}  // extern "C"

// =============================================================================================
// Map initialization and expansion.
// =============================================================================================
namespace {

gs::ExpandArgs expand_args(const gs_points *pts, const gs_camera *cam, const float *opacity, float tau) {
  gs::ExpandArgs a{};
  a.xyz = pts->xyz;
  a.rgb = pts->rgb;
  a.n = pts->n;
  for (int i = 0; i < 9; ++i) a.R[i] = cam->R_cw[i];
  for (int i = 0; i < 3; ++i) a.t[i] = cam->t_cw[i];
  a.fx = cam->fx;
  a.fy = cam->fy;
  a.cx = cam->cx;
  a.cy = cam->cy;
  a.x0 = cam->x0;
  a.y0 = cam->y0;
  a.w = cam->w;
  a.h = cam->h;
  a.opacity = opacity;
  a.tau = tau;
  return a;
}

int check_points(const gs_points *p) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "points are NULL");
  if (p->n < 0 || p->n >= (int64_t(1) << 31)) return fail(GS_ERR_INVALID_ARG, "point count must be in [0, 2^31)");
  if (p->n > 0 && !p->xyz) return fail(GS_ERR_INVALID_ARG, "xyz is NULL");
  return GS_OK;
}

}  // namespace

extern "C" {

size_t gs_expand_scratch_bytes(int64_t n_points) {
  if (n_points < 0) return 0;
  return gs::expand_scratch_bytes(n_points);
}

int gs_expand_select(const gs_points *pts, const gs_camera *cam, const float *opacity, float tau, int64_t *count_out,
                     void *scratch, size_t scratch_bytes, gs_stream_t stream) {
  int rc;
  if ((rc = check_points(pts)) || (rc = check_camera(cam))) return rc;
  if (!std::isfinite(tau)) return fail(GS_ERR_INVALID_ARG, "tau is not finite");
  if (!count_out) return fail(GS_ERR_INVALID_ARG, "count_out is NULL");
  if (!scratch || scratch_bytes < gs::expand_scratch_bytes(pts->n))
    return fail(GS_ERR_INVALID_ARG, "scratch must hold gs_expand_scratch_bytes bytes");
  GS_CHECK_DEVICE();
  GS_TRY_HIP(gs::launch_expand_select(expand_args(pts, cam, opacity, tau), scratch, count_out, (hipStream_t)stream),
             "expand select");
  return GS_OK;
}

int gs_expand_write(const gs_points *pts, const gs_camera *cam, const gs_gaussians *old_map, int64_t added,
                    const void *scratch, size_t scratch_bytes, const gs_gaussians_out *out, gs_stream_t stream) {
  int rc;
  if ((rc = check_points(pts)) || (rc = check_camera(cam))) return rc;
  if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
  if (added < 0 || added > pts->n) return fail(GS_ERR_INVALID_ARG, "added must be in [0, n_points]");
  if (added > 0 && !pts->rgb) return fail(GS_ERR_INVALID_ARG, "rgb is NULL");
  if (!scratch || scratch_bytes < gs::expand_scratch_bytes(pts->n))
    return fail(GS_ERR_INVALID_ARG, "scratch must hold gs_expand_scratch_bytes bytes");
  const int64_t n_old = old_map ? old_map->n : 0;
  if (old_map && (rc = check_gaussians(old_map))) return rc;
  if (out->sh_degree < 0 || out->sh_degree > 3) return fail(GS_ERR_INVALID_ARG, "out sh_degree must be 0..3");
  if (old_map && old_map->sh_degree != out->sh_degree) return fail(GS_ERR_INVALID_ARG, "SH degrees differ");
  if (out->n != n_old + added) return fail(GS_ERR_INVALID_ARG, "out->n must be old n + added");
  if (out->n >= ((int64_t)1 << 30)) return fail(GS_ERR_INVALID_ARG, "grown map too large (at most 2^30 - 1)");
  const int k_rest = 3 * ((out->sh_degree + 1) * (out->sh_degree + 1) - 1);
  if (out->n > 0 && (!out->mean || !out->scale || !out->rot || !out->opacity || !out->sh_dc ||
                     (k_rest > 0 && !out->sh_rest)))
    return fail(GS_ERR_INVALID_ARG, "an output plane is NULL");
  GS_CHECK_DEVICE();
  gs::ExpandOut o{};
  o.n = out->n;
  o.n_old = n_old;
  o.added = added;
  o.k_rest = k_rest;
  o.mean = out->mean;
  o.scale = out->scale;
  o.rot = out->rot;
  o.opacity = out->opacity;
  o.sh_dc = out->sh_dc;
  o.sh_rest = out->sh_rest;
  // every plane of the grown map: the existing part copied (when there is one), the new
  // part of the constant planes filled with its initial value
  gs::PlaneCopy pc{};
  int np = 0;
  const bool has_old = n_old > 0;
  auto group = [&](const float *src, float *dst, int k, bool constant, const float *fill) {
    for (int i = 0; i < k; ++i) {
      pc.src[np] = has_old ? src : nullptr;
      pc.dst[np] = dst;
      pc.plane[np] = i;
      pc.constant[np] = constant ? 1 : 0;
      pc.fill[np] = constant ? fill[i] : 0.f;
      ++np;
    }
  };
  const float rot0[4] = {1.f, 0.f, 0.f, 0.f}, opa0[1] = {0.1f}, zero[1] = {0.f};
  static const float zeros[45] = {};
  group(has_old ? old_map->mean : nullptr, out->mean, 3, false, zero);
  group(has_old ? old_map->scale : nullptr, out->scale, 3, false, zero);
  group(has_old ? old_map->rot : nullptr, out->rot, 4, true, rot0);
  group(has_old ? old_map->opacity : nullptr, out->opacity, 1, true, opa0);
  group(has_old ? old_map->sh_dc : nullptr, out->sh_dc, 3, false, zero);
  if (k_rest > 0) group(has_old ? old_map->sh_rest : nullptr, out->sh_rest, k_rest, true, zeros);
  GS_TRY_HIP(gs::launch_expand_write(expand_args(pts, cam, nullptr, 0.f), scratch, o, pc, np, (hipStream_t)stream),
             "expand write");
  return GS_OK;
}

}  // extern "C"
