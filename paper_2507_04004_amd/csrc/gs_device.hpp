// Device-side types shared by the rasterizer kernels (gfx950, wave64).
//
// Every stage kernel takes a ViewTable by value: up to 16 cameras with their tile grids,
// so one launch covers all views of a batch and a single view is a batch of one. Records
// of view v occupy entries [v*n, (v+1)*n) of the per-record arrays ("entry" index e).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kMaxViews = GS_MAX_VIEWS;
constexpr float kNear = 0.2f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kDilate = 0.3f;

struct ViewCam {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float cw[3];  // camera centre -R^T t in world coordinates
  float bg[3];
  int32_t W, H, x0, y0, w, h;
  int32_t tiles_x, tiles_y;
  uint32_t tile_base;  // first global tile id of this view
  uint32_t pix_base;   // first pixel of this view in concatenated per-pixel scratch
};

struct ViewTable {
  int32_t n_views;
  int32_t tile_w, tile_h;
  int32_t sh_degree;
  int64_t n;             // Gaussians per view
  uint32_t total_tiles;  // sum of tiles over views
  uint32_t pad;
  // Device-resident pose of view 0 (one view only): R_cw row-major (9), t_cw (3), camera
  // centre (3). When set, the kernels that use the pose read it here instead of from v[0],
  // so a pose updated on the device between launches needs no host round trip.
  const float *pose_dev;
  ViewCam v[kMaxViews];
};

// The camera of view vi. DP (device pose): view 0 with its pose from vt.pose_dev, built in
// `tmp`; otherwise the table entry itself.
template <bool DP>
__device__ __forceinline__ const ViewCam &view_cam(const ViewTable &vt, int vi, ViewCam &tmp) {
  if constexpr (!DP) {
    return vt.v[vi];
  } else {
    tmp = vt.v[0];
    const float *p = vt.pose_dev;
#pragma unroll
    for (int i = 0; i < 9; ++i) tmp.R[i] = p[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      tmp.t[i] = p[9 + i];
      tmp.cw[i] = p[12 + i];
    }
    return tmp;
  }
}

struct ViewImg {
  float *color, *depth, *alpha, *t_final;
  int32_t *last, *n_contrib;
};
struct ImgTable {
  ViewImg v[kMaxViews];
};

// Per-view upstream gradients for the blend backward. gD / gO are dense window planes
// (user-given or built from the LiDAR term), or null when the view has none.
struct ViewGrad {
  const float *gC, *gD, *gO;
};
struct GradTable {
  ViewGrad v[kMaxViews];
};

struct LidarView {
  const int32_t *pix;
  const float *target;
  const float *grad_scale;
  float *loss_out;
  float weight;
  int32_t m;
  int32_t npx;  // window pixels: hits outside [0, npx) are ignored
};
struct LidarTable {
  int32_t n_views;
  uint32_t total_hits;
  LidarView v[kMaxViews];
};

__device__ __forceinline__ int view_of_tile(const ViewTable &vt, uint32_t gt) {
  int v = 0;
#pragma unroll 1
  for (int i = 1; i < vt.n_views; ++i)
    if (gt >= vt.v[i].tile_base) v = i;
  return v;
}

// Compositing form of a splat, staged once per chunk: the conic is pre-scaled so that the
// exponent comes out in base 2 with the -1/2 folded in, and the opacity enters the exponent
// as its base-2 logarithm (alpha = o exp(-q/2) = 2^p, p = log2(e) (-q/2) + log2 o):
//   sa = (u, v, a', b'), sb = (c', log2 o, d, b'/2), with a' = kA a, b' = 2 kA b, c' = kA c,
//   kA = -log2(e) / 2, and log2 o = -inf for o <= 0 (and for the padding records).
// p = (a' dx^2 + log2 o) + dy (b' dx + c' dy) <= log2 o in exact arithmetic, evaluated as a
// column part (splat_col: the terms in dx alone, shared by the pixels of a lane, which sit in
// one column of the tile) and the rest (splat_p2); splat_e2 returns 2^p clamped to [0, 1]. The
// forward and the backward both evaluate it through these with fixed FMA placement, so they
// take identical alpha decisions, and p depends on the pixel's offset from the splat only, not
// on the tile size.
constexpr float kA = -0.72134752044448170368f;  // -log2(e) / 2

__device__ __forceinline__ void stage_card(const float4 &A, const float4 &B, const float4 &C, float4 &sa, float4 &sb,
                                           float4 &sc) {
  const float bp = (2.0f * kA) * B.y;
  sa = make_float4(A.x, A.y, kA * B.x, bp);
  sb = make_float4(kA * B.z, A.z > 0.0f ? log2f(A.z) : -INFINITY, A.w, 0.5f * bp);
  sc = C;
}

// The terms of the exponent in the column offset dx alone: a' dx^2 + log2 o, and b' dx.
struct SplatCol {
  float p0, bx;
};
__device__ __forceinline__ SplatCol splat_col(const float4 &sa, const float4 &sb, float dx) {
#pragma clang fp contract(off)
  return SplatCol{fmaf(sa.z * dx, dx, sb.y), sa.w * dx};
}

// Exponent p at row offset dy from the column part, the opacity's logarithm included.
__device__ __forceinline__ float splat_p2(const float4 &sb, const SplatCol &col, float dy) {
  return fmaf(dy, fmaf(sb.x, dy, col.bx), col.p0);
}

// A staged record that no pixel blends (alpha 0 everywhere): the padding of a chunk.
__device__ __forceinline__ void stage_empty(float4 &sa, float4 &sb, float4 &sc) {
  sa = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  sb = make_float4(0.0f, -INFINITY, 0.0f, 0.0f);
  sc = sa;
}

// 2^p clamped to [0, 1] (the median with 0 and 1 becomes the clamp bit of the exp instruction).
__device__ __forceinline__ float splat_e2(float p) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(p), 0.0f, 1.0f);
}

// Smallest value of q over the pixel-centre rectangle [xl,xh] x [yl,yh]: zero when the
// centre lies inside, else the least of the clamped 1-D minima on the facing edges.
__device__ __forceinline__ float rect_qmin(float u, float v, float a, float b, float c, float xl, float xh,
                                           float yl, float yh) {
#pragma clang fp contract(off)
  bool inx = (u >= xl) && (u <= xh);
  bool iny = (v >= yl) && (v <= yh);
  if (inx && iny) return 0.0f;
  float best = INFINITY;
  if (!inx) {
    float X = (u < xl) ? xl : xh;
    float dx = X - u;
    float dy = -(b * dx) / c;
    dy = fminf(fmaxf(dy, yl - v), yh - v);
    float q = a * dx * dx + 2.0f * b * dx * dy + c * dy * dy;
    best = q;
  }
  if (!iny) {
    float Y = (v < yl) ? yl : yh;
    float dy = Y - v;
    float dx = -(b * dy) / a;
    dx = fminf(fmaxf(dx, xl - u), xh - u);
    float q = a * dx * dx + 2.0f * b * dx * dy + c * dy * dy;
    best = fminf(best, q);
  }
  return best;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Exclusive scan of one value per thread over a block of NT threads; returns the total too.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds /*NT/64 + 1*/, uint32_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t t = __shfl_up(inc, off);
    if (lane >= off) inc += t;
  }
  __syncthreads();
  if (lane == 63) lds[wave] = inc;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t x = lds[w];
    if (w < wave) wbase += x;
    tot += x;
  }
  total = tot;
  return wbase + inc - v;
}

// Kept tiles of one splat visited by a whole wavefront: lane l tests tiles l, l + 64, ... of
// the rectangle (row-major) and f(local tile id, rank) is called for kept tiles, where rank
// counts kept tiles in row-major order. All lanes must call this with the same arguments.
template <typename F>
__device__ __forceinline__ uint32_t wave_visit_kept_tiles(const ViewCam &cam, int tw, int th, float u, float v,
                                                          float a, float b, float c, float kappa2, int tx0, int ty0,
                                                          int tx1, int ty1, F &&f) {
  const int rw = tx1 - tx0 + 1;
  const int area = rw * (ty1 - ty0 + 1);
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  const int xend = cam.x0 + cam.w - 1, yend = cam.y0 + cam.h - 1;
  uint32_t done = 0;
  for (int t0 = 0; t0 < area; t0 += 64) {
    const int t = t0 + lane;
    bool keep = false;
    int tx = 0, ty = 0;
    if (t < area) {
      tx = tx0 + t % rw;
      ty = ty0 + t / rw;
      const int xa = cam.x0 + tx * tw, ya = cam.y0 + ty * th;
      const int xb = min(xa + tw - 1, xend), yb = min(ya + th - 1, yend);
      keep = rect_qmin(u, v, a, b, c, (float)xa, (float)xb, (float)ya, (float)yb) <= kappa2;
    }
    const uint64_t m = __ballot(keep);
    if (keep) f((uint32_t)(ty * cam.tiles_x + tx), done + (uint32_t)__popcll(m & lt), (uint32_t)t);
    done += (uint32_t)__popcll(m);
  }
  return done;
}

// One splat record (64 B, one memory line): centre / opacity / depth, conic / kappa^2,
// colour / clamp bits, and the tile rectangle (two int16 pairs), tile count and depth key.
// d = (tx0 | ty0 << 16, tx1 | ty1 << 16, kept tile count, kept-tile mask): for rectangles of
// at most kCoopArea tiles the mask has bit t set when the t-th tile of the rectangle
// (row-major) passed the cull, so pair emission needs no second cull test; 0 otherwise.
struct alignas(64) Card {
  float4 a, b, c;
  uint4 d;
};
static_assert(sizeof(Card) == 64, "splat card is 64 B");

__device__ __forceinline__ uint32_t pack_i16x2(int lo, int hi) {
  return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
}
__device__ __forceinline__ int lo_i16(uint32_t w) { return (int)(int16_t)(w & 0xFFFFu); }
__device__ __forceinline__ int hi_i16(uint32_t w) { return (int)(int16_t)(w >> 16); }

// Planar [k][n] float arrays through buffer instructions: the descriptor of plane k (base
// + k n, n floats long) lives in scalar registers and every plane shares one 32-bit lane
// offset, so a lane holds a single address register however many planes it touches. Out-of-
// range offsets read 0 and drop stores (hardware range check). Needs n < 2^30.
struct Planes {
  uint32_t off, bytes;
  int64_t n;
  __device__ __forceinline__ Planes(int64_t n_, uint32_t idx) : off(idx * 4u), bytes((uint32_t)(n_ * 4)), n(n_) {}
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const float *base, int k) const {
    return __builtin_amdgcn_make_buffer_rsrc((void *)(base + k * n), (short)0, (int)bytes, 0x00020000);
  }
  __device__ __forceinline__ float ld(const float *base, int k) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc(base, k), (int)off, 0, 0));
  }
  __device__ __forceinline__ void st(float *base, int k, float v) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rsrc(base, k), (int)off, 0, 0);
  }
  __device__ __forceinline__ void add(float *base, int k, float v) const { st(base, k, ld(base, k) + v); }
};

// Rectangles with more tiles than this are visited cooperatively by the whole wavefront.
constexpr int kCoopArea = 32;

}  // namespace gs
