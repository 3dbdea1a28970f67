// Stage a1 (projection / SH colour / footprint / tile count) and stage a5 (its backward and
// the pose gradient) of the Gaussian rasterizer, gfx950.
//
// Sec. "3D Gaussian Splatting Representation": Sigma = R S S^T R^T; mu_hat = R_cw mu + p;
// d = e3^T mu_hat; mu' = pi_c(mu_hat / d); Sigma' = J R_cw Sigma R_cw^T J^T; colour from SH
// up to degree 3 along the view direction. Sec. "CUDA-Related Acceleration Strategies":
// alpha-max tile cull at 1/255 and separated SH planes.
//
// One lane per (Gaussian, view). SoA parameter planes are read coalesced; invalid lanes are
// flagged and all lanes leave through the same exit, so a wavefront whose lanes are all
// culled skips the SH planes entirely (the wave-level predicate masking of Sec. "CUDA-
// Related Acceleration Strategies" d).
//
// Binning decisions (validity, depth key, tile rectangle, cull) are computed in float32 with
// FMA contraction off and a fixed operation order, the order the float32 binning oracle
// implements independently; the rest (colour, gradients) is ordinary float32.
#include <algorithm>

#include "gs_internal.hpp"

namespace gs {

struct Splat {
  bool ok;
  float px, py, pz;        // camera-frame mean
  float inv_q, qw, qx, qy, qz;  // 1/|q| and the unit quaternion
  float r[9];              // rotation of the unit quaternion
  float sx, sy, sz;
  float S00, S01, S02, S11, S12, S22;  // 3D covariance
  float xn, yn, tx, ty;    // x/d, y/d and their clamped values inside J
  float j00, j02, j11, j12;
  float t0[3], t1[3];      // rows of Tm = J R_cw
  float s00, s01, s11, det;
  float a, b, c;           // conic
  float u, v, o, kappa2;
  int32_t px0, px1, py0, py1;  // clipped pixel-centre span of the footprint
};

// Everything below up to the tile rectangle is a binning decision: contraction off.
__device__ __forceinline__ void splat_decide(const ViewCam &cam, float mx, float my, float mz, float sx, float sy,
                                             float sz, float qw, float qx, float qy, float qz, float o, Splat &s) {
#pragma clang fp contract(off)
  const float *R = cam.R;
  const float *t = cam.t;
  bool ok = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sx) && isfinite(sy) && isfinite(sz) &&
            isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz) && isfinite(o);
  float px = R[0] * mx + R[1] * my + R[2] * mz + t[0];
  float py = R[3] * mx + R[4] * my + R[5] * mz + t[1];
  float pz = R[6] * mx + R[7] * my + R[8] * mz + t[2];
  ok = ok && pz > kNear;
  float qq = qw * qw + qx * qx + qy * qy + qz * qz;
  ok = ok && qq > 0.0f && isfinite(qq);
  ok = ok && sx > 0.0f && sy > 0.0f && sz > 0.0f;
  float inv = 1.0f / sqrtf(qq);
  float w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  float r00 = 1.0f - 2.0f * (y * y + z * z), r01 = 2.0f * (x * y - w * z), r02 = 2.0f * (x * z + w * y);
  float r10 = 2.0f * (x * y + w * z), r11 = 1.0f - 2.0f * (x * x + z * z), r12 = 2.0f * (y * z - w * x);
  float r20 = 2.0f * (x * z - w * y), r21 = 2.0f * (y * z + w * x), r22 = 1.0f - 2.0f * (x * x + y * y);
  float m00 = r00 * sx, m01 = r01 * sy, m02 = r02 * sz;
  float m10 = r10 * sx, m11 = r11 * sy, m12 = r12 * sz;
  float m20 = r20 * sx, m21 = r21 * sy, m22 = r22 * sz;
  float S00 = m00 * m00 + m01 * m01 + m02 * m02;
  float S01 = m00 * m10 + m01 * m11 + m02 * m12;
  float S02 = m00 * m20 + m01 * m21 + m02 * m22;
  float S11 = m10 * m10 + m11 * m11 + m12 * m12;
  float S12 = m10 * m20 + m11 * m21 + m12 * m22;
  float S22 = m20 * m20 + m21 * m21 + m22 * m22;
  float xn = px / pz, yn = py / pz;
  float u = cam.fx * xn + cam.cx;
  float v = cam.fy * yn + cam.cy;
  float limx = (0.65f * (float)cam.W) / cam.fx;
  float limy = (0.65f * (float)cam.H) / cam.fy;
  float tx = fminf(fmaxf(xn, -limx), limx);
  float ty = fminf(fmaxf(yn, -limy), limy);
  float j00 = cam.fx / pz, j02 = -(cam.fx * tx) / pz;
  float j11 = cam.fy / pz, j12 = -(cam.fy * ty) / pz;
  float t00 = j00 * R[0] + j02 * R[6], t01 = j00 * R[1] + j02 * R[7], t02 = j00 * R[2] + j02 * R[8];
  float t10 = j11 * R[3] + j12 * R[6], t11 = j11 * R[4] + j12 * R[7], t12 = j11 * R[5] + j12 * R[8];
  float u00 = t00 * S00 + t01 * S01 + t02 * S02;
  float u01 = t00 * S01 + t01 * S11 + t02 * S12;
  float u02 = t00 * S02 + t01 * S12 + t02 * S22;
  float u10 = t10 * S00 + t11 * S01 + t12 * S02;
  float u11 = t10 * S01 + t11 * S11 + t12 * S12;
  float u12 = t10 * S02 + t11 * S12 + t12 * S22;
  float s00 = u00 * t00 + u01 * t01 + u02 * t02 + 0.3f;
  float s01 = u00 * t10 + u01 * t11 + u02 * t12;
  float s11 = u10 * t10 + u11 * t11 + u12 * t12 + 0.3f;
  float det = s00 * s11 - s01 * s01;
  ok = ok && det > 0.0f;
  ok = ok && (255.0 * (double)o >= 1.0);
  float a = s11 / det, b = -s01 / det, c = s00 / det;
  float kappa2 = (float)(2.0 * log(255.0 * (double)o));
  float hx = sqrtf(kappa2 * s00), hy = sqrtf(kappa2 * s11);
  ok = ok && isfinite(u) && isfinite(v) && isfinite(hx) && isfinite(hy);
  float xlo = fmaxf(ceilf(u - hx), (float)cam.x0), xhi = fminf(floorf(u + hx), (float)(cam.x0 + cam.w - 1));
  float ylo = fmaxf(ceilf(v - hy), (float)cam.y0), yhi = fminf(floorf(v + hy), (float)(cam.y0 + cam.h - 1));
  ok = ok && xlo <= xhi && ylo <= yhi;
  s.ok = ok;
  s.px = px; s.py = py; s.pz = pz;
  s.inv_q = inv; s.qw = w; s.qx = x; s.qy = y; s.qz = z;
  s.r[0] = r00; s.r[1] = r01; s.r[2] = r02; s.r[3] = r10; s.r[4] = r11; s.r[5] = r12;
  s.r[6] = r20; s.r[7] = r21; s.r[8] = r22;
  s.sx = sx; s.sy = sy; s.sz = sz;
  s.S00 = S00; s.S01 = S01; s.S02 = S02; s.S11 = S11; s.S12 = S12; s.S22 = S22;
  s.xn = xn; s.yn = yn; s.tx = tx; s.ty = ty;
  s.j00 = j00; s.j02 = j02; s.j11 = j11; s.j12 = j12;
  s.t0[0] = t00; s.t0[1] = t01; s.t0[2] = t02; s.t1[0] = t10; s.t1[1] = t11; s.t1[2] = t12;
  s.s00 = s00; s.s01 = s01; s.s11 = s11; s.det = det;
  s.a = a; s.b = b; s.c = c;
  s.u = u; s.v = v; s.o = o; s.kappa2 = kappa2;
  // spans are only meaningful when ok; keep them in range otherwise
  s.px0 = ok ? (int32_t)xlo : 0;
  s.px1 = ok ? (int32_t)xhi : -1;
  s.py0 = ok ? (int32_t)ylo : 0;
  s.py1 = ok ? (int32_t)yhi : -1;
}

// Real spherical harmonics up to degree 3 (Condon-Shortley phase), index k = l^2 + l + m.
struct SHConst {
  static constexpr float c0 = 0.28209479177387814f;
  static constexpr float c1 = 0.4886025119029199f;
  static constexpr float c2a = 1.0925484305920792f;
  static constexpr float c2b = 0.31539156525252005f;
  static constexpr float c2c = 0.5462742152960396f;
  static constexpr float c3a = 0.5900435899266435f;
  static constexpr float c3b = 2.890611442640554f;
  static constexpr float c3c = 0.4570457994644658f;
  static constexpr float c3d = 0.3731763325901154f;
  static constexpr float c3e = 1.445305721320277f;
};

__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float *Y) {
#pragma clang fp contract(off)
  using K = SHConst;
  Y[0] = K::c0;
  if (deg >= 1) {
    Y[1] = -K::c1 * y;
    Y[2] = K::c1 * z;
    Y[3] = -K::c1 * x;
  }
  if (deg >= 2) {
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = K::c2a * (x * y);
    Y[5] = -K::c2a * (y * z);
    Y[6] = K::c2b * (2.0f * zz - xx - yy);
    Y[7] = -K::c2a * (x * z);
    Y[8] = K::c2c * (xx - yy);
    if (deg >= 3) {
      Y[9] = -K::c3a * y * (3.0f * xx - yy);
      Y[10] = K::c3b * (x * y * z);
      Y[11] = -K::c3c * y * (4.0f * zz - xx - yy);
      Y[12] = K::c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = -K::c3c * x * (4.0f * zz - xx - yy);
      Y[14] = K::c3e * z * (xx - yy);
      Y[15] = -K::c3a * x * (xx - 3.0f * yy);
    }
  }
}

// Colour pre-activation per channel: SH . Y + 0.5, from coefficients already in registers
// (dc [3], rest [3 (K-1)] with index 3 (k-1) + channel). Contraction off and one fixed order,
// so the forward and the backward take the same max(0, .) clamp decision.
__device__ __forceinline__ void sh_colour_raw_v(int deg, const float *dc, const float *rest, const float *Y,
                                                float raw[3]) {
#pragma clang fp contract(off)
  const int K = (deg + 1) * (deg + 1);
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) raw[ch] = dc[ch] * Y[0];
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    if (k < K) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) raw[ch] = raw[ch] + rest[3 * (k - 1) + ch] * Y[k];
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) raw[ch] = raw[ch] + 0.5f;
}

// Loads one Gaussian's coefficients (all lanes issue their loads together) and evaluates.
__device__ __forceinline__ void sh_colour_raw(int deg, const Planes &P, const float *__restrict__ sh_dc,
                                              const float *__restrict__ sh_rest, const float *Y, float raw[3]) {
  const int K = (deg + 1) * (deg + 1);
  float dc[3], rest[45];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) dc[ch] = P.ld(sh_dc, ch);
#pragma unroll
  for (int i = 0; i < 45; ++i) rest[i] = i < 3 * (K - 1) ? P.ld(sh_rest, i) : 0.f;
  sh_colour_raw_v(deg, dc, rest, Y, raw);
}

__device__ __forceinline__ void view_dir(const ViewCam &cam, float mx, float my, float mz, float dir[3], float &dist) {
  float dx = mx - cam.cw[0], dy = my - cam.cw[1], dz = mz - cam.cw[2];
  dist = sqrtf(dx * dx + dy * dy + dz * dz);
  float inv = 1.0f / dist;
  dir[0] = dx * inv; dir[1] = dy * inv; dir[2] = dz * inv;
}

// Kept-tile masks of the small rectangles (at most kCoopArea tiles) of a wavefront, with its
// cull tests dealt out flat over the lanes. Lane order fixes the test numbering: record r owns
// tests [P_r, P_r + area_r), P the exclusive prefix of the areas. In a round of 64 tests a lane
// finds its record as the latest record that starts at or before it (head marks in LDS and a
// max-scan over the lanes; record ids grow with the test number), or the record carried over
// from the previous round. Each test is rect_qmin of the record's centre and conic over the
// tile's pixel-centre rectangle against kappa^2, the same call a walk over each record's own
// rectangle would make, so the masks do not depend on how the tests are dealt out.
__device__ __forceinline__ uint32_t small_rect_masks(const ViewCam &cam, int tw, int th, const Splat &s, bool small,
                                                     int area, int tx0, int ty0, int rw) {
  __shared__ float4 s_p0[256], s_p1[256];
  __shared__ int s_p2[256], s_head[256];
  const int lane = (int)threadIdx.x & 63, wb = (int)threadIdx.x & ~63;
  const int na = small ? area : 0;
  int incl = na;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  const int P = incl - na;
  const int total = __shfl(incl, 63);
  if (total == 0) return 0u;  // uniform
  s_p0[threadIdx.x] = make_float4(s.u, s.v, s.a, s.b);
  s_p1[threadIdx.x] = make_float4(s.c, s.kappa2, small ? 1.0f / (float)rw : 0.f, (float)rw);
  s_p2[threadIdx.x] = (int)pack_i16x2(tx0, ty0);
  const int xend = cam.x0 + cam.w - 1, yend = cam.y0 + cam.h - 1;
  uint32_t mask = 0u;
  int carry = -1;
  for (int T0 = 0; T0 < total; T0 += 64) {
    s_head[threadIdx.x] = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (na > 0 && P >= T0 && P < T0 + 64) s_head[wb + P - T0] = lane;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int r = s_head[threadIdx.x];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(r, off);
      if (lane >= off) r = max(r, t);
    }
    if (r < 0) r = carry;
    carry = __shfl(r, 63);
    const int T = T0 + lane;
    // every lane takes part (a lane shuffle reads nothing from a lane that is switched off)
    const int pr = __shfl(P, max(r, 0));
    bool keep = false;
    if (T < total) {
      const float4 p0 = s_p0[wb + r], p1 = s_p1[wb + r];
      const int t = T - pr;
      const int rwr = (int)p1.w;
      const int row = (int)(((float)t + 0.5f) * p1.z);  // exact for t < 32: (t + 1/2) / rw is never near an integer
      const int txy = s_p2[wb + r];
      const int tx = lo_i16((uint32_t)txy) + (t - row * rwr), ty = hi_i16((uint32_t)txy) + row;
      const int xa = cam.x0 + tx * tw, ya = cam.y0 + ty * th;
      const int xb = min(xa + tw - 1, xend), yb = min(ya + th - 1, yend);
      keep = rect_qmin(p0.x, p0.y, p0.z, p0.w, p1.x, (float)xa, (float)xb, (float)ya, (float)yb) <= p1.y;
    }
    const uint64_t m = __ballot(keep);
    const int lo = max(P, T0), hi = min(P + na, T0 + 64);
    if (lo < hi) mask |= (uint32_t)((m >> (lo - T0)) & ((1ull << (hi - lo)) - 1ull)) << (lo - P);
  }
  return mask;
}

template <bool DP>
__global__ __launch_bounds__(256) void k_preprocess(ViewTable vt, const float *__restrict__ mean,
                                                    const float *__restrict__ scale, const float *__restrict__ rot,
                                                    const float *__restrict__ opacity,
                                                    const float *__restrict__ sh_dc,
                                                    const float *__restrict__ sh_rest, Card *__restrict__ card,
                                                    uint32_t *__restrict__ n_tiles, uint32_t *__restrict__ dkey) {
  const int64_t n = vt.n;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int vi = blockIdx.y;
  const bool in = g < n;  // every lane stays active: the wavefront-wide tile visit below needs all
  ViewCam tmp;
  const ViewCam &cam = view_cam<DP>(vt, vi, tmp);
  const int64_t e = (int64_t)vi * n + g;
  const Planes P(n, (uint32_t)(in ? g : 0));
  float mx = P.ld(mean, 0), my = P.ld(mean, 1), mz = P.ld(mean, 2);
  Splat s;
  splat_decide(cam, mx, my, mz, P.ld(scale, 0), P.ld(scale, 1), P.ld(scale, 2), P.ld(rot, 0), P.ld(rot, 1),
               P.ld(rot, 2), P.ld(rot, 3), P.ld(opacity, 0), s);
  s.ok = s.ok && in;
  uint32_t cnt = 0;
  int tx0 = 0, ty0 = 0, tx1 = -1, ty1 = -1;
  if (s.ok) {
    tx0 = (s.px0 - cam.x0) / vt.tile_w;
    tx1 = (s.px1 - cam.x0) / vt.tile_w;
    ty0 = (s.py0 - cam.y0) / vt.tile_h;
    ty1 = (s.py1 - cam.y0) / vt.tile_h;
  }
  const int area = s.ok ? (tx1 - tx0 + 1) * (ty1 - ty0 + 1) : 0;
  // Small rectangles: the wavefront's tile tests are dealt out flat (test k of the wavefront,
  // counted over its records in lane order, runs in lane k % 64 of round k / 64), so a
  // wavefront spends rounds on its total number of tests instead of on its largest rectangle.
  // Each record's lane collects its tests' results from the round ballots.
  const uint32_t kept_mask = small_rect_masks(cam, vt.tile_w, vt.tile_h, s, s.ok && area <= kCoopArea, area, tx0,
                                              ty0, tx1 - tx0 + 1);
  if (s.ok && area <= kCoopArea) cnt = (uint32_t)__popc(kept_mask);
  // large rectangles are counted by the whole wavefront, one splat at a time
  uint64_t big = __ballot(s.ok && area > kCoopArea);
  while (big) {
    const int src = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const uint32_t c = wave_visit_kept_tiles(
        cam, vt.tile_w, vt.tile_h, __shfl(s.u, src), __shfl(s.v, src), __shfl(s.a, src), __shfl(s.b, src),
        __shfl(s.c, src), __shfl(s.kappa2, src), __shfl(tx0, src), __shfl(ty0, src), __shfl(tx1, src),
        __shfl(ty1, src), [](uint32_t, uint32_t, uint32_t) {});
    if ((int)(threadIdx.x & 63) == src) cnt = c;
  }
  float4 col = make_float4(0.f, 0.f, 0.f, 0.f);
  if (cnt > 0) {
    float dir[3], dist;
    view_dir(cam, mx, my, mz, dir, dist);
    float Y[16];
    sh_eval(vt.sh_degree, dir[0], dir[1], dir[2], Y);
    float raw[3];
    sh_colour_raw(vt.sh_degree, P, sh_dc, sh_rest, Y, raw);
    const uint32_t on = (raw[0] > 0.f ? 1u : 0u) | (raw[1] > 0.f ? 2u : 0u) | (raw[2] > 0.f ? 4u : 0u);
    col = make_float4(fmaxf(raw[0], 0.f), fmaxf(raw[1], 0.f), fmaxf(raw[2], 0.f), __uint_as_float(on));
  }
  if (!in) return;
  const bool vis = cnt > 0;
  const uint32_t key = vis ? __float_as_uint(s.pz) : 0xFFFFFFFFu;
  Card &cd = card[e];
  cd.a = vis ? make_float4(s.u, s.v, s.o, s.pz) : make_float4(0.f, 0.f, 0.f, 0.f);
  cd.b = vis ? make_float4(s.a, s.b, s.c, s.kappa2) : make_float4(0.f, 0.f, 0.f, 0.f);
  cd.c = col;
  cd.d = vis ? make_uint4(pack_i16x2(tx0, ty0), pack_i16x2(tx1, ty1), cnt, kept_mask)
             : make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u);
  n_tiles[e] = cnt;
  dkey[e] = key;
}

// ---------------------------------------------------------------------------------------------
// Stage a5: chain rule from the 2D quantities to the parameters and the pose.
// grad2d records [E][12] (48 B, last two unused), as the compositing backward leaves them:
// sums over pixels of dp dx, dp dy, dp dx^2, dp dx dy, dp dy^2 and dp (the conic, the
// constant factors and the opacity are applied below), then dL/d(r, g, b), dL/d(depth).
// ---------------------------------------------------------------------------------------------
struct ParamGradOut {
  float *mean, *scale, *rot, *opacity, *sh_dc, *sh_rest;
};

// Six block sums at once in a fixed order (deterministic): the same xor butterfly in every
// wave for all six values, then the waves' partials in wave order. Thread t < 6 finds sum t
// in lds[24 + t] on return; lds holds 4 * 6 + 6 floats.
template <int NT>
__device__ __forceinline__ void block_sum6_det(float (&v)[6], float *lds) {
  static_assert(NT == 256, "four waves");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] += __shfl_xor(v[i], off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // lds may still be read from the previous call
  if (lane < 6) {
    float x = v[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) x = lane == i ? v[i] : x;
    lds[wave * 6 + lane] = x;
  }
  __syncthreads();
  if (threadIdx.x < 6) lds[24 + threadIdx.x] = ((lds[threadIdx.x] + lds[6 + threadIdx.x]) + lds[12 + threadIdx.x]) +
                                               lds[18 + threadIdx.x];
}

// One real SH basis function Y_k (1 <= k <= 15) and its gradient as a polynomial of the
// (unnormalised) direction; k is uniform across the wavefront, so the switch is a scalar branch.
__device__ __forceinline__ void sh_term(int k, float x, float y, float z, float &yk, float &dx, float &dy, float &dz) {
  using Kc = SHConst;
  const float xx = x * x, yy = y * y, zz = z * z;
  switch (k) {
    case 1: yk = -Kc::c1 * y; dx = 0.f; dy = -Kc::c1; dz = 0.f; break;
    case 2: yk = Kc::c1 * z; dx = 0.f; dy = 0.f; dz = Kc::c1; break;
    case 3: yk = -Kc::c1 * x; dx = -Kc::c1; dy = 0.f; dz = 0.f; break;
    case 4: yk = Kc::c2a * (x * y); dx = Kc::c2a * y; dy = Kc::c2a * x; dz = 0.f; break;
    case 5: yk = -Kc::c2a * (y * z); dx = 0.f; dy = -Kc::c2a * z; dz = -Kc::c2a * y; break;
    case 6:
      yk = Kc::c2b * (2.0f * zz - xx - yy);
      dx = -2.f * Kc::c2b * x; dy = -2.f * Kc::c2b * y; dz = 4.f * Kc::c2b * z;
      break;
    case 7: yk = -Kc::c2a * (x * z); dx = -Kc::c2a * z; dy = 0.f; dz = -Kc::c2a * x; break;
    case 8: yk = Kc::c2c * (xx - yy); dx = 2.f * Kc::c2c * x; dy = -2.f * Kc::c2c * y; dz = 0.f; break;
    case 9:
      yk = -Kc::c3a * y * (3.0f * xx - yy);
      dx = -6.f * Kc::c3a * x * y; dy = -3.f * Kc::c3a * (xx - yy); dz = 0.f;
      break;
    case 10:
      yk = Kc::c3b * (x * y * z);
      dx = Kc::c3b * y * z; dy = Kc::c3b * x * z; dz = Kc::c3b * x * y;
      break;
    case 11:
      yk = -Kc::c3c * y * (4.0f * zz - xx - yy);
      dx = 2.f * Kc::c3c * x * y; dy = -Kc::c3c * (4.f * zz - xx - 3.f * yy); dz = -8.f * Kc::c3c * y * z;
      break;
    case 12:
      yk = Kc::c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      dx = -6.f * Kc::c3d * x * z; dy = -6.f * Kc::c3d * y * z; dz = Kc::c3d * (6.f * zz - 3.f * xx - 3.f * yy);
      break;
    case 13:
      yk = -Kc::c3c * x * (4.0f * zz - xx - yy);
      dx = -Kc::c3c * (4.f * zz - 3.f * xx - yy); dy = 2.f * Kc::c3c * x * y; dz = -8.f * Kc::c3c * x * z;
      break;
    case 14:
      yk = Kc::c3e * z * (xx - yy);
      dx = 2.f * Kc::c3e * x * z; dy = -2.f * Kc::c3e * y * z; dz = Kc::c3e * (xx - yy);
      break;
    default:
      yk = -Kc::c3a * x * (xx - 3.0f * yy);
      dx = -3.f * Kc::c3a * (xx - yy); dy = 6.f * Kc::c3a * x * y; dz = 0.f;
      break;
  }
}

// Stage a5 runs as two kernels over the Gaussians, each looping over the views:
//   k_sh_bwd   colour: SH coefficient gradients and the view-direction gradient, which it
//              leaves in a compact [E] float4 array;
//   k_geo_bwd  geometry: mean, scale, rotation, opacity and the pose partials.
// Split this way, the coefficient traffic (48 floats in, 48 out per Gaussian) runs at the
// occupancy of a light kernel instead of that of the geometry chain rule.
// OVERWRITE: every output element of the launched range is written (zeros where no view
// contributes); otherwise the gradients are added to the outputs where some view contributes.
template <int DEG, bool SINGLE, bool OVERWRITE, bool DP>
__global__ __launch_bounds__(256) void k_sh_bwd(ViewTable vt, const float *__restrict__ mean,
                                                const float *__restrict__ sh_dc, const float *__restrict__ sh_rest,
                                                const uint32_t *__restrict__ n_tiles, const float *__restrict__ g2,
                                                float4 *__restrict__ gdir, float *__restrict__ out_dc,
                                                float *__restrict__ out_rest) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int NR = 3 * (K - 1);
  constexpr int NRA = NR > 0 ? NR : 1;
  const int64_t n = vt.n;
  const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)gi >= n) return;
  // every plane is addressed by a scalar descriptor and one shared 32-bit lane offset
  const Planes P(n, gi);
  const float mx = P.ld(mean, 0), my = P.ld(mean, 1), mz = P.ld(mean, 2);
  if constexpr (SINGLE && OVERWRITE) {
    // One view, every plane written. All lanes run the body (a lane without a contribution
    // with zero weights and a fixed direction, its coefficients not loaded), so each plane
    // leaves the wavefront as one full-width store instead of a store of the contributing
    // lanes now and one of zeros later, which the L2 could write back in pieces.
    ViewCam tmp;
    const ViewCam &cam = view_cam<DP>(vt, 0, tmp);
    bool live = n_tiles[gi] > 0;
    float2 G67 = make_float2(0.f, 0.f);
    float G8 = 0.f;
    if (live) {
      G67 = *reinterpret_cast<const float2 *>(g2 + (int64_t)gi * 12 + 6);
      G8 = g2[(int64_t)gi * 12 + 8];
      live = G67.x != 0.f || G67.y != 0.f || G8 != 0.f;
    }
    float c_dc[3] = {0.f, 0.f, 0.f}, c_rest[NRA];
#pragma unroll
    for (int i = 0; i < NRA; ++i) c_rest[i] = 0.f;
    if (live) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) c_dc[ch] = P.ld(sh_dc, ch);
#pragma unroll
      for (int i = 0; i < NR; ++i) c_rest[i] = P.ld(sh_rest, i);
    }
    float dir[3], dist;
    view_dir(cam, mx, my, mz, dir, dist);
    if (!live) {
      dir[0] = 0.f;
      dir[1] = 0.f;
      dir[2] = 1.f;
      dist = 1.f;
    }
    float Y[16];
    sh_eval(DEG, dir[0], dir[1], dir[2], Y);
    float raw[3];
    sh_colour_raw_v(DEG, c_dc, c_rest, Y, raw);
    const float gr[3] = {live && raw[0] > 0.f ? G67.x : 0.f, live && raw[1] > 0.f ? G67.y : 0.f,
                         live && raw[2] > 0.f ? G8 : 0.f};
    if (out_dc) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) P.st(out_dc, ch, gr[ch] * Y[0]);
    }
    float gd[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 1; k < K; ++k) {
      float yk, d0, d1, d2;
      sh_term(k, dir[0], dir[1], dir[2], yk, d0, d1, d2);
      float sk = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int i = 3 * (k - 1) + ch;
        sk += gr[ch] * c_rest[i];
        if (out_rest) P.st(out_rest, i, gr[ch] * yk);
      }
      gd[0] += sk * d0;
      gd[1] += sk * d1;
      gd[2] += sk * d2;
    }
    const float dd = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
    const float idist = 1.0f / dist;
    gdir[gi] = live ? make_float4((gd[0] - dd * dir[0]) * idist, (gd[1] - dd * dir[1]) * idist,
                                  (gd[2] - dd * dir[2]) * idist, 0.f)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  bool any_live = false, loaded = false;
  float c_dc[3], c_rest[NRA];
  float acc_dc[3] = {0.f, 0.f, 0.f};
  float acc_rest[SINGLE ? 1 : NRA];
#pragma unroll
  for (int i = 0; i < (SINGLE ? 1 : NRA); ++i) acc_rest[i] = 0.f;
  for (int vi = 0; vi < vt.n_views; ++vi) {
    ViewCam tmp;
    const ViewCam &cam = view_cam<DP>(vt, vi, tmp);
    const int64_t e = (int64_t)vi * n + gi;
    bool live = n_tiles[e] > 0;
    float2 G67 = make_float2(0.f, 0.f);
    float G8 = 0.f;
    if (live) {
      G67 = *reinterpret_cast<const float2 *>(g2 + e * 12 + 6);
      G8 = g2[e * 12 + 8];
      live = G67.x != 0.f || G67.y != 0.f || G8 != 0.f;
    }
    if (!live) {
      gdir[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    any_live = true;
    if (!loaded) {  // all coefficients at once: one burst of independent loads
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) c_dc[ch] = P.ld(sh_dc, ch);
#pragma unroll
      for (int i = 0; i < NR; ++i) c_rest[i] = P.ld(sh_rest, i);
      loaded = true;
    }
    float dir[3], dist;
    view_dir(cam, mx, my, mz, dir, dist);
    float Y[16];
    sh_eval(DEG, dir[0], dir[1], dir[2], Y);
    // the forward's clamp decision, recomputed with the same operations
    float raw[3];
    sh_colour_raw_v(DEG, c_dc, c_rest, Y, raw);
    const float gr[3] = {raw[0] > 0.f ? G67.x : 0.f, raw[1] > 0.f ? G67.y : 0.f, raw[2] > 0.f ? G8 : 0.f};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) acc_dc[ch] += gr[ch] * Y[0];
    float gd[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 1; k < K; ++k) {
      float yk, d0, d1, d2;
      sh_term(k, dir[0], dir[1], dir[2], yk, d0, d1, d2);
      float sk = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int i = 3 * (k - 1) + ch;
        sk += gr[ch] * c_rest[i];
        if constexpr (SINGLE) {
          if (out_rest) {
            if constexpr (OVERWRITE) P.st(out_rest, i, gr[ch] * yk);
            else P.add(out_rest, i, gr[ch] * yk);
          }
        } else {
          acc_rest[i] += gr[ch] * yk;
        }
      }
      gd[0] += sk * d0;
      gd[1] += sk * d1;
      gd[2] += sk * d2;
    }
    // d dir / d mean = (I - dir dir^T) / dist
    const float dd = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
    const float idist = 1.0f / dist;
    gdir[e] = make_float4((gd[0] - dd * dir[0]) * idist, (gd[1] - dd * dir[1]) * idist,
                          (gd[2] - dd * dir[2]) * idist, 0.f);
  }
  if (out_dc && (OVERWRITE || any_live)) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      if constexpr (OVERWRITE) P.st(out_dc, ch, acc_dc[ch]);
      else P.add(out_dc, ch, acc_dc[ch]);
    }
  }
  if (out_rest && NR > 0) {
    if constexpr (SINGLE) {
      if constexpr (OVERWRITE) {
        if (!any_live)
#pragma unroll
          for (int i = 0; i < NR; ++i) P.st(out_rest, i, 0.f);
      }
    } else if (OVERWRITE || any_live) {
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        if constexpr (OVERWRITE) P.st(out_rest, i, acc_rest[i]);
        else P.add(out_rest, i, acc_rest[i]);
      }
    }
  }
}

template <bool OVERWRITE, bool DP>
__global__ __launch_bounds__(256) void k_geo_bwd(ViewTable vt, const float *__restrict__ mean,
                                                 const float *__restrict__ scale, const float *__restrict__ rot,
                                                 const float *__restrict__ opacity,
                                                 const uint32_t *__restrict__ n_tiles, const float *__restrict__ g2,
                                                 const float4 *__restrict__ gdir, ParamGradOut out,
                                                 float *__restrict__ pose_partial /*[grid][V][6]*/) {
  __shared__ float red[32];
  const int64_t n = vt.n;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = g < n;  // every lane stays for the block sums of the pose
  const Planes P(n, (uint32_t)g);
  float mx = 0, my = 0, mz = 0, sx = 1, sy = 1, sz = 1, qw = 1, qx = 0, qy = 0, qz = 0, o = 0;
  if (in) {
    mx = P.ld(mean, 0); my = P.ld(mean, 1); mz = P.ld(mean, 2);
    sx = P.ld(scale, 0); sy = P.ld(scale, 1); sz = P.ld(scale, 2);
    qw = P.ld(rot, 0); qx = P.ld(rot, 1); qy = P.ld(rot, 2); qz = P.ld(rot, 3);
    o = P.ld(opacity, 0);
  }
  float acc_m[3] = {0, 0, 0}, acc_s[3] = {0, 0, 0}, acc_q[4] = {0, 0, 0, 0}, acc_o = 0;
  bool any_view = false;

  for (int vi = 0; vi < vt.n_views; ++vi) {
    ViewCam tmp;
    const ViewCam &cam = view_cam<DP>(vt, vi, tmp);
    const int64_t e = (int64_t)vi * n + g;
    float pose[6] = {0, 0, 0, 0, 0, 0};
    bool live = in && n_tiles[e] > 0;
    float G[10];
    if (live) {
      bool nz = false;
      const float4 *g4 = reinterpret_cast<const float4 *>(g2 + e * 12);
      const float4 A = g4[0], B = g4[1], Cc = g4[2];
      G[0] = A.x; G[1] = A.y; G[2] = A.z; G[3] = A.w; G[4] = B.x; G[5] = B.y; G[6] = B.z; G[7] = B.w;
      G[8] = Cc.x; G[9] = Cc.y;
#pragma unroll
      for (int k = 0; k < 10; ++k) nz |= G[k] != 0.f;
      live = nz;
    }
    if (live) {
      any_view = true;
      const float4 gv4 = gdir[e];  // view-direction path, left by k_sh_bwd
      const float gdf[3] = {gv4.x, gv4.y, gv4.z};
      Splat s;
      splat_decide(cam, mx, my, mz, sx, sy, sz, qw, qx, qy, qz, o, s);
      // grad2d slots 0-4 hold the compositing kernel's sums over pixels of dp dx, dp dy,
      // dp dx^2, dp dx dy, dp dy^2 (dp = dL/dp of the base-2 exponent p = kA q)
      const float a = s.a, b = s.b, c = s.c;
      const float gu = a * G[0] + b * G[1], gv = b * G[0] + c * G[1];
      // dalpha/do = alpha / o: slot 5 sums dp = dL/dalpha alpha over the pixels (a splat of
      // opacity 0 reaches no pixel, and its slot stays 0)
      const float ga = -0.5f * G[2], gb = -G[3], gc = -0.5f * G[4], go = o > 0.f ? G[5] / o : 0.f;
      const float gd = G[9];
      // conic -> Sigma': G_S = -Q Ghat Q, Ghat = [[ga, gb/2], [gb/2, gc]]
      const float hb = 0.5f * gb;
      const float qg00 = a * ga + b * hb, qg01 = a * hb + b * gc;
      const float qg10 = b * ga + c * hb, qg11 = b * hb + c * gc;
      const float GS00 = -(qg00 * a + qg01 * b);
      const float GS01 = -(qg00 * b + qg01 * c);
      const float GS11 = -(qg10 * b + qg11 * c);
      // dL/dSigma = Tm^T G_S Tm (symmetric 3x3)
      const float *T0 = s.t0, *T1 = s.t1;
      float GT0[3], GT1[3];  // G_S Tm (2x3)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GT0[j] = GS00 * T0[j] + GS01 * T1[j];
        GT1[j] = GS01 * T0[j] + GS11 * T1[j];
      }
      float GSig[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) GSig[i][j] = T0[i] * GT0[j] + T1[i] * GT1[j];
      // dL/dTm = 2 G_S Tm Sigma
      const float Sg[3][3] = {{s.S00, s.S01, s.S02}, {s.S01, s.S11, s.S12}, {s.S02, s.S12, s.S22}};
      float dT0[3], dT1[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dT0[j] = 2.f * (GT0[0] * Sg[0][j] + GT0[1] * Sg[1][j] + GT0[2] * Sg[2][j]);
        dT1[j] = 2.f * (GT1[0] * Sg[0][j] + GT1[1] * Sg[1][j] + GT1[2] * Sg[2][j]);
      }
      const float *R = cam.R;
      // Tm = J R: dL/dJ = dT R^T (only the non-zero J entries matter)
      const float gJ00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
      const float gJ02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
      const float gJ11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
      const float gJ12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
      // covariance path of R: dL/dR = J^T dT
      float GRc[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        GRc[0][j] = s.j00 * dT0[j];
        GRc[1][j] = s.j11 * dT1[j];
        GRc[2][j] = s.j02 * dT0[j] + s.j12 * dT1[j];
      }
      // dL/dmu_hat: projection, depth and the J entries
      const float d = s.pz, id = 1.0f / d, id2 = id * id;
      const bool clx = s.tx != s.xn, cly = s.ty != s.yn;
      float gm0 = gu * cam.fx * id;
      float gm1 = gv * cam.fy * id;
      float gm2 = -(gu * cam.fx * s.px + gv * cam.fy * s.py) * id2 + gd;
      gm2 += -(gJ00 * cam.fx + gJ11 * cam.fy) * id2;
      // J02 = -fx tx / d, tx = x/d unless clamped
      if (!clx) {
        gm0 += gJ02 * (-cam.fx * id2);
        gm2 += gJ02 * (2.f * cam.fx * s.px * id2 * id);
      } else {
        gm2 += gJ02 * (cam.fx * s.tx * id2);
      }
      if (!cly) {
        gm1 += gJ12 * (-cam.fy * id2);
        gm2 += gJ12 * (2.f * cam.fy * s.py * id2 * id);
      } else {
        gm2 += gJ12 * (cam.fy * s.ty * id2);
      }
      // Sigma = M M^T, M = Rq diag(S): dL/dM = 2 GSig M
      const float sc[3] = {s.sx, s.sy, s.sz};
      float M[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i][j] = s.r[3 * i + j] * sc[j];
      float GM[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          GM[i][j] = 2.f * (GSig[i][0] * M[0][j] + GSig[i][1] * M[1][j] + GSig[i][2] * M[2][j]);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc_s[j] += GM[0][j] * s.r[j] + GM[1][j] * s.r[3 + j] + GM[2][j] * s.r[6 + j];
      float GR[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) GR[3 * i + j] = GM[i][j] * sc[j];
      const float w = s.qw, x = s.qx, y = s.qy, z = s.qz;
      float gw = 2.f * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
      float gx = 2.f * (y * GR[1] + z * GR[2] + y * GR[3] - 2.f * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] -
                        2.f * x * GR[8]);
      float gy = 2.f * (-2.f * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] -
                        2.f * y * GR[8]);
      float gz = 2.f * (-2.f * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2.f * z * GR[4] + y * GR[5] +
                        x * GR[6] + y * GR[7]);
      const float dotq = gw * w + gx * x + gy * y + gz * z;
      acc_q[0] += (gw - dotq * w) * s.inv_q;
      acc_q[1] += (gx - dotq * x) * s.inv_q;
      acc_q[2] += (gy - dotq * y) * s.inv_q;
      acc_q[3] += (gz - dotq * z) * s.inv_q;
      acc_o += go;
      // mean: R^T dL/dmu_hat + direction path
      acc_m[0] += R[0] * gm0 + R[3] * gm1 + R[6] * gm2 + gdf[0];
      acc_m[1] += R[1] * gm0 + R[4] * gm1 + R[7] * gm2 + gdf[1];
      acc_m[2] += R[2] * gm0 + R[5] * gm1 + R[8] * gm2 + gdf[2];
      // pose, xi = (rho, phi), T_cw <- Exp(xi) T_cw
      //   rho: dL/dmu_hat + R dL/ddiff   (the camera centre moves by -R^T rho)
      //   phi: mu_hat x dL/dmu_hat + vee(N^T - N), N = R GRc^T
      pose[0] = gm0 + (R[0] * gdf[0] + R[1] * gdf[1] + R[2] * gdf[2]);
      pose[1] = gm1 + (R[3] * gdf[0] + R[4] * gdf[1] + R[5] * gdf[2]);
      pose[2] = gm2 + (R[6] * gdf[0] + R[7] * gdf[1] + R[8] * gdf[2]);
      pose[3] = s.py * gm2 - s.pz * gm1;
      pose[4] = s.pz * gm0 - s.px * gm2;
      pose[5] = s.px * gm1 - s.py * gm0;
      float N[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) N[i][j] = R[3 * i] * GRc[j][0] + R[3 * i + 1] * GRc[j][1] + R[3 * i + 2] * GRc[j][2];
      pose[3] += N[1][2] - N[2][1];
      pose[4] += N[2][0] - N[0][2];
      pose[5] += N[0][1] - N[1][0];
    }
    // deterministic per-block partial of the pose gradient for this view
    block_sum6_det<256>(pose, red);
    if (threadIdx.x < 6) pose_partial[((int64_t)blockIdx.x * vt.n_views + vi) * 6 + threadIdx.x] = red[24 + threadIdx.x];
  }
  if (!in || (!OVERWRITE && !any_view)) return;
  auto put = [&](float *base, int i, float v) {
    if constexpr (OVERWRITE) P.st(base, i, v);
    else P.add(base, i, v);
  };
  if (out.mean)
#pragma unroll
    for (int i = 0; i < 3; ++i) put(out.mean, i, acc_m[i]);
  if (out.scale)
#pragma unroll
    for (int i = 0; i < 3; ++i) put(out.scale, i, acc_s[i]);
  if (out.rot)
#pragma unroll
    for (int i = 0; i < 4; ++i) put(out.rot, i, acc_q[i]);
  if (out.opacity) put(out.opacity, 0, acc_o);
}

}  // namespace gs

// ---- launchers used by the host API ------------------------------------------------------
namespace gs {

hipError_t launch_preprocess(const ViewTable &vt, const gs_gaussians &g, const gs_projected &p, hipStream_t st) {
  if (vt.n == 0) return hipSuccess;
  if (vt.pose_dev && vt.n_views != 1) return hipErrorInvalidValue;  // a device pose is view 0's alone
  dim3 grid((unsigned)((vt.n + 255) / 256), (unsigned)vt.n_views);
  if (vt.pose_dev)
    hipLaunchKernelGGL(k_preprocess<true>, grid, dim3(256), 0, st, vt, g.mean, g.scale, g.rot, g.opacity, g.sh_dc,
                       g.sh_rest, (Card *)p.card, p.n_tiles, p.dkey);
  else
    hipLaunchKernelGGL(k_preprocess<false>, grid, dim3(256), 0, st, vt, g.mean, g.scale, g.rot, g.opacity, g.sh_dc,
                       g.sh_rest, (Card *)p.card, p.n_tiles, p.dkey);
  return hipGetLastError();
}

int64_t preprocess_bwd_blocks(int64_t n) { return (n + 255) / 256; }

// Sums the per-block pose partials of each view in a fixed order (float64) and adds the
// result to the view's pose gradient.
struct PosePtrs {
  float *p[kMaxViews];
};

__global__ void k_pose_reduce_tab(const float *__restrict__ partial, int32_t n_blocks, int32_t n_views, PosePtrs out,
                                  int32_t overwrite) {
  __shared__ double red[256];
  const int vi = blockIdx.x / 6, i = blockIdx.x % 6;
  double s = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += 256) s += (double)partial[((int64_t)b * n_views + vi) * 6 + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && out.p[vi]) {
    if (overwrite) out.p[vi][i] = (float)red[0];
    else out.p[vi][i] += (float)red[0];
  }
}

hipError_t launch_preprocess_bwd(const ViewTable &vt, const gs_gaussians &g, const gs_projected &p, const float *g2,
                                 float4 *gdir, const gs_grads &out, float *const *pose_out, float *pose_partial,
                                 hipStream_t st) {
  if (vt.pose_dev && vt.n_views != 1) return hipErrorInvalidValue;
  if (vt.n == 0) {
    // no Gaussians: nothing to differentiate, but overwrite mode still writes the pose
    // gradients (zero; the reduction of zero partials)
    if (out.overwrite == 0) return hipSuccess;
    PosePtrs pp;
    for (int i = 0; i < kMaxViews; ++i) pp.p[i] = i < vt.n_views ? pose_out[i] : nullptr;
    hipLaunchKernelGGL(k_pose_reduce_tab, dim3((unsigned)(6 * vt.n_views)), dim3(256), 0, st, pose_partial, 0,
                       vt.n_views, pp, 1);
    return hipGetLastError();
  }
  const int64_t nb = preprocess_bwd_blocks(vt.n);
  const bool ow = out.overwrite != 0;
  const bool single = vt.n_views == 1;
  // colour first: it hands the view-direction gradient to the geometry kernel
  {
    switch (vt.sh_degree) {
#define GS_SH_BWD(D, S, O, DP)                                                                                 \
  hipLaunchKernelGGL((k_sh_bwd<D, S, O, DP>), dim3((unsigned)nb), dim3(256), 0, st, vt, g.mean, g.sh_dc,         \
                     g.sh_rest, p.n_tiles, g2, gdir, out.sh_dc, out.sh_rest)
#define GS_SH_CASE(D)                                                                                          \
  case D:                                                                                                      \
    if (vt.pose_dev) {                                                                                         \
      if (ow) GS_SH_BWD(D, true, true, true); else GS_SH_BWD(D, true, false, true);                            \
    } else if (single) {                                                                                       \
      if (ow) GS_SH_BWD(D, true, true, false); else GS_SH_BWD(D, true, false, false);                          \
    } else {                                                                                                   \
      if (ow) GS_SH_BWD(D, false, true, false); else GS_SH_BWD(D, false, false, false);                        \
    }                                                                                                          \
    break;
      GS_SH_CASE(0)
      GS_SH_CASE(1)
      GS_SH_CASE(2)
      GS_SH_CASE(3)
#undef GS_SH_CASE
#undef GS_SH_BWD
      default:
        return hipErrorInvalidValue;
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  ParamGradOut po{out.mean, out.scale, out.rot, out.opacity, out.sh_dc, out.sh_rest};
#define GS_GEO_BWD(O, DP)                                                                                       \
  hipLaunchKernelGGL((k_geo_bwd<O, DP>), dim3((unsigned)nb), dim3(256), 0, st, vt, g.mean, g.scale, g.rot,        \
                     g.opacity, p.n_tiles, g2, (const float4 *)gdir, po, pose_partial)
  if (vt.pose_dev) {
    if (ow) GS_GEO_BWD(true, true); else GS_GEO_BWD(false, true);
  } else {
    if (ow) GS_GEO_BWD(true, false); else GS_GEO_BWD(false, false);
  }
#undef GS_GEO_BWD
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  PosePtrs pp;
  for (int i = 0; i < kMaxViews; ++i) pp.p[i] = i < vt.n_views ? pose_out[i] : nullptr;
  hipLaunchKernelGGL(k_pose_reduce_tab, dim3((unsigned)(6 * vt.n_views)), dim3(256), 0, st, pose_partial, (int32_t)nb,
                     vt.n_views, pp, (int32_t)ow);
  return hipGetLastError();
}

}  // namespace gs
