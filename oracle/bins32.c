/* FP32 binning oracle: which (tile, Gaussian) pairs exist and in what order.
 *
 * TEST INFRASTRUCTURE ONLY (see gs_oracle.c). The tile lists are integers decided by
 * floating-point comparisons: the footprint rectangle, the alpha-max tile cull at 1/255
 * (Sec. "CUDA-Related Acceleration Strategies", fast tile-based culling) and the depth
 * order of the splatted Gaussians (Sec. "3D Gaussian Splatting Representation"). For the
 * lists to be comparable bit for bit, this file takes each of those decisions in float32,
 * the precision of the kernel, with every operation written out in a fixed order and
 * compiled without FMA contraction. The operation order is part of the specification of
 * the binning step; this file is an independent implementation of it, not shared code.
 *
 * Order of operations (each line one IEEE float32 operation unless marked):
 *   mu_hat_i = ((R_i0*mx + R_i1*my) + R_i2*mz) + t_i ; d = mu_hat_2 ; valid needs d > 0.2f
 *   qq = ((qw*qw + qx*qx) + qy*qy) + qz*qz ; inv = 1/sqrt(qq) ; (w,x,y,z) = q*inv
 *   rotation entries 1-2(y*y+z*z), 2(x*y-w*z), ... ; M_ij = Rq_ij * S_j
 *   Sigma_ij = (M_i0*M_j0 + M_i1*M_j1) + M_i2*M_j2
 *   xn = x/d ; yn = y/d ; u = fx*xn + cx ; v = fy*yn + cy
 *   lim_x = (0.65f*W)/fx ; tx = min(max(xn, -lim_x), lim_x) (same for y)
 *   J00 = fx/d ; J02 = -(fx*tx)/d ; J11 = fy/d ; J12 = -(fy*ty)/d
 *   Tm0j = J00*R0j + J02*R2j ; Tm1j = J11*R1j + J12*R2j
 *   U_ij = (Tm_i0*Sig_0j + Tm_i1*Sig_1j) + Tm_i2*Sig_2j
 *   s00 = ((U00*Tm00 + U01*Tm01) + U02*Tm02) + 0.3f ; s01 = (U00*Tm10 + U01*Tm11) + U02*Tm12 ;
 *   s11 = ((U10*Tm10 + U11*Tm11) + U12*Tm12) + 0.3f
 *   det = s00*s11 - s01*s01 ; a = s11/det ; b = -s01/det ; c = s00/det
 *   kappa2 = (float)(2.0 * log(255.0 * (double)o))   [float64, rounded once to float32]
 *   hx = sqrt(kappa2*s00) ; hy = sqrt(kappa2*s11)
 *   pixel span [ceil(u-hx), floor(u+hx)] clipped to the window; tiles = (span - x0) / B_w
 *   per tile, q_min over the facing edges with the clamped 1-D minimiser, kept iff q_min <= kappa2
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FP_CONTRACT OFF

typedef struct {
  int32_t W, H, x0, y0, w, h;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
} b32_camera;

typedef struct {
  int ok;
  float u, v, d, a, b, c, kappa2;
  int tx0, ty0, tx1, ty1; /* inclusive tile rectangle */
} b32_proj;

static void b32_project(int64_t n, int64_t g, const float *mean, const float *scale, const float *rot,
                        const float *opacity, const b32_camera *cam, b32_proj *p) {
  const float *R = cam->R, *t = cam->t;
  float mx = mean[g], my = mean[n + g], mz = mean[2 * n + g];
  float sx = scale[g], sy = scale[n + g], sz = scale[2 * n + g];
  float qw = rot[g], qx = rot[n + g], qy = rot[2 * n + g], qz = rot[3 * n + g];
  float o = opacity[g];
  int ok = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sx) && isfinite(sy) && isfinite(sz) &&
           isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz) && isfinite(o);
  float px = R[0] * mx + R[1] * my + R[2] * mz + t[0];
  float py = R[3] * mx + R[4] * my + R[5] * mz + t[1];
  float pz = R[6] * mx + R[7] * my + R[8] * mz + t[2];
  ok = ok && pz > 0.2f;
  float qq = qw * qw + qx * qx + qy * qy + qz * qz;
  ok = ok && qq > 0.0f && isfinite(qq);
  ok = ok && sx > 0.0f && sy > 0.0f && sz > 0.0f;
  memset(p, 0, sizeof *p);
  if (!ok) { p->ok = 0; return; }
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
  float u = cam->fx * xn + cam->cx;
  float v = cam->fy * yn + cam->cy;
  float limx = (0.65f * (float)cam->W) / cam->fx;
  float limy = (0.65f * (float)cam->H) / cam->fy;
  float tx = fminf(fmaxf(xn, -limx), limx);
  float ty = fminf(fmaxf(yn, -limy), limy);
  float j00 = cam->fx / pz, j02 = -(cam->fx * tx) / pz;
  float j11 = cam->fy / pz, j12 = -(cam->fy * ty) / pz;
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
  if (!ok) { p->ok = 0; return; }
  float xlo = fmaxf(ceilf(u - hx), (float)cam->x0), xhi = fminf(floorf(u + hx), (float)(cam->x0 + cam->w - 1));
  float ylo = fmaxf(ceilf(v - hy), (float)cam->y0), yhi = fminf(floorf(v + hy), (float)(cam->y0 + cam->h - 1));
  ok = xlo <= xhi && ylo <= yhi;
  p->ok = ok;
  p->u = u; p->v = v; p->d = pz; p->a = a; p->b = b; p->c = c; p->kappa2 = kappa2;
  p->tx0 = (int)xlo - cam->x0; p->tx1 = (int)xhi - cam->x0;
  p->ty0 = (int)ylo - cam->y0; p->ty1 = (int)yhi - cam->y0;
}

static float b32_qmin(float u, float v, float a, float b, float c, float xl, float xh, float yl, float yh) {
  int inx = (u >= xl) && (u <= xh);
  int iny = (v >= yl) && (v <= yh);
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

typedef struct {
  uint32_t tile, dkey, id;
} b32_pair;

static int cmp_pair(const void *A, const void *B) {
  const b32_pair *p = A, *q = B;
  if (p->tile != q->tile) return p->tile < q->tile ? -1 : 1;
  if (p->dkey != q->dkey) return p->dkey < q->dkey ? -1 : 1;
  return (p->id > q->id) - (p->id < q->id);
}

/* Visit the kept tiles of Gaussian p in row-major order; emit (tile, ...) if out != NULL. */
static uint32_t b32_tiles(const b32_proj *p, const b32_camera *cam, int bw, int bh, int tiles_x,
                          uint32_t tile_base, uint32_t id, b32_pair *out) {
  if (!p->ok) return 0;
  uint32_t cnt = 0;
  int tx0 = p->tx0 / bw, tx1 = p->tx1 / bw, ty0 = p->ty0 / bh, ty1 = p->ty1 / bh;
  for (int ty = ty0; ty <= ty1; ++ty) {
    int ya = cam->y0 + ty * bh;
    int yb = ya + bh - 1 < cam->y0 + cam->h - 1 ? ya + bh - 1 : cam->y0 + cam->h - 1;
    for (int tx = tx0; tx <= tx1; ++tx) {
      int xa = cam->x0 + tx * bw;
      int xb = xa + bw - 1 < cam->x0 + cam->w - 1 ? xa + bw - 1 : cam->x0 + cam->w - 1;
      float q = b32_qmin(p->u, p->v, p->a, p->b, p->c, (float)xa, (float)xb, (float)ya, (float)yb);
      if (q <= p->kappa2) {
        if (out) {
          out[cnt].tile = tile_base + (uint32_t)(ty * tiles_x + tx);
          union { float f; uint32_t u; } cv;
          cv.f = p->d;
          out[cnt].dkey = cv.u;
          out[cnt].id = id;
        }
        cnt++;
      }
    }
  }
  return cnt;
}

/* One view. Outputs per Gaussian: n_tiles, the inclusive tile rectangle (tx0, ty0, tx1, ty1;
 * all -1 if invisible) and the depth key (float bits of d, or 0xFFFFFFFF). Sorted pairs are
 * written to vals (ids offset by id_base, tiles offset by tile_base) up to `capacity`; the
 * required count goes to *num_pairs. tile_range[2*t], [2*t+1] = [begin, end) into vals. */
int or32_bin(int64_t n, const float *mean, const float *scale, const float *rot, const float *opacity,
             const b32_camera *cam, int bw, int bh, uint32_t tile_base, uint32_t id_base,
             uint32_t *n_tiles, int32_t *rect, uint32_t *dkey, int64_t capacity, uint32_t *vals,
             uint32_t *tiles_of_pairs, uint32_t *tile_range, int64_t *num_pairs) {
  if (bw <= 0 || bh <= 0 || cam->w <= 0 || cam->h <= 0) return 1;
  int tiles_x = (cam->w + bw - 1) / bw, tiles_y = (cam->h + bh - 1) / bh;
  b32_proj *P = malloc((n > 0 ? n : 1) * sizeof(b32_proj));
  int64_t total = 0;
  for (int64_t g = 0; g < n; ++g) {
    b32_project(n, g, mean, scale, rot, opacity, cam, &P[g]);
    uint32_t c = b32_tiles(&P[g], cam, bw, bh, tiles_x, tile_base, (uint32_t)(id_base + g), NULL);
    n_tiles[g] = c;
    if (c) {
      rect[4 * g] = P[g].tx0 / bw; rect[4 * g + 1] = P[g].ty0 / bh;
      rect[4 * g + 2] = P[g].tx1 / bw; rect[4 * g + 3] = P[g].ty1 / bh;
      union { float f; uint32_t u; } cv;
      cv.f = P[g].d;
      dkey[g] = cv.u;
    } else {
      rect[4 * g] = rect[4 * g + 1] = rect[4 * g + 2] = rect[4 * g + 3] = -1;
      dkey[g] = 0xFFFFFFFFu;
    }
    total += c;
  }
  *num_pairs = total;
  b32_pair *pairs = malloc((total > 0 ? total : 1) * sizeof(b32_pair));
  int64_t off = 0;
  for (int64_t g = 0; g < n; ++g) off += b32_tiles(&P[g], cam, bw, bh, tiles_x, tile_base, (uint32_t)(id_base + g), pairs + off);
  qsort(pairs, (size_t)total, sizeof(b32_pair), cmp_pair);
  int64_t T = (int64_t)tiles_x * tiles_y;
  for (int64_t t = 0; t < 2 * T; ++t) tile_range[t] = 0;
  for (int64_t i = 0; i < total; ++i) {
    uint32_t lt = pairs[i].tile - tile_base;
    if (i == 0 || pairs[i - 1].tile != pairs[i].tile) tile_range[2 * lt] = (uint32_t)i;
    tile_range[2 * lt + 1] = (uint32_t)(i + 1);
  }
  for (int64_t i = 0; i < total && i < capacity; ++i) {
    vals[i] = pairs[i].id;
    if (tiles_of_pairs) tiles_of_pairs[i] = pairs[i].tile;
  }
  free(pairs);
  free(P);
  return 0;
}
