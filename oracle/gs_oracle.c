/* FP64 CPU oracle of the differentiable tile-based Gaussian-splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference the HIP kernels are
 * checked against. Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does. It shares no code, header or constant
 * table with the GPU library.
 *
 * What it computes, in the paper's order (Sec. "3D Gaussian Splatting Representation"):
 *   - 3D covariance Sigma = R S S^T R^T from a quaternion and a linear scale;
 *   - camera-frame mean mu_hat = R_cw mu + p, depth d = e3^T mu_hat, projection mu' = pi_c(mu_hat/d);
 *   - EWA 2D covariance Sigma' = J R_cw Sigma R_cw^T J^T (+0.3 px^2 low-pass, see below);
 *   - per-pixel weight alpha = o exp(-1/2 (mu'-rho)^T Sigma'^-1 (mu'-rho))           (eq:alpha);
 *   - front-to-back compositing of colour, depth and opacity     (eq:rendered_rgb/_depth/_opacity);
 *   - view-dependent colour from real spherical harmonics up to degree 3;
 *   - tiles of B_w x B_h pixels with the alpha-max tile cull at 1/255
 *     (Sec. "CUDA-Related Acceleration Strategies", fast tile-based culling);
 *   - the analytic backward to every Gaussian parameter and to the camera pose on SE(3)
 *     (eq:3dgs_jacobi and the manifold-derivative definition that follows it).
 *
 * Readings of points the paper leaves open (all shared with the GPU path by specification,
 * not by code): pixel centres at integer coordinates; cull d <= 0.2; J built from x/d, y/d
 * clamped to +-1.3 of the full image's half field of view; 0.3 px^2 added to the diagonal of
 * Sigma'; opacity-aware footprint kappa^2 = 2 ln(255 o); alpha = min(0.99, o e^power);
 * a Gaussian contributes only when alpha >= 1/255; compositing stops before a Gaussian that
 * would bring the transmittance below 1e-4; colour = max(0, SH . Y(dir) + 0.5) with dir from
 * the camera centre -R^T p; pose tangent xi = (rho, phi) applied as T_cw <- Exp(xi) T_cw.
 *
 * Everything here is float64. Tiles and the cull only select which Gaussians a pixel visits;
 * the per-pixel result equals compositing every Gaussian with alpha >= 1/255 in (depth, index)
 * order, which the brute-force NumPy oracle checks.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t W, H;           /* full image size */
  int32_t x0, y0, w, h;   /* render window in full-image pixel coordinates */
  double fx, fy, cx, cy;  /* pinhole */
  double R[9];            /* world-to-camera rotation, row-major */
  double t[3];            /* world-to-camera translation */
  double bg[3];           /* background colour */
} or_camera;

typedef struct {
  int64_t n;
  int32_t deg;            /* SH degree 0..3 */
  const double *mean;     /* [3][n] */
  const double *scale;    /* [3][n] linear */
  const double *rot;      /* [4][n] (w, x, y, z) */
  const double *opacity;  /* [n] */
  const double *sh_dc;    /* [3][n] */
  const double *sh_rest;  /* [3*((deg+1)^2-1)][n], plane 3*(k-1)+channel */
} or_gaussians;

#define OR_NEAR 0.2
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_ALPHA_MAX 0.99
#define OR_T_MIN 1e-4
#define OR_DILATE 0.3
#define OR_CLAMP_FOV 1.3

/* ------------------------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3, Condon-Shortley phase, index k = l^2 + l + m.        */
/* Constants are written from their closed forms so a reader can check them.                  */
/* ------------------------------------------------------------------------------------------ */
static void sh_basis(double x, double y, double z, int deg, double *Y, double *dY /* [16][3] or NULL */) {
  const double PI = 3.14159265358979323846;
  const double c0 = 1.0 / (2.0 * sqrt(PI));
  const double c1 = sqrt(3.0) / (2.0 * sqrt(PI));
  const double c2a = sqrt(15.0) / (2.0 * sqrt(PI));
  const double c2b = sqrt(5.0) / (4.0 * sqrt(PI));
  const double c2c = sqrt(15.0) / (4.0 * sqrt(PI));
  const double c3a = sqrt(35.0) / (4.0 * sqrt(2.0 * PI));
  const double c3b = sqrt(105.0) / (2.0 * sqrt(PI));
  const double c3c = sqrt(21.0) / (4.0 * sqrt(2.0 * PI));
  const double c3d = sqrt(7.0) / (4.0 * sqrt(PI));
  const double c3e = sqrt(105.0) / (4.0 * sqrt(PI));
  double g[16][3];
  memset(g, 0, sizeof g);
  Y[0] = c0;
  if (deg >= 1) {
    Y[1] = -c1 * y; g[1][1] = -c1;
    Y[2] = c1 * z;  g[2][2] = c1;
    Y[3] = -c1 * x; g[3][0] = -c1;
  }
  if (deg >= 2) {
    Y[4] = c2a * x * y;                       g[4][0] = c2a * y; g[4][1] = c2a * x;
    Y[5] = -c2a * y * z;                      g[5][1] = -c2a * z; g[5][2] = -c2a * y;
    Y[6] = c2b * (2 * z * z - x * x - y * y); g[6][0] = -2 * c2b * x; g[6][1] = -2 * c2b * y; g[6][2] = 4 * c2b * z;
    Y[7] = -c2a * x * z;                      g[7][0] = -c2a * z; g[7][2] = -c2a * x;
    Y[8] = c2c * (x * x - y * y);             g[8][0] = 2 * c2c * x; g[8][1] = -2 * c2c * y;
  }
  if (deg >= 3) {
    Y[9] = -c3a * y * (3 * x * x - y * y);
    g[9][0] = -6 * c3a * x * y; g[9][1] = -c3a * (3 * x * x - 3 * y * y);
    Y[10] = c3b * x * y * z;
    g[10][0] = c3b * y * z; g[10][1] = c3b * x * z; g[10][2] = c3b * x * y;
    Y[11] = -c3c * y * (4 * z * z - x * x - y * y);
    g[11][0] = 2 * c3c * x * y; g[11][1] = -c3c * (4 * z * z - x * x - 3 * y * y); g[11][2] = -8 * c3c * y * z;
    Y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
    g[12][0] = -6 * c3d * x * z; g[12][1] = -6 * c3d * y * z; g[12][2] = c3d * (6 * z * z - 3 * x * x - 3 * y * y);
    Y[13] = -c3c * x * (4 * z * z - x * x - y * y);
    g[13][0] = -c3c * (4 * z * z - 3 * x * x - y * y); g[13][1] = 2 * c3c * x * y; g[13][2] = -8 * c3c * x * z;
    Y[14] = c3e * z * (x * x - y * y);
    g[14][0] = 2 * c3e * x * z; g[14][1] = -2 * c3e * y * z; g[14][2] = c3e * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3 * y * y);
    g[15][0] = -c3a * (3 * x * x - 3 * y * y); g[15][1] = 6 * c3a * x * y;
  }
  if (dY) memcpy(dY, g, sizeof g);
}

/* Exported for the orthonormality / library-definition pins. */
void or_sh_basis(int64_t m, const double *dirs /*[m][3]*/, int deg, double *out /*[m][16]*/) {
  for (int64_t i = 0; i < m; ++i) {
    double Y[16] = {0};
    sh_basis(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], deg, Y, NULL);
    memcpy(out + 16 * i, Y, sizeof Y);
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Per-Gaussian projection.                                                                    */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
  int valid;
  double m[3], mh[3], d, u, v;
  double qraw[4], qlen, qn[4], Rq[9], S[3], M[9], Sig[9];
  double xn, yn, tx, ty, limx, limy;
  int clx, cly;               /* -1, 0, +1: which side of the J clamp is active */
  double J[6], Tm[6];         /* 2x3 row-major */
  double s00, s01, s11, det, a, b, c;
  double o, kappa2, hx, hy;
  double cw[3], diff[3], dist, dir[3];
  double Y[16], raw[3], rgb[3];
  float dkey;                 /* float32 depth: the compositing order key */
} proj;

static int finite3(const double *a) { return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]); }

/* frozen: if non-NULL, force J-clamp sides (fz[0], fz[1]) and SH clamp mask fz[2] (replay mode). */
static void project(const or_gaussians *G, const or_camera *cam, int64_t k, proj *p, const int *frozen) {
  const int64_t n = G->n;
  const double *R = cam->R, *t = cam->t;
  memset(p, 0, sizeof *p);
  int ok = 1;
  for (int i = 0; i < 3; ++i) p->m[i] = G->mean[i * n + k];
  for (int i = 0; i < 3; ++i) p->S[i] = G->scale[i * n + k];
  for (int i = 0; i < 4; ++i) p->qraw[i] = G->rot[i * n + k];
  p->o = G->opacity[k];
  ok &= finite3(p->m) && finite3(p->S) && isfinite(p->qraw[0]) && isfinite(p->qraw[1]) &&
        isfinite(p->qraw[2]) && isfinite(p->qraw[3]) && isfinite(p->o);
  /* transform into the camera frame; depth is the camera-frame z */
  for (int i = 0; i < 3; ++i) p->mh[i] = R[3 * i] * p->m[0] + R[3 * i + 1] * p->m[1] + R[3 * i + 2] * p->m[2] + t[i];
  p->d = p->mh[2];
  /* The order key is the depth in float32 (R12): the camera-frame z of the float32 inputs,
   * formed as ((R6 mx + R7 my) + R8 mz) + tz in float32, each operation rounded (this file is
   * compiled without contraction). Depths float32 cannot tell apart fall back to the index. */
  {
    const float r6 = (float)R[6], r7 = (float)R[7], r8 = (float)R[8], tz = (float)t[2];
    const float mx = (float)p->m[0], my = (float)p->m[1], mz = (float)p->m[2];
    float acc = r6 * mx;
    acc = acc + r7 * my;
    acc = acc + r8 * mz;
    p->dkey = acc + tz;
  }
  ok &= p->d > OR_NEAR;
  /* rotation from the normalised quaternion (Hamilton convention, w first) */
  p->qlen = sqrt(p->qraw[0] * p->qraw[0] + p->qraw[1] * p->qraw[1] + p->qraw[2] * p->qraw[2] + p->qraw[3] * p->qraw[3]);
  ok &= p->qlen > 0;
  ok &= p->S[0] > 0 && p->S[1] > 0 && p->S[2] > 0;
  if (!ok) { p->valid = 0; return; }
  for (int i = 0; i < 4; ++i) p->qn[i] = p->qraw[i] / p->qlen;
  double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
  double *Rq = p->Rq;
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
  /* Sigma = (Rq S)(Rq S)^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) p->M[3 * i + j] = Rq[3 * i + j] * p->S[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += p->M[3 * i + l] * p->M[3 * j + l];
      p->Sig[3 * i + j] = s;
    }
  /* projection to pixels */
  p->xn = p->mh[0] / p->d;
  p->yn = p->mh[1] / p->d;
  p->u = cam->fx * p->xn + cam->cx;
  p->v = cam->fy * p->yn + cam->cy;
  /* Jacobian of the perspective projection, evaluated at clamped x/d, y/d */
  p->limx = OR_CLAMP_FOV * 0.5 * cam->W / cam->fx;
  p->limy = OR_CLAMP_FOV * 0.5 * cam->H / cam->fy;
  if (frozen) {
    p->clx = frozen[0]; p->cly = frozen[1];
  } else {
    p->clx = p->xn < -p->limx ? -1 : (p->xn > p->limx ? 1 : 0);
    p->cly = p->yn < -p->limy ? -1 : (p->yn > p->limy ? 1 : 0);
  }
  p->tx = p->clx ? p->clx * p->limx : p->xn;
  p->ty = p->cly ? p->cly * p->limy : p->yn;
  double *J = p->J;
  J[0] = cam->fx / p->d; J[1] = 0; J[2] = -cam->fx * p->tx / p->d;
  J[3] = 0; J[4] = cam->fy / p->d; J[5] = -cam->fy * p->ty / p->d;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += J[3 * i + l] * R[3 * l + j];
      p->Tm[3 * i + j] = s;
    }
  /* Sigma' = Tm Sigma Tm^T + 0.3 I */
  double S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l)
        for (int q = 0; q < 3; ++q) s += p->Tm[3 * i + l] * p->Sig[3 * l + q] * p->Tm[3 * j + q];
      S2[2 * i + j] = s;
    }
  p->s00 = S2[0] + OR_DILATE;
  p->s01 = S2[1];
  p->s11 = S2[3] + OR_DILATE;
  p->det = p->s00 * p->s11 - p->s01 * p->s01;
  ok &= p->det > 0;
  ok &= p->o >= OR_ALPHA_MIN;
  ok &= isfinite(p->u) && isfinite(p->v);
  if (ok) {
    p->a = p->s11 / p->det;
    p->b = -p->s01 / p->det;
    p->c = p->s00 / p->det;
    p->kappa2 = 2.0 * log(255.0 * p->o);
    p->hx = sqrt(p->kappa2 * p->s00);
    p->hy = sqrt(p->kappa2 * p->s11);
  }
  /* colour from SH, direction from the camera centre -R^T t to the mean */
  for (int i = 0; i < 3; ++i) p->cw[i] = -(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
  for (int i = 0; i < 3; ++i) p->diff[i] = p->m[i] - p->cw[i];
  p->dist = sqrt(p->diff[0] * p->diff[0] + p->diff[1] * p->diff[1] + p->diff[2] * p->diff[2]);
  for (int i = 0; i < 3; ++i) p->dir[i] = p->diff[i] / p->dist;
  sh_basis(p->dir[0], p->dir[1], p->dir[2], G->deg, p->Y, NULL);
  int K = (G->deg + 1) * (G->deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double s = G->sh_dc[ch * n + k] * p->Y[0];
    for (int kk = 1; kk < K; ++kk) s += G->sh_rest[(3 * (kk - 1) + ch) * n + k] * p->Y[kk];
    p->raw[ch] = s + 0.5;
    int on = frozen ? ((frozen[2] >> ch) & 1) : (p->raw[ch] > 0);
    p->rgb[ch] = on ? p->raw[ch] : 0.0;
  }
  p->valid = ok;
}

/* Exported per-Gaussian records for parity checks of the projection stage. */
void or_project(const or_gaussians *G, const or_camera *cam,
                int32_t *valid, double *uv /*[2][n]*/, double *depth, double *conic /*[3][n]*/,
                double *kappa2, double *rgb /*[3][n]*/, double *ext /*[2][n] hx,hy*/, int32_t *frozen /*[3][n]*/) {
  const int64_t n = G->n;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    proj p;
    project(G, cam, k, &p, NULL);
    valid[k] = p.valid;
    uv[k] = p.u; uv[n + k] = p.v;
    depth[k] = p.d;
    conic[k] = p.a; conic[n + k] = p.b; conic[2 * n + k] = p.c;
    kappa2[k] = p.kappa2;
    for (int ch = 0; ch < 3; ++ch) rgb[ch * n + k] = p.rgb[ch];
    ext[k] = p.hx; ext[n + k] = p.hy;
    if (frozen) {
      frozen[k] = p.clx; frozen[n + k] = p.cly;
      frozen[2 * n + k] = (p.raw[0] > 0) | ((p.raw[1] > 0) << 1) | ((p.raw[2] > 0) << 2);
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Tiles and the alpha-max cull.                                                               */
/* ------------------------------------------------------------------------------------------ */
/* Minimum of q(D) = a Dx^2 + 2 b Dx Dy + c Dy^2 over the rectangle [xl,xh] x [yl,yh] of
 * pixel-centre positions, D = position - (u, v). Zero when the centre is inside; otherwise
 * the minimum of the 1-D constrained minima on the edges that face the centre. */
static double rect_qmin_arg(double u, double v, double a, double b, double c, double xl, double xh, double yl,
                            double yh, double *arg_dx, double *arg_dy) {
  int inx = u >= xl && u <= xh, iny = v >= yl && v <= yh;
  *arg_dx = *arg_dy = 0.0;
  if (inx && iny) return 0.0;
  double best = INFINITY;
  if (!inx) {
    double dx = (u < xl ? xl : xh) - u;
    double dy = -b * dx / c;
    if (dy < yl - v) dy = yl - v;
    if (dy > yh - v) dy = yh - v;
    double q = a * dx * dx + 2 * b * dx * dy + c * dy * dy;
    if (q < best) { best = q; *arg_dx = dx; *arg_dy = dy; }
  }
  if (!iny) {
    double dy = (v < yl ? yl : yh) - v;
    double dx = -b * dy / a;
    if (dx < xl - u) dx = xl - u;
    if (dx > xh - u) dx = xh - u;
    double q = a * dx * dx + 2 * b * dx * dy + c * dy * dy;
    if (q < best) { best = q; *arg_dx = dx; *arg_dy = dy; }
  }
  return best;
}

static double rect_qmin(double u, double v, double a, double b, double c, double xl, double xh, double yl, double yh) {
  double dx, dy;
  return rect_qmin_arg(u, v, a, b, c, xl, xh, yl, yh, &dx, &dy);
}

double or_rect_qmin(double u, double v, double a, double b, double c, double xl, double xh, double yl, double yh) {
  return rect_qmin(u, v, a, b, c, xl, xh, yl, yh);
}

typedef struct {
  int32_t tiles_x, tiles_y, bw, bh;
} tiling;

static tiling make_tiling(const or_camera *cam, int bw, int bh) {
  tiling tg = {(cam->w + bw - 1) / bw, (cam->h + bh - 1) / bh, bw, bh};
  return tg;
}

/* Pixel-centre rectangle covered by tile (tx, ty), clipped to the window. */
static void tile_rect(const or_camera *cam, const tiling *tg, int tx, int ty, double *xl, double *xh, double *yl, double *yh) {
  int ax = cam->x0 + tx * tg->bw, ay = cam->y0 + ty * tg->bh;
  int bx = ax + tg->bw - 1, by = ay + tg->bh - 1;
  if (bx > cam->x0 + cam->w - 1) bx = cam->x0 + cam->w - 1;
  if (by > cam->y0 + cam->h - 1) by = cam->y0 + cam->h - 1;
  *xl = ax; *xh = bx; *yl = ay; *yh = by;
}

/* Tile range [*t0, *t1] (inclusive) whose clipped pixel-centre range meets [c - e, c + e]; 0 if none. */
static int tile_span(double c, double e, int org, int len, int B, int *t0, int *t1) {
  double lo = ceil(c - e), hi = floor(c + e);
  if (lo < org) lo = org;
  if (hi > org + len - 1) hi = org + len - 1;
  if (!(lo <= hi)) return 0;
  *t0 = ((int)lo - org) / B;
  *t1 = ((int)hi - org) / B;
  return 1;
}

typedef struct {
  int64_t *start;  /* [T+1] */
  int32_t *ids;    /* Gaussian ids, per tile sorted by (float32 depth, id) */
} tile_lists;

static const proj *g_sort_proj; /* qsort comparator context (lists are sorted serially) */
static int cmp_depth_id(const void *A, const void *B) {
  int32_t i = *(const int32_t *)A, j = *(const int32_t *)B;
  float di = g_sort_proj[i].dkey, dj = g_sort_proj[j].dkey;
  if (di < dj) return -1;
  if (di > dj) return 1;
  return (i > j) - (i < j);
}

/* Gaussian k is listed in tile (tx, ty) if its footprint rectangle meets the tile and, with
 * culling on, the largest weight it can reach in the tile is >= 1/255 (kappa2_pad widens
 * both tests so near-threshold Gaussians are visited for the marginal flags). */
static int listed(const proj *p, const or_camera *cam, const tiling *tg, int tx, int ty, int cull, double kappa2_pad) {
  if (!cull) return 1;
  double xl, xh, yl, yh;
  tile_rect(cam, tg, tx, ty, &xl, &xh, &yl, &yh);
  return rect_qmin(p->u, p->v, p->a, p->b, p->c, xl, xh, yl, yh) <= p->kappa2 + kappa2_pad;
}

static int footprint(const proj *p, const or_camera *cam, const tiling *tg, double kappa2_pad, int *tx0, int *tx1, int *ty0, int *ty1) {
  if (!p->valid) return 0;
  double k2 = p->kappa2 + kappa2_pad;
  double hx = sqrt(k2 * p->s00), hy = sqrt(k2 * p->s11);
  return tile_span(p->u, hx, cam->x0, cam->w, tg->bw, tx0, tx1) && tile_span(p->v, hy, cam->y0, cam->h, tg->bh, ty0, ty1);
}

static void build_lists(const proj *P, int64_t n, const or_camera *cam, const tiling *tg, int cull, double pad, tile_lists *L) {
  int64_t T = (int64_t)tg->tiles_x * tg->tiles_y;
  int64_t *cnt = calloc(T + 1, sizeof(int64_t));
  for (int64_t k = 0; k < n; ++k) {
    int tx0, tx1, ty0, ty1;
    if (!footprint(&P[k], cam, tg, pad, &tx0, &tx1, &ty0, &ty1)) continue;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx)
        if (listed(&P[k], cam, tg, tx, ty, cull, pad)) cnt[(int64_t)ty * tg->tiles_x + tx]++;
  }
  L->start = malloc((T + 1) * sizeof(int64_t));
  L->start[0] = 0;
  for (int64_t i = 0; i < T; ++i) L->start[i + 1] = L->start[i] + cnt[i];
  L->ids = malloc((L->start[T] > 0 ? L->start[T] : 1) * sizeof(int32_t));
  memset(cnt, 0, (T + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < n; ++k) {
    int tx0, tx1, ty0, ty1;
    if (!footprint(&P[k], cam, tg, pad, &tx0, &tx1, &ty0, &ty1)) continue;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx)
        if (listed(&P[k], cam, tg, tx, ty, cull, pad)) {
          int64_t tt = (int64_t)ty * tg->tiles_x + tx;
          L->ids[L->start[tt] + cnt[tt]++] = (int32_t)k;
        }
  }
  g_sort_proj = P;
  for (int64_t i = 0; i < T; ++i)
    qsort(L->ids + L->start[i], (size_t)(L->start[i + 1] - L->start[i]), sizeof(int32_t), cmp_depth_id);
  free(cnt);
}

static proj *project_all(const or_gaussians *G, const or_camera *cam) {
  proj *P = malloc((G->n > 0 ? G->n : 1) * sizeof(proj));
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < G->n; ++k) project(G, cam, k, &P[k], NULL);
  return P;
}

/* ------------------------------------------------------------------------------------------ */
/* Compositing of one pixel.                                                                   */
/* ------------------------------------------------------------------------------------------ */
#define MB_ALPHA 1   /* some alpha within the relative band of 1/255 */
#define MB_STOP 2    /* some transmittance within the relative band of 1e-4 */
#define MB_CLAMP 4   /* some contributor's alpha within the band of 0.99 (gradient kink) */

typedef struct {
  double C[3], D, O, T;
  int64_t ncontrib;
  int32_t last_id;
  int marginal;
} pix_out;

static double pixel_alpha_raw(const proj *p, double px, double py, double *power_out) {
  double dx = px - p->u, dy = py - p->v;
  double power = -0.5 * (p->a * dx * dx + 2 * p->b * dx * dy + p->c * dy * dy);
  if (power > 0) power = 0; /* the quadratic form is positive definite; guard rounding only */
  if (power_out) *power_out = power;
  return p->o * exp(power);
}

/* Front-to-back over `ids` (already in (float32 depth, id) order). If contrib_ids != NULL, the ids of
 * contributors and their alpha-clamp flags are written there. */
static void composite(const proj *P, const int32_t *ids, int64_t len, double px, double py, const double *bg,
                      double band, pix_out *o, int32_t *contrib_ids, int8_t *contrib_clamped) {
  double T = 1.0, C[3] = {0, 0, 0}, D = 0, O = 0;
  int64_t nc = 0;
  int32_t last = -1;
  int marg = 0;
  for (int64_t i = 0; i < len; ++i) {
    const proj *p = &P[ids[i]];
    double araw = pixel_alpha_raw(p, px, py, NULL);
    if (fabs(araw - OR_ALPHA_MIN) <= band * OR_ALPHA_MIN) marg |= MB_ALPHA;
    double alpha = araw < OR_ALPHA_MAX ? araw : OR_ALPHA_MAX;
    if (alpha < OR_ALPHA_MIN) continue;
    double Tn = T * (1.0 - alpha);
    if (fabs(Tn - OR_T_MIN) <= band * OR_T_MIN) marg |= MB_STOP;
    if (Tn < OR_T_MIN) break;
    if (fabs(araw - OR_ALPHA_MAX) <= band * OR_ALPHA_MAX) marg |= MB_CLAMP;
    double wgt = alpha * T;
    for (int ch = 0; ch < 3; ++ch) C[ch] += wgt * p->rgb[ch];
    D += wgt * p->d;
    O += wgt;
    T = Tn;
    if (contrib_ids) {
      contrib_ids[nc] = ids[i];
      contrib_clamped[nc] = araw >= OR_ALPHA_MAX;
    }
    nc++;
    last = ids[i];
  }
  for (int ch = 0; ch < 3; ++ch) o->C[ch] = C[ch] + T * bg[ch];
  o->D = D;
  o->O = O;
  o->T = T;
  o->ncontrib = nc;
  o->last_id = last;
  o->marginal = marg;
}

/* ------------------------------------------------------------------------------------------ */
/* Forward render of the window. Outputs are window-sized planes ([3][h][w] for colour).       */
/* band: relative width of the marginal bands (0 disables the flags and the list padding).     */
/* ------------------------------------------------------------------------------------------ */
int or_render(const or_gaussians *G, const or_camera *cam, int bw, int bh, int cull, double band,
              double *color, double *depth, double *alpha, double *t_final,
              int32_t *last_id, int64_t *ncontrib, uint8_t *marginal) {
  if (bw <= 0 || bh <= 0 || cam->w <= 0 || cam->h <= 0) return 1;
  proj *P = project_all(G, cam);
  tiling tg = make_tiling(cam, bw, bh);
  tile_lists L;
  double pad = band > 0 ? 2.5 * band : 0.0;
  build_lists(P, G->n, cam, &tg, cull, pad, &L);
  const int64_t npx = (int64_t)cam->w * cam->h;
  const int64_t T = (int64_t)tg.tiles_x * tg.tiles_y;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t tt = 0; tt < T; ++tt) {
    int tx = (int)(tt % tg.tiles_x), ty = (int)(tt / tg.tiles_x);
    for (int j = 0; j < bh; ++j)
      for (int i = 0; i < bw; ++i) {
        int lx = tx * bw + i, ly = ty * bh + j;
        if (lx >= cam->w || ly >= cam->h) continue;
        pix_out po;
        composite(P, L.ids + L.start[tt], L.start[tt + 1] - L.start[tt], cam->x0 + lx, cam->y0 + ly, cam->bg, band, &po, NULL, NULL);
        int64_t pi = (int64_t)ly * cam->w + lx;
        for (int ch = 0; ch < 3; ++ch) color[ch * npx + pi] = po.C[ch];
        depth[pi] = po.D;
        alpha[pi] = po.O;
        t_final[pi] = po.T;
        if (last_id) last_id[pi] = po.last_id;
        if (ncontrib) ncontrib[pi] = po.ncontrib;
        if (marginal) marginal[pi] = (uint8_t)po.marginal;
      }
  }
  free(L.start); free(L.ids); free(P);
  return 0;
}

/* Brute force for listed pixels: every valid Gaussian, sorted by (float32 depth, id), no tiles. */
int or_render_pixels(const or_gaussians *G, const or_camera *cam, int64_t npix, const int32_t *px, const int32_t *py,
                     double band, double *color /*[3][npix]*/, double *depth, double *alpha, double *t_final,
                     int32_t *last_id, int64_t *ncontrib, uint8_t *marginal) {
  proj *P = project_all(G, cam);
  int32_t *ids = malloc((G->n > 0 ? G->n : 1) * sizeof(int32_t));
  int64_t nv = 0;
  for (int64_t k = 0; k < G->n; ++k)
    if (P[k].valid) ids[nv++] = (int32_t)k;
  g_sort_proj = P;
  qsort(ids, (size_t)nv, sizeof(int32_t), cmp_depth_id);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < npix; ++i) {
    pix_out po;
    composite(P, ids, nv, px[i], py[i], cam->bg, band, &po, NULL, NULL);
    for (int ch = 0; ch < 3; ++ch) color[ch * npix + i] = po.C[ch];
    depth[i] = po.D; alpha[i] = po.O; t_final[i] = po.T;
    if (last_id) last_id[i] = po.last_id;
    if (ncontrib) ncontrib[i] = po.ncontrib;
    if (marginal) marginal[i] = (uint8_t)po.marginal;
  }
  free(ids); free(P);
  return 0;
}

/* Contributor lists per pixel (CSR over window pixels): offsets must come from ncontrib. */
int or_contributors(const or_gaussians *G, const or_camera *cam, int bw, int bh,
                    const int64_t *offsets /*[npx+1]*/, int32_t *ids, int8_t *clamped) {
  proj *P = project_all(G, cam);
  tiling tg = make_tiling(cam, bw, bh);
  tile_lists L;
  build_lists(P, G->n, cam, &tg, 1, 0.0, &L);
  const int64_t T = (int64_t)tg.tiles_x * tg.tiles_y;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t tt = 0; tt < T; ++tt) {
    int tx = (int)(tt % tg.tiles_x), ty = (int)(tt / tg.tiles_x);
    for (int j = 0; j < bh; ++j)
      for (int i = 0; i < bw; ++i) {
        int lx = tx * bw + i, ly = ty * bh + j;
        if (lx >= cam->w || ly >= cam->h) continue;
        int64_t pi = (int64_t)ly * cam->w + lx;
        pix_out po;
        composite(P, L.ids + L.start[tt], L.start[tt + 1] - L.start[tt], cam->x0 + lx, cam->y0 + ly, cam->bg, 0.0, &po,
                  ids + offsets[pi], clamped + offsets[pi]);
      }
  }
  free(L.start); free(L.ids); free(P);
  return 0;
}

/* Frozen-branch replay: the smooth function selected by the base point's decisions.
 * Contributor lists, alpha clamps, J-clamp sides and SH clamps are inputs; nothing is tested. */
int or_replay(const or_gaussians *G, const or_camera *cam, const int64_t *offsets, const int32_t *ids,
              const int8_t *clamped, const int32_t *frozen /*[3][n]*/,
              double *color, double *depth, double *alpha) {
  const int64_t n = G->n, npx = (int64_t)cam->w * cam->h;
  proj *P = malloc((n > 0 ? n : 1) * sizeof(proj));
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    int fz[3] = {frozen[k], frozen[n + k], frozen[2 * n + k]};
    project(G, cam, k, &P[k], fz);
    /* validity is not re-tested in replay; the conic is needed for every listed Gaussian */
    P[k].a = P[k].s11 / P[k].det;
    P[k].b = -P[k].s01 / P[k].det;
    P[k].c = P[k].s00 / P[k].det;
  }
#pragma omp parallel for schedule(static)
  for (int64_t pi = 0; pi < npx; ++pi) {
    double px = cam->x0 + (double)(pi % cam->w), py = cam->y0 + (double)(pi / cam->w);
    double T = 1.0, C[3] = {0, 0, 0}, D = 0, O = 0;
    for (int64_t e = offsets[pi]; e < offsets[pi + 1]; ++e) {
      const proj *p = &P[ids[e]];
      double a = clamped[e] ? OR_ALPHA_MAX : pixel_alpha_raw(p, px, py, NULL);
      double wgt = a * T;
      for (int ch = 0; ch < 3; ++ch) C[ch] += wgt * p->rgb[ch];
      D += wgt * p->d;
      O += wgt;
      T *= (1.0 - a);
    }
    for (int ch = 0; ch < 3; ++ch) color[ch * npx + pi] = C[ch] + T * cam->bg[ch];
    depth[pi] = D;
    alpha[pi] = O;
  }
  free(P);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Backward.                                                                                   */
/* grad2d layout [10][n]: u, v, a, b, c, o, r, g, b(colour), d.                                */
/* ------------------------------------------------------------------------------------------ */
static void atomic_add(double *p, double v) {
#pragma omp atomic
  *p += v;
}

/* Per-pixel backward of the compositing: walks the pixel's contributors from the last one to
 * the first, rebuilding each transmittance by division. */
static void pixel_backward(const proj *P, const int32_t *ids, int64_t len, double px, double py, const double *bg,
                           const double *gC, double gD, double gO, int64_t n, double *g2, int32_t *buf_id,
                           double *buf_alpha, int8_t *buf_clamped) {
  /* forward pass to collect the contributors */
  double T = 1.0;
  int64_t nc = 0;
  for (int64_t i = 0; i < len; ++i) {
    const proj *p = &P[ids[i]];
    double araw = pixel_alpha_raw(p, px, py, NULL);
    double alpha = araw < OR_ALPHA_MAX ? araw : OR_ALPHA_MAX;
    if (alpha < OR_ALPHA_MIN) continue;
    double Tn = T * (1.0 - alpha);
    if (Tn < OR_T_MIN) break;
    buf_id[nc] = ids[i];
    buf_alpha[nc] = alpha;
    buf_clamped[nc] = araw >= OR_ALPHA_MAX;
    nc++;
    T = Tn;
  }
  const double Tfin = T;
  double AC[3] = {0, 0, 0}, AD = 0, Tnext = Tfin;
  double gbg = gC[0] * bg[0] + gC[1] * bg[1] + gC[2] * bg[2];
  for (int64_t i = nc - 1; i >= 0; --i) {
    const int32_t k = buf_id[i];
    const proj *p = &P[k];
    const double al = buf_alpha[i];
    const double Ti = Tnext / (1.0 - al);
    const double wgt = al * Ti;
    for (int ch = 0; ch < 3; ++ch) atomic_add(&g2[(6 + ch) * n + k], gC[ch] * wgt);
    atomic_add(&g2[9 * n + k], gD * wgt);
    double dLda = Ti * (gC[0] * (p->rgb[0] - AC[0]) + gC[1] * (p->rgb[1] - AC[1]) + gC[2] * (p->rgb[2] - AC[2]) +
                        gD * (p->d - AD)) +
                  (Tfin / (1.0 - al)) * (gO - gbg);
    for (int ch = 0; ch < 3; ++ch) AC[ch] = al * p->rgb[ch] + (1.0 - al) * AC[ch];
    AD = al * p->d + (1.0 - al) * AD;
    Tnext = Ti;
    if (buf_clamped[i]) continue; /* alpha = 0.99 is constant in o, mu', conic */
    double dx = px - p->u, dy = py - p->v, power;
    double araw = pixel_alpha_raw(p, px, py, &power);
    double G = exp(power);
    atomic_add(&g2[5 * n + k], dLda * G);
    double dLdp = dLda * araw; /* d alpha / d power = alpha */
    /* power = -1/2 (a dx^2 + 2 b dx dy + c dy^2), dx = px - u */
    atomic_add(&g2[0 * n + k], dLdp * (p->a * dx + p->b * dy));
    atomic_add(&g2[1 * n + k], dLdp * (p->b * dx + p->c * dy));
    atomic_add(&g2[2 * n + k], dLdp * (-0.5 * dx * dx));
    atomic_add(&g2[3 * n + k], dLdp * (-dx * dy));
    atomic_add(&g2[4 * n + k], dLdp * (-0.5 * dy * dy));
  }
}

/* Chain rule from the 2D quantities to the parameters and the pose (one Gaussian). */
static void gaussian_backward(const or_gaussians *G, const or_camera *cam, const proj *p, int64_t k, const double *g2l,
                              double *gmean, double *gscale, double *grot, double *gopac, double *gdc, double *grest,
                              double *pose6) {
  const int64_t n = G->n;
  const double *R = cam->R;
  const double fx = cam->fx, fy = cam->fy, d = p->d;
  const double gu = g2l[0], gv = g2l[1], ga = g2l[2], gb = g2l[3], gc = g2l[4], go = g2l[5];
  const double grgb[3] = {g2l[6], g2l[7], g2l[8]}, gd = g2l[9];
  /* conic -> Sigma': G_S = -Q Ghat Q with Ghat = [[ga, gb/2], [gb/2, gc]] */
  double Q[4] = {p->a, p->b, p->b, p->c};
  double Gh[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
  double QG[4], GS[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * Gh[j] + Q[2 * i + 1] * Gh[2 + j];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) GS[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
  /* Sigma' = Tm Sigma Tm^T (+0.3 I): dL/dSigma = Tm^T G_S Tm, dL/dTm = 2 G_S Tm Sigma */
  double GSig[9], GT[6], TS[6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += p->Tm[3 * a + i] * GS[2 * a + b] * p->Tm[3 * b + j];
      GSig[3 * i + j] = s;
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += p->Tm[3 * i + l] * p->Sig[3 * l + j];
      TS[3 * i + j] = s;
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) GT[3 * i + j] = 2.0 * (GS[2 * i] * TS[j] + GS[2 * i + 1] * TS[3 + j]);
  /* Tm = J R: dL/dJ = GT R^T, dL/dR (covariance path) = J^T GT */
  double GJ[6], GRc[9];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += GT[3 * i + l] * R[3 * j + l];
      GJ[3 * i + j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GRc[3 * i + j] = p->J[i] * GT[j] + p->J[3 + i] * GT[3 + j];
  /* J entries as functions of mu_hat (x/d, y/d clamps give zero derivative when active) */
  double gmh[3] = {0, 0, 0};
  double dtx_dx = p->clx ? 0.0 : 1.0 / d, dtx_dz = p->clx ? 0.0 : -p->mh[0] / (d * d);
  double dty_dy = p->cly ? 0.0 : 1.0 / d, dty_dz = p->cly ? 0.0 : -p->mh[1] / (d * d);
  /* J00 = fx/d; J02 = -fx tx/d; J11 = fy/d; J12 = -fy ty/d */
  gmh[2] += GJ[0] * (-fx / (d * d)) + GJ[4] * (-fy / (d * d));
  gmh[0] += GJ[2] * (-fx / d) * dtx_dx;
  gmh[2] += GJ[2] * (fx * p->tx / (d * d) - fx / d * dtx_dz);
  gmh[1] += GJ[5] * (-fy / d) * dty_dy;
  gmh[2] += GJ[5] * (fy * p->ty / (d * d) - fy / d * dty_dz);
  /* projection u = fx x/d + cx, v = fy y/d + cy, and depth d = z */
  gmh[0] += gu * fx / d;
  gmh[1] += gv * fy / d;
  gmh[2] += -gu * fx * p->mh[0] / (d * d) - gv * fy * p->mh[1] / (d * d) + gd;
  /* Sigma = M M^T, M = Rq diag(S) */
  double GM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += (GSig[3 * i + l] + GSig[3 * l + i]) * p->M[3 * l + j];
      GM[3 * i + j] = s;
    }
  for (int j = 0; j < 3; ++j) {
    double s = 0;
    for (int i = 0; i < 3; ++i) s += GM[3 * i + j] * p->Rq[3 * i + j];
    gscale[j * n + k] += s;
  }
  double GRq[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) GRq[3 * i + j] = GM[3 * i + j] * p->S[j];
  double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
  /* d Rq / d (w, x, y, z), entry by entry */
  double gq[4];
  gq[0] = GRq[1] * (-2 * z) + GRq[2] * (2 * y) + GRq[3] * (2 * z) + GRq[5] * (-2 * x) + GRq[6] * (-2 * y) + GRq[7] * (2 * x);
  gq[1] = GRq[1] * (2 * y) + GRq[2] * (2 * z) + GRq[3] * (2 * y) + GRq[4] * (-4 * x) + GRq[5] * (-2 * w) +
          GRq[6] * (2 * z) + GRq[7] * (2 * w) + GRq[8] * (-4 * x);
  gq[2] = GRq[0] * (-4 * y) + GRq[1] * (2 * x) + GRq[2] * (2 * w) + GRq[3] * (2 * x) + GRq[5] * (2 * z) +
          GRq[6] * (-2 * w) + GRq[7] * (2 * z) + GRq[8] * (-4 * y);
  gq[3] = GRq[0] * (-4 * z) + GRq[1] * (-2 * w) + GRq[2] * (2 * x) + GRq[3] * (2 * w) + GRq[4] * (-4 * z) +
          GRq[5] * (2 * y) + GRq[7] * (2 * y) + GRq[6] * (2 * x);
  double qdot = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
  for (int i = 0; i < 4; ++i) grot[i * n + k] += (gq[i] - qdot * p->qn[i]) / p->qlen;
  /* colour: SH coefficients and the viewing direction */
  int K = (G->deg + 1) * (G->deg + 1);
  double Y[16], dY[16][3];
  sh_basis(p->dir[0], p->dir[1], p->dir[2], G->deg, Y, &dY[0][0]);
  double gdir[3] = {0, 0, 0};
  for (int ch = 0; ch < 3; ++ch) {
    if (!(p->raw[ch] > 0)) continue;
    double g = grgb[ch];
    gdc[ch * n + k] += g * Y[0];
    for (int kk = 1; kk < K; ++kk) {
      grest[(3 * (kk - 1) + ch) * n + k] += g * Y[kk];
      double coef = G->sh_rest[(3 * (kk - 1) + ch) * n + k];
      for (int i = 0; i < 3; ++i) gdir[i] += g * coef * dY[kk][i];
    }
  }
  double dd = gdir[0] * p->dir[0] + gdir[1] * p->dir[1] + gdir[2] * p->dir[2];
  double gdiff[3];
  for (int i = 0; i < 3; ++i) gdiff[i] = (gdir[i] - dd * p->dir[i]) / p->dist;
  /* mean: through mu_hat = R mu + t and through the direction */
  for (int i = 0; i < 3; ++i) gmean[i * n + k] += R[i] * gmh[0] + R[3 + i] * gmh[1] + R[6 + i] * gmh[2] + gdiff[i];
  gopac[k] += go;
  /* pose, xi = (rho, phi), T_cw <- Exp(xi) T_cw:
   *   d mu_hat = rho + phi x mu_hat;  d c_w = -R^T rho;  d R = [phi]x R  */
  double gcw[3] = {-gdiff[0], -gdiff[1], -gdiff[2]};
  for (int i = 0; i < 3; ++i) pose6[i] += gmh[i] - (R[3 * i] * gcw[0] + R[3 * i + 1] * gcw[1] + R[3 * i + 2] * gcw[2]);
  pose6[3] += p->mh[1] * gmh[2] - p->mh[2] * gmh[1];
  pose6[4] += p->mh[2] * gmh[0] - p->mh[0] * gmh[2];
  pose6[5] += p->mh[0] * gmh[1] - p->mh[1] * gmh[0];
  double N[9]; /* N = R GRc^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += R[3 * i + l] * GRc[3 * j + l];
      N[3 * i + j] = s;
    }
  pose6[3] += N[5] - N[7];
  pose6[4] += N[6] - N[2];
  pose6[5] += N[1] - N[3];
}

/* Gradients of  sum gC.C + sum gD.D + sum gO.O  (window planes) with respect to every
 * parameter (accumulated into the zeroed outputs) and the 6-vector pose tangent. */
int or_backward(const or_gaussians *G, const or_camera *cam, int bw, int bh,
                const double *gC /*[3][h][w]*/, const double *gD /*[h][w] or NULL*/, const double *gO /*or NULL*/,
                double *grad2d /*[10][n]*/, double *gmean, double *gscale, double *grot, double *gopac,
                double *gdc, double *grest, double *pose6) {
  const int64_t n = G->n, npx = (int64_t)cam->w * cam->h;
  proj *P = project_all(G, cam);
  tiling tg = make_tiling(cam, bw, bh);
  tile_lists L;
  build_lists(P, n, cam, &tg, 1, 0.0, &L);
  const int64_t T = (int64_t)tg.tiles_x * tg.tiles_y;
  int64_t maxlen = 1;
  for (int64_t i = 0; i < T; ++i)
    if (L.start[i + 1] - L.start[i] > maxlen) maxlen = L.start[i + 1] - L.start[i];
  memset(grad2d, 0, sizeof(double) * 10 * (size_t)n);
#pragma omp parallel
  {
    int32_t *bid = malloc(maxlen * sizeof(int32_t));
    double *bal = malloc(maxlen * sizeof(double));
    int8_t *bcl = malloc(maxlen * sizeof(int8_t));
#pragma omp for schedule(dynamic, 1)
    for (int64_t tt = 0; tt < T; ++tt) {
      int tx = (int)(tt % tg.tiles_x), ty = (int)(tt / tg.tiles_x);
      for (int j = 0; j < bh; ++j)
        for (int i = 0; i < bw; ++i) {
          int lx = tx * bw + i, ly = ty * bh + j;
          if (lx >= cam->w || ly >= cam->h) continue;
          int64_t pi = (int64_t)ly * cam->w + lx;
          double gc3[3] = {gC[pi], gC[npx + pi], gC[2 * npx + pi]};
          pixel_backward(P, L.ids + L.start[tt], L.start[tt + 1] - L.start[tt], cam->x0 + lx, cam->y0 + ly, cam->bg, gc3,
                         gD ? gD[pi] : 0.0, gO ? gO[pi] : 0.0, n, grad2d, bid, bal, bcl);
        }
    }
    free(bid); free(bal); free(bcl);
  }
  for (int i = 0; i < 6; ++i) pose6[i] = 0;
  for (int64_t k = 0; k < n; ++k) {
    if (!P[k].valid) continue;
    double g2l[10];
    int any = 0;
    for (int i = 0; i < 10; ++i) { g2l[i] = grad2d[i * n + k]; any |= g2l[i] != 0.0; }
    if (!any) continue;
    gaussian_backward(G, cam, &P[k], k, g2l, gmean, gscale, grot, gopac, gdc, grest, pose6);
  }
  free(L.start); free(L.ids); free(P);
  return 0;
}

/* Camera-frame quantities for a chosen Gaussian (diagnostics and pins). */
void or_project_one(const or_gaussians *G, const or_camera *cam, int64_t k, double *out /*[32]*/) {
  proj p;
  project(G, cam, k, &p, NULL);
  double v[32] = {p.valid, p.mh[0], p.mh[1], p.mh[2], p.u, p.v, p.s00, p.s01, p.s11, p.a, p.b, p.c, p.kappa2,
                  p.hx, p.hy, p.rgb[0], p.rgb[1], p.rgb[2], p.J[0], p.J[2], p.J[4], p.J[5],
                  p.Sig[0], p.Sig[1], p.Sig[2], p.Sig[4], p.Sig[5], p.Sig[8], p.clx, p.cly, p.dist, p.o};
  memcpy(out, v, sizeof v);
}

/* ------------------------------------------------------------------------------------------ */
/* Float64 tile lists and the margin of each (Gaussian, tile) decision.                        */
/* ------------------------------------------------------------------------------------------ */
/* The float64 tile lists (no marginal band) as CSR over the window's tiles: start [T+1] and,
 * when ids != NULL, ids [start[T]] with each tile's Gaussians in (depth, index) order. */
int or_lists(const or_gaussians *G, const or_camera *cam, int bw, int bh, int64_t *start, int32_t *ids) {
  if (bw <= 0 || bh <= 0 || cam->w <= 0 || cam->h <= 0) return 1;
  proj *P = project_all(G, cam);
  tiling tg = make_tiling(cam, bw, bh);
  tile_lists L;
  build_lists(P, G->n, cam, &tg, 1, 0.0, &L);
  const int64_t T = (int64_t)tg.tiles_x * tg.tiles_y;
  memcpy(start, L.start, (size_t)(T + 1) * sizeof(int64_t));
  if (ids && L.start[T] > 0) memcpy(ids, L.ids, (size_t)L.start[T] * sizeof(int32_t));
  free(L.start); free(L.ids); free(P);
  return 0;
}

/* A conjunction of conditions c_i (true when the signed margin m_i >= 0) flips when its
 * smallest margin does if it holds, and only when every false term flips if it does not. */
typedef struct {
  int all_true;
  double min_true, max_false;
} conj;

static void conj_add(conj *c, double m) {
  if (m >= 0) {
    if (m < c->min_true) c->min_true = m;
  } else {
    c->all_true = 0;
    if (-m > c->max_false) c->max_false = -m;
  }
}

/* For m queried pairs (Gaussian gid[i], window tile tile[i]): listed[i] = the float64
 * decision, margin[i] = its relative distance from flipping. A pair exists when the Gaussian
 * is valid, the tile's clipped pixel-centre rectangle meets the footprint's pixel span
 * [u - hx, u + hx] x [v - hy, v + hy], and the largest weight over the tile,
 * o exp(-q_min / 2), is at least 1/255 (Sec. "CUDA-Related Acceleration Strategies", fast
 * tile-based culling). Signed relative margins of the rounded comparisons:
 *   depth (d - 0.2) / 0.2; determinant det / (s00 s11); opacity 255 o - 1;
 *   span ends (x_hi - (u - hx)) / s and ((u + hx) - x_lo) / s with s = max(1, |u|, hx)
 *   (likewise in y), the pixel-centre comparisons that ceil / floor of the span ends take;
 *   cull: the smaller of 255 o exp(-q_min / 2) - 1 (the largest weight relative to 1/255) and
 *   (kappa^2 - q_min) / (|grad q_min| max(1, |u|, |v|)), the shift of the centre, relative to
 *   its coordinates, that moves q_min onto kappa^2 (a float32 centre is off by a few units in
 *   the last place of u and v, which the small footprints of distant Gaussians magnify).
 * The exact tests (finite inputs, |q| > 0, S > 0) have no margin. */
void or_pair_margins(const or_gaussians *G, const or_camera *cam, int bw, int bh, int64_t m, const int32_t *gid,
                     const int32_t *tile, int8_t *listed, double *margin) {
  tiling tg = make_tiling(cam, bw, bh);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    proj p;
    project(G, cam, gid[i], &p, NULL);
    conj c = {1, INFINITY, 0.0};
    int exact_ok = finite3(p.m) && finite3(p.S) && isfinite(p.qraw[0]) && isfinite(p.qraw[1]) &&
                   isfinite(p.qraw[2]) && isfinite(p.qraw[3]) && isfinite(p.o) && p.qlen > 0 && p.S[0] > 0 &&
                   p.S[1] > 0 && p.S[2] > 0;
    if (!exact_ok) {
      listed[i] = 0;
      margin[i] = INFINITY;
      continue;
    }
    conj_add(&c, (p.d - OR_NEAR) / OR_NEAR);
    if (p.d > OR_NEAR) {
      conj_add(&c, p.det / (p.s00 * p.s11));
      conj_add(&c, 255.0 * p.o - 1.0);
    }
    if (c.all_true) {
      int tx = tile[i] % tg.tiles_x, ty = tile[i] / tg.tiles_x;
      double xl, xh, yl, yh;
      tile_rect(cam, &tg, tx, ty, &xl, &xh, &yl, &yh);
      double sx = fmax(1.0, fmax(fabs(p.u), p.hx)), sy = fmax(1.0, fmax(fabs(p.v), p.hy));
      conj_add(&c, (xh - (p.u - p.hx)) / sx);
      conj_add(&c, ((p.u + p.hx) - xl) / sx);
      conj_add(&c, (yh - (p.v - p.hy)) / sy);
      conj_add(&c, ((p.v + p.hy) - yl) / sy);
      double dx, dy;
      double q = rect_qmin_arg(p.u, p.v, p.a, p.b, p.c, xl, xh, yl, yh, &dx, &dy);
      /* the cull flips when the largest weight moves by its margin relative to 1/255, or when
         the centre moves by (kappa^2 - q_min) / |grad q_min|; the gradient of the minimum with
         respect to the centre is -2 Q D at the minimiser D (zero inside the rectangle) */
      double wm = expm1(0.5 * (p.kappa2 - q));
      double gx = 2.0 * (p.a * dx + p.b * dy), gy = 2.0 * (p.b * dx + p.c * dy);
      double gn = sqrt(gx * gx + gy * gy);
      double pm = gn > 0 ? (p.kappa2 - q) / (gn * fmax(1.0, fmax(fabs(p.u), fabs(p.v)))) : wm;
      conj_add(&c, fabs(pm) < fabs(wm) ? pm : wm);
    }
    listed[i] = (int8_t)c.all_true;
    margin[i] = c.all_true ? c.min_true : c.max_false;
  }
}

/* Gaussians that take a marginal decision at some pixel of the window: weight within the
 * relative band of 1/255 (enters or not) or of 0.99 (clamped or not), or the transmittance
 * after it within the band of 1e-4 (blended or the stop). Their gradients may differ between
 * two correct implementations by a whole pixel's term, so element-wise gradient comparisons
 * leave them out (the pose gradient, a sum over all Gaussians, keeps them). flag [n]. */
int or_marginal_gaussians(const or_gaussians *G, const or_camera *cam, int bw, int bh, double band, uint8_t *flag) {
  if (bw <= 0 || bh <= 0 || cam->w <= 0 || cam->h <= 0) return 1;
  proj *P = project_all(G, cam);
  tiling tg = make_tiling(cam, bw, bh);
  tile_lists L;
  build_lists(P, G->n, cam, &tg, 1, 2.5 * band, &L);
  memset(flag, 0, (size_t)G->n);
  const int64_t T = (int64_t)tg.tiles_x * tg.tiles_y;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t tt = 0; tt < T; ++tt) {
    int tx = (int)(tt % tg.tiles_x), ty = (int)(tt / tg.tiles_x);
    const int32_t *ids = L.ids + L.start[tt];
    const int64_t len = L.start[tt + 1] - L.start[tt];
    for (int j = 0; j < bh; ++j)
      for (int i = 0; i < bw; ++i) {
        int lx = tx * bw + i, ly = ty * bh + j;
        if (lx >= cam->w || ly >= cam->h) continue;
        double T_ = 1.0;
        for (int64_t k = 0; k < len; ++k) {
          const proj *p = &P[ids[k]];
          double araw = pixel_alpha_raw(p, cam->x0 + lx, cam->y0 + ly, NULL);
          int m = fabs(araw - OR_ALPHA_MIN) <= band * OR_ALPHA_MIN;
          double alpha = araw < OR_ALPHA_MAX ? araw : OR_ALPHA_MAX;
          if (alpha >= OR_ALPHA_MIN) {
            double Tn = T_ * (1.0 - alpha);
            m |= fabs(Tn - OR_T_MIN) <= band * OR_T_MIN;
            m |= fabs(araw - OR_ALPHA_MAX) <= band * OR_ALPHA_MAX;
            if (m) {
#pragma omp atomic write
              flag[ids[k]] = 1;
            }
            if (Tn < OR_T_MIN) break;
            T_ = Tn;
          } else if (m) {
#pragma omp atomic write
            flag[ids[k]] = 1;
          }
        }
      }
  }
  free(L.start); free(L.ids); free(P);
  return 0;
}

/* Thread count of the OpenMP loops (for timing the oracle at one and at all threads). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }
