// D-SSIM term of the photometric tracking loss (eq:tracking_loss, the D-SSIM term of the
// original 3DGS loss): weight * (1 - mean SSIM) over pixels and channels, and its gradient
// added to dL/dC. SSIM per channel from the local statistics under an 11x11 Gaussian window
// (sigma 1.5, weights summing to one), zero outside the image, C1 = 0.01^2, C2 = 0.03^2:
//   S = A B / (C D),  A = 2 mu_x mu_y + C1,  B = 2 s_xy + C2,  C = mu_x^2 + mu_y^2 + C1,
//   D = s_x^2 + s_y^2 + C2,  with mu = G*x, s_x^2 = G*x^2 - mu_x^2, s_xy = G*(x y) - mu_x mu_y.
// The window is separable (efficient SSIM, Sec. "Additional Strategies", c): each workgroup
// stages a 32x16 tile of one channel plus a 5-pixel halo in LDS and filters rows, then columns.
//
// Forward: the five filtered maps give S; with g = -weight / (c h w) the kernel writes, per
// pixel, the derivatives of g S w.r.t. the three maps that depend on x:
//   d mu_x = g (2 mu_y (S/A - S/B) + 2 mu_x (S/D - S/C)),  d E[x^2] = -g S/D,  d E[xy] = 2 g S/B
// (mu_x enters A, B through s_xy, C and D through s_x^2), and one partial sum of S per
// workgroup; the loss weight + g sum S is then summed in a fixed order (deterministic).
// Backward: the window is symmetric, so the adjoint of each filtering is the same filtering:
//   dL/dx = G * d mu_x + 2 x (G * d E[x^2]) + y (G * d E[xy]).
#include <cmath>

#include "gs_internal.hpp"

namespace gs {

constexpr int kSsimR = 5;               // window radius
constexpr int kSsimTX = 32, kSsimTY = 16;  // output tile
constexpr int kSsimW = kSsimTX + 2 * kSsimR, kSsimH = kSsimTY + 2 * kSsimR;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct SsimWeights {
  float w[2 * kSsimR + 1];
};

// Tile of this workgroup. Workgroups are dealt to the 8 XCDs round-robin by launch index;
// the remap gives each XCD one contiguous run of tiles (whole rows of tiles), so the halo a
// tile shares with its neighbours is read once into that XCD's L2 instead of into several.
// The grid is rounded up to a multiple of 8; indices past the last tile return.
constexpr int kSsimXcds = 8;
struct SsimTile {
  int tx, ty, c;
  int64_t id;
};
__device__ __forceinline__ bool ssim_tile(int nbx, int nby, int nbc, SsimTile &t) {
  const int64_t total = (int64_t)nbx * nby * nbc;
  const int64_t per = (total + kSsimXcds - 1) / kSsimXcds;
  const int64_t b = blockIdx.x;
  t.id = (b % kSsimXcds) * per + b / kSsimXcds;
  if (t.id >= total) return false;
  t.c = (int)(t.id / ((int64_t)nbx * nby));
  const int64_t r = t.id - (int64_t)t.c * nbx * nby;
  t.ty = (int)(r / nbx);
  t.tx = (int)(r - (int64_t)t.ty * nbx);
  return true;
}

// Zero-padded loads of a tile and its halo from M planes into LDS. Every load of the
// workgroup is issued before the first LDS store, so the wait is one memory latency.
constexpr int kHaloElems = kSsimW * kSsimH;
constexpr int kHaloIters = (kHaloElems + 255) / 256;
template <int M>
__device__ __forceinline__ void load_halo(const float *const (&src)[M], int h, int w, int x0, int y0,
                                          float *const (&dst)[M]) {
  float v[M][kHaloIters];
  int64_t off[kHaloIters];
  bool ok[kHaloIters];
#pragma unroll
  for (int i = 0; i < kHaloIters; ++i) {
    const int k = threadIdx.x + 256 * i;
    const int ly = k / kSsimW, lx = k - ly * kSsimW;
    const int gy = y0 + ly - kSsimR, gx = x0 + lx - kSsimR;
    ok[i] = k < kHaloElems && gy >= 0 && gy < h && gx >= 0 && gx < w;
    off[i] = ok[i] ? (int64_t)gy * w + gx : 0;
  }
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i) v[m][i] = ok[i] ? src[m][off[i]] : 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i) {
      const int k = threadIdx.x + 256 * i;
      if (k < kHaloElems) dst[m][k] = v[m][i];
    }
}

__global__ __launch_bounds__(256) void k_dssim_fwd(const float *__restrict__ x, const float *__restrict__ y, int h,
                                                   int w, int nbx, int nby, int nbc, SsimWeights sw, float g,
                                                   float *__restrict__ dmu, float *__restrict__ dxx,
                                                   float *__restrict__ dxy, float *__restrict__ partial) {
  __shared__ float sx[kSsimW * kSsimH], sy[kSsimW * kSsimH];
  __shared__ float hs[5][kSsimH * kSsimTX];
  __shared__ float red[4];
  SsimTile tile;
  if (!ssim_tile(nbx, nby, nbc, tile)) return;  // whole workgroup, before any barrier
  const int c = tile.c;
  const int64_t plane = (int64_t)h * w;
  const int x0 = tile.tx * kSsimTX, y0 = tile.ty * kSsimTY;
  {
    const float *const src[2] = {x + c * plane, y + c * plane};
    float *const dst[2] = {sx, sy};
    load_halo<2>(src, h, w, x0, y0, dst);
  }
  __syncthreads();
  // rows: every halo row, the tile's columns
  for (int k = threadIdx.x; k < kSsimH * kSsimTX; k += 256) {
    const int r = k / kSsimTX, col = k - r * kSsimTX;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; ++t) {
      const float u = sx[r * kSsimW + col + t], v = sy[r * kSsimW + col + t], wt = sw.w[t];
      a += wt * u;
      b += wt * v;
      aa += wt * (u * u);
      bb += wt * (v * v);
      ab += wt * (u * v);
    }
    hs[0][k] = a; hs[1][k] = b; hs[2][k] = aa; hs[3][k] = bb; hs[4][k] = ab;
  }
  __syncthreads();
  float part = 0.f;
  for (int k = threadIdx.x; k < kSsimTY * kSsimTX; k += 256) {
    const int r = k / kSsimTX, col = k - r * kSsimTX;
    const int gy = y0 + r, gx = x0 + col;
    if (gy >= h || gx >= w) continue;
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; ++t) {
      const int i = (r + t) * kSsimTX + col;
      const float wt = sw.w[t];
      mx += wt * hs[0][i];
      my += wt * hs[1][i];
      exx += wt * hs[2][i];
      eyy += wt * hs[3][i];
      exy += wt * hs[4][i];
    }
    const float A = 2.f * mx * my + kC1, B = 2.f * (exy - mx * my) + kC2;
    const float Cc = mx * mx + my * my + kC1, D = (exx - mx * mx) + (eyy - my * my) + kC2;
    const float S = (A * B) / (Cc * D);
    part += S;
    const int64_t p = c * plane + (int64_t)gy * w + gx;
    dmu[p] = g * (2.f * my * (S / A - S / B) + 2.f * mx * (S / D - S / Cc));
    dxx[p] = -g * (S / D);
    dxy[p] = 2.f * g * (S / B);
  }
  // the block's sum of S, reduced in a fixed order by k_dssim_loss
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) partial[tile.id] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss = weight + g * sum of the block partials (float64, fixed order): deterministic.
__global__ __launch_bounds__(256) void k_dssim_loss(const float *__restrict__ partial, int64_t nb, float weight,
                                                    double g, float *__restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = threadIdx.x; b < nb; b += 256) s += (double)partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)((double)weight + g * red[0]);
}

__global__ __launch_bounds__(256) void k_dssim_bwd(const float *__restrict__ x, const float *__restrict__ y, int h,
                                                   int w, int nbx, int nby, int nbc, SsimWeights sw,
                                                   const float *__restrict__ dmu, const float *__restrict__ dxx,
                                                   const float *__restrict__ dxy, float *__restrict__ dldc) {
  __shared__ float s0[kSsimW * kSsimH], s1[kSsimW * kSsimH], s2[kSsimW * kSsimH];
  __shared__ float hs[3][kSsimH * kSsimTX];
  SsimTile tile;
  if (!ssim_tile(nbx, nby, nbc, tile)) return;
  const int c = tile.c;
  const int64_t plane = (int64_t)h * w;
  const int x0 = tile.tx * kSsimTX, y0 = tile.ty * kSsimTY;
  {
    const float *const src[3] = {dmu + c * plane, dxx + c * plane, dxy + c * plane};
    float *const dst[3] = {s0, s1, s2};
    load_halo<3>(src, h, w, x0, y0, dst);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSsimH * kSsimTX; k += 256) {
    const int r = k / kSsimTX, col = k - r * kSsimTX;
    float a = 0.f, b = 0.f, d = 0.f;
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; ++t) {
      const int i = r * kSsimW + col + t;
      const float wt = sw.w[t];
      a += wt * s0[i];
      b += wt * s1[i];
      d += wt * s2[i];
    }
    hs[0][k] = a; hs[1][k] = b; hs[2][k] = d;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSsimTY * kSsimTX; k += 256) {
    const int r = k / kSsimTX, col = k - r * kSsimTX;
    const int gy = y0 + r, gx = x0 + col;
    if (gy >= h || gx >= w) continue;
    float P = 0.f, Q = 0.f, R = 0.f;
#pragma unroll
    for (int t = 0; t <= 2 * kSsimR; ++t) {
      const int i = (r + t) * kSsimTX + col;
      const float wt = sw.w[t];
      P += wt * hs[0][i];
      Q += wt * hs[1][i];
      R += wt * hs[2][i];
    }
    const int64_t p = c * plane + (int64_t)gy * w + gx;
    dldc[p] += P + 2.f * x[p] * Q + y[p] * R;
  }
}

__global__ void k_set_f32(float *p, float v) { *p = v; }

namespace {
int64_t dssim_blocks(int c, int h, int w) {
  return (int64_t)c * ((w + kSsimTX - 1) / kSsimTX) * ((h + kSsimTY - 1) / kSsimTY);
}
}  // namespace

// three derivative maps per value, then one partial sum per workgroup
size_t dssim_scratch_bytes(int c, int h, int w) {
  return 3 * sizeof(float) * (size_t)c * h * w + sizeof(float) * (size_t)dssim_blocks(c, h, w);
}

// Enough for any window of at most `pixels` pixels and sides up to 32768, three channels.
size_t dssim_scratch_bound(int64_t pixels) {
  const int64_t blocks = pixels / (kSsimTX * kSsimTY) + 32768 / kSsimTX + 32768 / kSsimTY + 1;
  return 3 * sizeof(float) * 3 * (size_t)pixels + sizeof(float) * 3 * (size_t)blocks;
}

hipError_t launch_dssim(const float *x, const float *y, int c, int h, int w, float weight, float *dldc, float *loss,
                        float *scratch, hipStream_t st) {
  SsimWeights sw;
  double tot = 0.0, wd[2 * kSsimR + 1];
  for (int t = 0; t <= 2 * kSsimR; ++t) {
    const double r = t - kSsimR;
    wd[t] = std::exp(-r * r / (2.0 * 1.5 * 1.5));
    tot += wd[t];
  }
  for (int t = 0; t <= 2 * kSsimR; ++t) sw.w[t] = (float)(wd[t] / tot);
  const int64_t n = (int64_t)c * h * w;
  if (n == 0) {
    if (loss) hipLaunchKernelGGL(k_set_f32, dim3(1), dim3(1), 0, st, loss, weight);
    return hipGetLastError();
  }
  const double gd = -(double)weight / (double)n;
  const float g = (float)gd;
  float *dmu = scratch, *dxx = scratch + n, *dxy = scratch + 2 * n, *partial = scratch + 3 * n;
  const int nbx = (w + kSsimTX - 1) / kSsimTX, nby = (h + kSsimTY - 1) / kSsimTY;
  const int64_t nb = dssim_blocks(c, h, w);
  const dim3 grid((unsigned)((nb + kSsimXcds - 1) / kSsimXcds * kSsimXcds));
  hipLaunchKernelGGL(k_dssim_fwd, grid, dim3(256), 0, st, x, y, h, w, nbx, nby, c, sw, g, dmu, dxx, dxy, partial);
  if (loss) hipLaunchKernelGGL(k_dssim_loss, dim3(1), dim3(256), 0, st, partial, nb, weight, gd, loss);
  if (dldc)
    hipLaunchKernelGGL(k_dssim_bwd, grid, dim3(256), 0, st, x, y, h, w, nbx, nby, c, sw, dmu, dxx, dxy, dldc);
  return hipGetLastError();
}

}  // namespace gs
