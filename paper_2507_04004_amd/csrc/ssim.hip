// D-SSIM term of the photometric tracking loss (eq:tracking_loss, the D-SSIM term of the
// original 3DGS loss): weight * (1 - mean SSIM) over pixels and channels, and its gradient
// added to dL/dC. SSIM per channel from the local statistics under an 11x11 Gaussian window
// (sigma 1.5, weights summing to one), zero outside the image, C1 = 0.01^2, C2 = 0.03^2:
//   S = A B / (C D),  A = 2 mu_x mu_y + C1,  B = 2 s_xy + C2,  C = mu_x^2 + mu_y^2 + C1,
//   D = s_x^2 + s_y^2 + C2,  with mu = G*x, s_x^2 = G*x^2 - mu_x^2, s_xy = G*(x y) - mu_x mu_y.
// The window is separable (efficient SSIM, Sec. "Additional Strategies", c): each workgroup
// stages a 32x32 tile of one channel plus a 5-pixel halo in LDS and filters rows, then columns;
// in both passes a lane computes 4 consecutive outputs from 14 inputs held in registers.
//
// Forward: the five filtered maps give S; with g = -weight / (c h w) the kernel writes, per
// pixel, the derivatives of g S w.r.t. the three maps that depend on x:
//   d mu_x = g (2 mu_y (S/A - S/B) + 2 mu_x (S/D - S/C)),  d E[x^2] = -g S/D,  d E[xy] = 2 g S/B
// (mu_x enters A, B through s_xy, C and D through s_x^2), and one partial sum of S per
// workgroup; the loss weight + g sum S is then summed in a fixed order (deterministic), by
// one extra workgroup of the backward launch (or its own launch when no gradient is asked).
// Backward: the window is symmetric, so the adjoint of each filtering is the same filtering:
//   dL/dx = G * d mu_x + 2 x (G * d E[x^2]) + y (G * d E[xy]).
#include <cmath>

#include "gs_internal.hpp"

namespace gs {

constexpr int kSsimR = 5;                  // window radius
constexpr int kSsimTX = 32, kSsimTY = 32;  // output tile
constexpr int kSsimW = kSsimTX + 2 * kSsimR, kSsimH = kSsimTY + 2 * kSsimR;  // tile + halo (42 x 42)
constexpr int kSsimLW = 44;               // LDS row stride of the halo tile (16-byte rows)
constexpr int kSeg = 4;                   // outputs per lane and pass (register sliding)
constexpr int kSegIn = kSeg + 2 * kSsimR; // 14 inputs per segment
constexpr int kRowJobs = kSsimH * (kSsimTX / kSeg);  // 42 rows x 8 segments
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

// Zero-padded loads of a tile and its halo from M planes into LDS (rows of kSsimLW floats).
// Every load of the workgroup is issued before the first LDS store, so the wait is one
// memory latency.
constexpr int kHaloElems = kSsimW * kSsimH;
constexpr int kHaloIters = (kHaloElems + 255) / 256;
template <int M>
__device__ __forceinline__ void load_halo(const float *const (&src)[M], int h, int w, int x0, int y0,
                                          float *const (&dst)[M]) {
  float v[M][kHaloIters];
  int64_t off[kHaloIters];
  bool ok[kHaloIters];
  int lo[kHaloIters];
#pragma unroll
  for (int i = 0; i < kHaloIters; ++i) {
    const int k = threadIdx.x + 256 * i;
    const int ly = k / kSsimW, lx = k - ly * kSsimW;
    const int gy = y0 + ly - kSsimR, gx = x0 + lx - kSsimR;
    ok[i] = k < kHaloElems && gy >= 0 && gy < h && gx >= 0 && gx < w;
    off[i] = ok[i] ? (int64_t)gy * w + gx : 0;
    lo[i] = ly * kSsimLW + lx;
  }
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i) v[m][i] = ok[i] ? src[m][off[i]] : 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i)
      if (threadIdx.x + 256 * i < kHaloElems) dst[m][lo[i]] = v[m][i];
}

// The 14 inputs of a row segment (16-byte LDS reads; the last two values are unused).
__device__ __forceinline__ void row_inputs(const float *row, float (&u)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 f = reinterpret_cast<const float4 *>(row)[q];
    u[4 * q] = f.x; u[4 * q + 1] = f.y; u[4 * q + 2] = f.z; u[4 * q + 3] = f.w;
  }
}

__global__ __launch_bounds__(256) void k_dssim_fwd(const float *__restrict__ x, const float *__restrict__ y, int h,
                                                   int w, int nbx, int nby, int nbc, SsimWeights sw, float g,
                                                   float *__restrict__ dmu, float *__restrict__ dxx,
                                                   float *__restrict__ dxy, float *__restrict__ partial) {
  __shared__ __align__(16) float sx[kSsimH * kSsimLW], sy[kSsimH * kSsimLW];
  __shared__ __align__(16) float hs[5][kSsimH * kSsimTX];
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
  // rows: 4 consecutive outputs per lane from 14 staged inputs of each image
  for (int j = threadIdx.x; j < kRowJobs; j += 256) {
    const int r = j >> 3, seg = j & 7;
    float u[16], v[16];
    row_inputs(sx + r * kSsimLW + seg * kSeg, u);
    row_inputs(sy + r * kSsimLW + seg * kSeg, v);
    float uu[kSegIn], vv[kSegIn], uv[kSegIn];
#pragma unroll
    for (int i = 0; i < kSegIn; ++i) {
      uu[i] = u[i] * u[i];
      vv[i] = v[i] * v[i];
      uv[i] = u[i] * v[i];
    }
    float o[5][kSeg];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
      for (int t = 0; t <= 2 * kSsimR; ++t) {
        const float wt = sw.w[t];
        a += wt * u[k + t];
        b += wt * v[k + t];
        aa += wt * uu[k + t];
        bb += wt * vv[k + t];
        ab += wt * uv[k + t];
      }
      o[0][k] = a; o[1][k] = b; o[2][k] = aa; o[3][k] = bb; o[4][k] = ab;
    }
#pragma unroll
    for (int m = 0; m < 5; ++m)
      reinterpret_cast<float4 *>(hs[m] + r * kSsimTX + seg * kSeg)[0] = make_float4(o[m][0], o[m][1], o[m][2], o[m][3]);
  }
  __syncthreads();
  // columns: lane (col, seg) slides down 4 outputs of one column
  const int col = threadIdx.x & (kSsimTX - 1), seg = threadIdx.x >> 5;
  float st[5][kSeg];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    float in[kSegIn];
#pragma unroll
    for (int i = 0; i < kSegIn; ++i) in[i] = hs[m][(seg * kSeg + i) * kSsimTX + col];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      float a = 0.f;
#pragma unroll
      for (int t = 0; t <= 2 * kSsimR; ++t) a += sw.w[t] * in[k + t];
      st[m][k] = a;
    }
  }
  float part = 0.f;
  const int gx = x0 + col;
#pragma unroll
  for (int k = 0; k < kSeg; ++k) {
    const int gy = y0 + seg * kSeg + k;
    if (gy >= h || gx >= w) continue;
    const float mx = st[0][k], my = st[1][k], exx = st[2][k], eyy = st[3][k], exy = st[4][k];
    const float A = 2.f * mx * my + kC1, B = 2.f * (exy - mx * my) + kC2;
    const float Cc = mx * mx + my * my + kC1, D = (exx - mx * mx) + (eyy - my * my) + kC2;
    // one division: with r = 1 / (C D), S = A B r, S/A = B r, S/B = A r, S/C = S D r, S/D = S C r
    const float rr = 1.0f / (Cc * D);
    const float S = A * B * rr;
    const float sA = B * rr, sB = A * rr, sC = S * D * rr, sD = S * Cc * rr;
    part += S;
    const int64_t p = c * plane + (int64_t)gy * w + gx;
    dmu[p] = g * (2.f * my * (sA - sB) + 2.f * mx * (sD - sC));
    dxx[p] = -g * sD;
    dxy[p] = 2.f * g * sB;
  }
  // the block's sum of S, reduced in a fixed order by k_dssim_loss
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) partial[tile.id] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss = weight + g * sum of the block partials (float64, fixed order): deterministic. One
// workgroup; `red` holds 256 doubles of LDS.
__device__ __forceinline__ void dssim_loss_sum(const float *__restrict__ partial, int64_t nb, float weight, double g,
                                               float *__restrict__ loss, double *red) {
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

__global__ __launch_bounds__(256) void k_dssim_loss(const float *__restrict__ partial, int64_t nb, float weight,
                                                    double g, float *__restrict__ loss) {
  __shared__ double red[256];
  dssim_loss_sum(partial, nb, weight, g, loss, red);
}

struct DssimLoss {  // the loss sum run by the backward's last workgroup (loss == null: none)
  const float *partial;
  int64_t nb;
  float weight;
  double g;
  float *loss;
};

__global__ __launch_bounds__(256) void k_dssim_bwd(const float *__restrict__ x, const float *__restrict__ y, int h,
                                                   int w, int nbx, int nby, int nbc, SsimWeights sw,
                                                   const float *__restrict__ dmu, const float *__restrict__ dxx,
                                                   const float *__restrict__ dxy, float *__restrict__ dldc,
                                                   DssimLoss ls) {
  __shared__ __align__(16) float sm[3][kSsimH * kSsimLW];
  __shared__ __align__(16) float hs[3][kSsimH * kSsimTX];
  if (ls.loss && blockIdx.x == gridDim.x - 1) {  // the extra workgroup: the loss, in parallel with the tiles
    dssim_loss_sum(ls.partial, ls.nb, ls.weight, ls.g, ls.loss, reinterpret_cast<double *>(sm[0]));
    return;
  }
  SsimTile tile;
  if (!ssim_tile(nbx, nby, nbc, tile)) return;
  const int c = tile.c;
  const int64_t plane = (int64_t)h * w;
  const int x0 = tile.tx * kSsimTX, y0 = tile.ty * kSsimTY;
  {
    const float *const src[3] = {dmu + c * plane, dxx + c * plane, dxy + c * plane};
    float *const dst[3] = {sm[0], sm[1], sm[2]};
    load_halo<3>(src, h, w, x0, y0, dst);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kRowJobs; j += 256) {
    const int r = j >> 3, seg = j & 7;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float u[16];
      row_inputs(sm[m] + r * kSsimLW + seg * kSeg, u);
      float o[kSeg];
#pragma unroll
      for (int k = 0; k < kSeg; ++k) {
        float a = 0.f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) a += sw.w[t] * u[k + t];
        o[k] = a;
      }
      reinterpret_cast<float4 *>(hs[m] + r * kSsimTX + seg * kSeg)[0] = make_float4(o[0], o[1], o[2], o[3]);
    }
  }
  __syncthreads();
  const int col = threadIdx.x & (kSsimTX - 1), seg = threadIdx.x >> 5;
  float st[3][kSeg];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    float in[kSegIn];
#pragma unroll
    for (int i = 0; i < kSegIn; ++i) in[i] = hs[m][(seg * kSeg + i) * kSsimTX + col];
#pragma unroll
    for (int k = 0; k < kSeg; ++k) {
      float a = 0.f;
#pragma unroll
      for (int t = 0; t <= 2 * kSsimR; ++t) a += sw.w[t] * in[k + t];
      st[m][k] = a;
    }
  }
  const int gx = x0 + col;
#pragma unroll
  for (int k = 0; k < kSeg; ++k) {
    const int gy = y0 + seg * kSeg + k;
    if (gy >= h || gx >= w) continue;
    const int64_t p = c * plane + (int64_t)gy * w + gx;
    dldc[p] += st[0][k] + 2.f * x[p] * st[1][k] + y[p] * st[2][k];
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
  if (dldc) {
    // the backward carries the loss sum in one extra workgroup
    const DssimLoss ls{partial, nb, weight, gd, loss};
    const dim3 gridb(grid.x + (loss ? 1u : 0u));
    hipLaunchKernelGGL(k_dssim_bwd, gridb, dim3(256), 0, st, x, y, h, w, nbx, nby, c, sw, dmu, dxx, dxy, dldc, ls);
  } else if (loss) {
    hipLaunchKernelGGL(k_dssim_loss, dim3(1), dim3(256), 0, st, partial, nb, weight, gd, loss);
  }
  return hipGetLastError();
}

}  // namespace gs
