// Stage a6 of the rasterizer, the sparse-LiDAR depth term of eq:depth_loss with the
// opacity-normalised depth D/O (loss in the forward, gradient maps for the backward), and
// the RGB L1 term of the mapping loss.
#include <algorithm>

#include "gs_internal.hpp"

namespace gs {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---- LiDAR depth term (a6) -----------------------------------------------------------------
// Forward: L_d = weight / m * sum |D/O - D_s| over hits with O > 0 (loss_out zeroed first).
__global__ __launch_bounds__(256) void k_lidar_loss(LidarTable lt, ImgTable it) {
  __shared__ float red[4];
  const int vi = blockIdx.y;
  const LidarView &L = lt.v[vi];
  const int i = blockIdx.x * 256 + threadIdx.x;
  float s = 0.f;
  if (i < L.m) {
    const int p = L.pix[i];
    if (p >= 0 && p < L.npx) {
      const float D = it.v[vi].depth[p], O = it.v[vi].alpha[p];
      if (O > 0.f) s = fabsf(D / O - L.target[i]);
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && L.m > 0 && (int64_t)blockIdx.x * 256 < L.m)
    atomicAdd(L.loss_out, (red[0] + red[1] + red[2] + red[3]) * (L.weight / (float)L.m));
}

__global__ void k_zero_loss(LidarTable lt) {
  const int vi = threadIdx.x;
  if (vi < lt.n_views && lt.v[vi].m > 0 && lt.v[vi].loss_out) *lt.v[vi].loss_out = 0.f;
}

// Backward: adds the LiDAR term's gradient to the view's dense depth / opacity gradient maps.

__global__ __launch_bounds__(256) void k_lidar_grad(LidarTable lt, ImgTable it, MapTable mt) {
  const int vi = blockIdx.y;
  const LidarView &L = lt.v[vi];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= L.m) return;
  const int p = L.pix[i];
  if (p < 0 || p >= L.npx) return;
  const float D = it.v[vi].depth[p], O = it.v[vi].alpha[p];
  if (!(O > 0.f)) return;
  const float r = D / O - L.target[i];
  const float sg = (r > 0.f) ? 1.f : (r < 0.f ? -1.f : 0.f);
  const float scale = L.grad_scale ? *L.grad_scale : 1.f;
  const float s = sg * scale * (L.weight / (float)L.m);
  mt.gD[vi][p] += s / O;
  mt.gO[vi][p] += -s * D / (O * O);
}

// Backward preparation in one pass: grad2d (n floats, float4 stores when vec) zeroed and the
// dense gradient maps of the views set to the caller's planes (or zero), before the LiDAR
// term is added.
__global__ __launch_bounds__(256) void k_bwd_prep(float *__restrict__ g2, int64_t n, int vec, MapSrc src,
                                                  MapTable dst, int n_views, int64_t max_npx) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (vec) {
    float4 *g4 = reinterpret_cast<float4 *>(g2);
    for (int64_t i = t; i < n / 4; i += stride) g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    for (int64_t i = t; i < n; i += stride) g2[i] = 0.f;
  }
  const int64_t total = (int64_t)n_views * max_npx;
  for (int64_t j = t; j < total; j += stride) {
    const int vi = (int)(j / max_npx);
    const int64_t i = j - (int64_t)vi * max_npx;
    if (i >= src.npx[vi]) continue;
    if (dst.gD[vi]) dst.gD[vi][i] = src.gD[vi] ? src.gD[vi][i] : 0.f;
    if (dst.gO[vi]) dst.gO[vi][i] = src.gO[vi] ? src.gO[vi][i] : 0.f;
  }
}

// ---- RGB L1 term ---------------------------------------------------------------------------
__global__ void k_zero_f32(float *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

constexpr int kLossUnroll = 4;

// vec: every pointer is 16-B aligned, so the bulk goes through float4 accesses
__global__ __launch_bounds__(256) void k_loss_l1(const float *__restrict__ c, const float *__restrict__ t, int64_t n,
                                                 float weight, float *__restrict__ dldc, float *__restrict__ loss,
                                                 int vec) {
  __shared__ float red[4];
  const float inv = weight / (float)n;
  auto sgn = [inv](float r) { return r > 0.f ? inv : (r < 0.f ? -inv : 0.f); };
  float s = 0.f;
  // four elements per lane and step (16-B loads and stores), then the tail
  const int64_t n4 = vec ? n / 4 : 0;
  const float4 *c4 = reinterpret_cast<const float4 *>(c), *t4 = reinterpret_cast<const float4 *>(t);
  float4 *d4 = reinterpret_cast<float4 *>(dldc);
  const int64_t stride = (int64_t)gridDim.x * 256;
  // kLossUnroll float4 per lane and step, all requested before the first is used
  for (int64_t i0 = (int64_t)blockIdx.x * (256 * kLossUnroll) + threadIdx.x; i0 < n4; i0 += stride * kLossUnroll) {
    float4 a[kLossUnroll], b[kLossUnroll];
#pragma unroll
    for (int u = 0; u < kLossUnroll; ++u) {
      const int64_t i = i0 + u * 256;
      if (i < n4) {
        a[u] = c4[i];
        b[u] = t4[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kLossUnroll; ++u) {
      const int64_t i = i0 + u * 256;
      if (i < n4) {
        const float r0 = a[u].x - b[u].x, r1 = a[u].y - b[u].y, r2 = a[u].z - b[u].z, r3 = a[u].w - b[u].w;
        s += (fabsf(r0) + fabsf(r1)) + (fabsf(r2) + fabsf(r3));
        if (dldc) d4[i] = make_float4(sgn(r0), sgn(r1), sgn(r2), sgn(r3));
      }
    }
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const float r = c[i] - t[i];
    s += fabsf(r);
    if (dldc) dldc[i] = sgn(r);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) * inv);
}

// ---- launchers ----------------------------------------------------------------------------
hipError_t launch_lidar_loss(const LidarTable &lt, const ImgTable &it, int max_m, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_loss, dim3(1), dim3(64), 0, st, lt);
  if (max_m > 0)
    hipLaunchKernelGGL(k_lidar_loss, dim3((unsigned)((max_m + 255) / 256), (unsigned)lt.n_views), dim3(256), 0, st,
                       lt, it);
  return hipGetLastError();
}

hipError_t launch_bwd_prep(float *g2, int64_t n, const MapSrc &src, const MapTable &dst, int n_views, int64_t max_npx,
                           const LidarTable &lt, const ImgTable &it, int max_m, hipStream_t st) {
  const int vec = (reinterpret_cast<uintptr_t>(g2) & 15u) == 0 && n % 4 == 0;
  const int64_t work = std::max<int64_t>(vec ? n / 4 : n, (int64_t)n_views * max_npx);
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((work + 255) / 256, 1), 8192);
  hipLaunchKernelGGL(k_bwd_prep, dim3((unsigned)blocks), dim3(256), 0, st, g2, n, vec, src, dst, n_views, max_npx);
  if (max_m > 0)
    hipLaunchKernelGGL(k_lidar_grad, dim3((unsigned)((max_m + 255) / 256), (unsigned)lt.n_views), dim3(256), 0, st,
                       lt, it, dst);
  return hipGetLastError();
}

hipError_t launch_loss_l1(const float *c, const float *t, int64_t n, float weight, float *dldc, float *loss,
                          hipStream_t st) {
  if (loss) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, loss, (int64_t)1);
  const int vec = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(t) |
                    reinterpret_cast<uintptr_t>(dldc)) & 15u) == 0;
  // one atomic per block; a block covers 256 * kLossUnroll float4 per step. At most 256 blocks
  // (one per CU), each looping over several steps: at 1280x720 that takes the kernel from 14.1
  // to 9.9 us against 676 blocks of one step (and 12.7 us at 128 blocks).
  const int64_t blocks = std::min<int64_t>((n / 4 + 256 * kLossUnroll - 1) / (256 * kLossUnroll) + 1, 256);
  if (n > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, c, t, n, weight,
                       dldc, loss, vec);
  return hipGetLastError();
}

}  // namespace gs
