// Stages a3/a4/a6 of the rasterizer: front-to-back alpha compositing of colour, depth and
// opacity per pixel (eq:alpha, eq:rendered_rgb, eq:rendered_depth, eq:rendered_opacity), its
// backward, and the sparse-LiDAR depth term of eq:depth_loss with the opacity-normalised
// depth D/O.
//
// One workgroup per tile (tile_w x tile_h pixels, one lane per pixel, 64-lane wavefronts).
// The tile's depth-sorted records are staged through LDS in batches of BD; every lane reads
// the same LDS word (a broadcast, no bank conflicts). A workgroup leaves as soon as all its
// pixels have stopped (transmittance would fall below 1e-4).
//
// The forward saves only a per-pixel checkpoint: the final transmittance and the position
// of the last blended record. The backward walks each pixel's records from that position
// towards the front, rebuilds the transmittance by division, reduces each record's
// gradient over the wavefront with shuffles and issues one atomic per value per wavefront.
#include <algorithm>

#include "gs_internal.hpp"

namespace gs {

template <int TW, int TH, int BD>
__global__ __launch_bounds__(TW *TH) void k_blend_fwd(ViewTable vt, ImgTable it, const float4 *__restrict__ rec_a,
                                                      const float4 *__restrict__ rec_b,
                                                      const float4 *__restrict__ rgb,
                                                      const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ tile_range) {
  constexpr int NT = TW * TH;
  __shared__ float4 s_a[BD], s_b[BD], s_c[BD];
  const uint32_t gt = blockIdx.x;
  const int vi = view_of_tile(vt, gt);
  const ViewCam &cam = vt.v[vi];
  const uint32_t lt = gt - cam.tile_base;
  const int tx = (int)(lt % (uint32_t)cam.tiles_x), ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int wx = tx * TW + lx, wy = ty * TH + ly;
  const bool inside = wx < cam.w && wy < cam.h;
  const float px = (float)(cam.x0 + wx), py = (float)(cam.y0 + wy);
  const uint32_t start = tile_range[2 * gt], end = tile_range[2 * gt + 1];

  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, O = 0.f;
  int32_t last = -1, ncontrib = 0;
  bool done = !inside;
  for (uint32_t base = start; base < end; base += BD) {
    const int cnt = (int)min<uint32_t>(BD, end - base);
    for (int k = threadIdx.x; k < cnt; k += NT) {
      const uint32_t e = vals[base + k];
      s_a[k] = rec_a[e];
      s_b[k] = rec_b[e];
      s_c[k] = rgb[e];
    }
    __syncthreads();
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 A = s_a[j], B = s_b[j];
        const float power = splat_power(B.x, B.y, B.z, px - A.x, py - A.y);
        const float alpha = fminf(kAlphaMax, splat_alpha_raw(A.z, power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float w = alpha * T;
        const float4 Cc = s_c[j];
        C0 += w * Cc.x;
        C1 += w * Cc.y;
        C2 += w * Cc.z;
        D += w * A.w;
        O += w;
        T = Tn;
        last = (int32_t)(base + j - start);
        ++ncontrib;
      }
    }
    if (__syncthreads_count(done) == NT) break;
  }
  if (inside) {
    const ViewImg &im = it.v[vi];
    const int64_t npx = (int64_t)cam.w * cam.h;
    const int64_t pi = (int64_t)wy * cam.w + wx;
    im.color[pi] = C0 + T * cam.bg[0];
    im.color[npx + pi] = C1 + T * cam.bg[1];
    im.color[2 * npx + pi] = C2 + T * cam.bg[2];
    im.depth[pi] = D;
    im.alpha[pi] = O;
    im.t_final[pi] = T;
    im.last[pi] = last;
    if (im.n_contrib) im.n_contrib[pi] = ncontrib;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int TW, int TH, int BD>
__global__ __launch_bounds__(TW *TH) void k_blend_bwd(ViewTable vt, ImgTable it, GradTable gtab,
                                                      const float4 *__restrict__ rec_a,
                                                      const float4 *__restrict__ rec_b,
                                                      const float4 *__restrict__ rgb,
                                                      const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ tile_range,
                                                      float *__restrict__ g2 /*[E][12]*/) {
  constexpr int NT = TW * TH;
  __shared__ float4 s_a[BD], s_b[BD], s_c[BD];
  __shared__ uint32_t s_e[BD];
  __shared__ int s_maxlast;
  const uint32_t gt = blockIdx.x;
  const int vi = view_of_tile(vt, gt);
  const ViewCam &cam = vt.v[vi];
  const uint32_t lt = gt - cam.tile_base;
  const int tx = (int)(lt % (uint32_t)cam.tiles_x), ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int wx = tx * TW + lx, wy = ty * TH + ly;
  const bool inside = wx < cam.w && wy < cam.h;
  const float px = (float)(cam.x0 + wx), py = (float)(cam.y0 + wy);
  const uint32_t start = tile_range[2 * gt], end = tile_range[2 * gt + 1];
  const int64_t npx = (int64_t)cam.w * cam.h;
  const int64_t pi = (int64_t)wy * cam.w + wx;
  const ViewImg &im = it.v[vi];
  const ViewGrad &vg = gtab.v[vi];

  float Tfin = 1.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f, gO = 0.f;
  int32_t last = -1;
  if (inside) {
    Tfin = im.t_final[pi];
    last = im.last[pi];
    gC0 = vg.gC[pi];
    gC1 = vg.gC[npx + pi];
    gC2 = vg.gC[2 * npx + pi];
    if (vg.gD) gD = vg.gD[pi];
    if (vg.gO) gO = vg.gO[pi];
  }
  if (threadIdx.x == 0) s_maxlast = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&s_maxlast, last);
  __syncthreads();
  const int maxlast = min(s_maxlast, (int)(end - start) - 1);  // a checkpoint never points past the list
  const float gbg = gC0 * cam.bg[0] + gC1 * cam.bg[1] + gC2 * cam.bg[2];
  const float gOb = gO - gbg;
  const int lane = threadIdx.x & 63;

  float T = Tfin, A0 = 0.f, A1 = 0.f, A2 = 0.f, AD = 0.f;
  for (int bend = maxlast + 1; bend > 0; bend -= BD) {
    const int bbeg = max(0, bend - BD);
    const int cnt = bend - bbeg;
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += NT) {
      const uint32_t e = vals[start + bbeg + k];
      s_e[k] = e;
      s_a[k] = rec_a[e];
      s_b[k] = rec_b[e];
      s_c[k] = rgb[e];
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int pos = bbeg + j;
      float g[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) g[q] = 0.f;
      bool contrib = false;
      if (pos <= last) {
        const float4 A = s_a[j], B = s_b[j];
        const float dx = px - A.x, dy = py - A.y;
        const float power = splat_power(B.x, B.y, B.z, dx, dy);
        const float ex = __expf(power);
        const float ar = A.z * ex;  // the same two operations as splat_alpha_raw
        const float alpha = fminf(kAlphaMax, ar);
        if (alpha >= kAlphaMin) {
          contrib = true;
          const float one_m = 1.f - alpha;
          T = T / one_m;  // transmittance in front of this record
          const float w = alpha * T;
          const float4 Cc = s_c[j];
          g[6] = gC0 * w;
          g[7] = gC1 * w;
          g[8] = gC2 * w;
          g[9] = gD * w;
          const float dLda = T * (gC0 * (Cc.x - A0) + gC1 * (Cc.y - A1) + gC2 * (Cc.z - A2) + gD * (A.w - AD)) +
                             (Tfin / one_m) * gOb;
          A0 = alpha * Cc.x + one_m * A0;
          A1 = alpha * Cc.y + one_m * A1;
          A2 = alpha * Cc.z + one_m * A2;
          AD = alpha * A.w + one_m * AD;
          if (ar < kAlphaMax) {
            g[5] = dLda * ex;
            const float dp = dLda * ar;
            g[0] = dp * (B.x * dx + B.y * dy);
            g[1] = dp * (B.y * dx + B.z * dy);
            g[2] = -0.5f * dp * dx * dx;
            g[3] = -dp * dx * dy;
            g[4] = -0.5f * dp * dy * dy;
          }
        }
      }
      if (__any(contrib)) {
        float mine = 0.f;
#pragma unroll
        for (int q = 0; q < 10; ++q) {
          const float s = wave_sum(g[q]);
          mine = lane == q ? s : mine;
        }
        if (lane < 10 && mine != 0.f) unsafeAtomicAdd(&g2[(int64_t)s_e[j] * 12 + lane], mine);
      }
    }
  }
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

// Dense gradient maps = user-given planes (or zero), before the LiDAR term is added.
__global__ __launch_bounds__(256) void k_init_maps(MapSrc src, MapTable dst) {
  const int vi = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= src.npx[vi]) return;
  if (dst.gD[vi]) dst.gD[vi][i] = src.gD[vi] ? src.gD[vi][i] : 0.f;
  if (dst.gO[vi]) dst.gO[vi][i] = src.gO[vi] ? src.gO[vi][i] : 0.f;
}

// ---- RGB L1 term ---------------------------------------------------------------------------
__global__ void k_zero_f32(float *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ __launch_bounds__(256) void k_loss_l1(const float *__restrict__ c, const float *__restrict__ t, int64_t n,
                                                 float weight, float *__restrict__ dldc, float *__restrict__ loss) {
  __shared__ float red[4];
  const float inv = weight / (float)n;
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float r = c[i] - t[i];
    s += fabsf(r);
    if (dldc) dldc[i] = (r > 0.f ? inv : (r < 0.f ? -inv : 0.f));
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) * inv);
}

// ---- dispatch -------------------------------------------------------------------------------
template <int TW, int TH>
static hipError_t blend_fwd_bd(int bd, const ViewTable &vt, const ImgTable &it, const gs_projected &p,
                               const uint32_t *vals, const uint32_t *range, hipStream_t st) {
  const dim3 grid(vt.total_tiles), block(TW * TH);
  switch (bd) {
    case 64:
      hipLaunchKernelGGL((k_blend_fwd<TW, TH, 64>), grid, block, 0, st, vt, it, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range);
      break;
    case 128:
      hipLaunchKernelGGL((k_blend_fwd<TW, TH, 128>), grid, block, 0, st, vt, it, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range);
      break;
    case 256:
      hipLaunchKernelGGL((k_blend_fwd<TW, TH, 256>), grid, block, 0, st, vt, it, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TW, int TH>
static hipError_t blend_bwd_bd(int bd, const ViewTable &vt, const ImgTable &it, const GradTable &gtab,
                               const gs_projected &p, const uint32_t *vals, const uint32_t *range, float *g2,
                               hipStream_t st) {
  const dim3 grid(vt.total_tiles), block(TW * TH);
  switch (bd) {
    case 64:
      hipLaunchKernelGGL((k_blend_bwd<TW, TH, 64>), grid, block, 0, st, vt, it, gtab, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range, g2);
      break;
    case 128:
      hipLaunchKernelGGL((k_blend_bwd<TW, TH, 128>), grid, block, 0, st, vt, it, gtab, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range, g2);
      break;
    case 256:
      hipLaunchKernelGGL((k_blend_bwd<TW, TH, 256>), grid, block, 0, st, vt, it, gtab, (const float4 *)p.rec_a,
                         (const float4 *)p.rec_b, (const float4 *)p.rgb, vals, range, g2);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_blend_fwd(int bd, const ViewTable &vt, const ImgTable &it, const gs_projected &p,
                            const uint32_t *vals, const uint32_t *range, hipStream_t st) {
  if (vt.total_tiles == 0) return hipSuccess;
  if (vt.tile_w == 8 && vt.tile_h == 8) return blend_fwd_bd<8, 8>(bd, vt, it, p, vals, range, st);
  if (vt.tile_w == 16 && vt.tile_h == 16) return blend_fwd_bd<16, 16>(bd, vt, it, p, vals, range, st);
  if (vt.tile_w == 32 && vt.tile_h == 32) return blend_fwd_bd<32, 32>(bd, vt, it, p, vals, range, st);
  return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(int bd, const ViewTable &vt, const ImgTable &it, const GradTable &gtab,
                            const gs_projected &p, const uint32_t *vals, const uint32_t *range, float *g2,
                            hipStream_t st) {
  if (vt.total_tiles == 0) return hipSuccess;
  if (vt.tile_w == 8 && vt.tile_h == 8) return blend_bwd_bd<8, 8>(bd, vt, it, gtab, p, vals, range, g2, st);
  if (vt.tile_w == 16 && vt.tile_h == 16) return blend_bwd_bd<16, 16>(bd, vt, it, gtab, p, vals, range, g2, st);
  if (vt.tile_w == 32 && vt.tile_h == 32) return blend_bwd_bd<32, 32>(bd, vt, it, gtab, p, vals, range, g2, st);
  return hipErrorInvalidValue;
}

hipError_t launch_lidar_loss(const LidarTable &lt, const ImgTable &it, int max_m, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_loss, dim3(1), dim3(64), 0, st, lt);
  if (max_m > 0)
    hipLaunchKernelGGL(k_lidar_loss, dim3((unsigned)((max_m + 255) / 256), (unsigned)lt.n_views), dim3(256), 0, st,
                       lt, it);
  return hipGetLastError();
}

hipError_t launch_grad_maps(const MapSrc &src, const MapTable &dst, int n_views, int64_t max_npx, const LidarTable &lt,
                            const ImgTable &it, int max_m, hipStream_t st) {
  hipLaunchKernelGGL(k_init_maps, dim3((unsigned)((max_npx + 255) / 256), (unsigned)n_views), dim3(256), 0, st, src,
                     dst);
  if (max_m > 0)
    hipLaunchKernelGGL(k_lidar_grad, dim3((unsigned)((max_m + 255) / 256), (unsigned)lt.n_views), dim3(256), 0, st,
                       lt, it, dst);
  return hipGetLastError();
}

hipError_t zero_f32(float *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_loss_l1(const float *c, const float *t, int64_t n, float weight, float *dldc, float *loss,
                          hipStream_t st) {
  if (loss) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, loss, (int64_t)1);
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  if (n > 0)
    hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, c, t, n, weight,
                       dldc, loss);
  return hipGetLastError();
}

}  // namespace gs
