// Map initialization and expansion (Sec. "Initialization of Gaussian Map" and Sec.
// "Expansion of Gaussian Map"): the points that project into the keyframe's newly observed
// region (rendered opacity O < tau at their nearest pixel; every point in front of the near
// plane when there is no opacity map) become Gaussians at their 3D location with scale
// (d / fx) (1, 1, 1), identity rotation, opacity 0.1 and their colour in the DC coefficient,
// appended after the existing map in point order.
//
// Selection (one pass): each workgroup takes 1024 points, 4 per lane in wavefront-strided
// order, and stores the wavefront ballots of its decisions (a bitmask, 1 bit per point) and
// its count. A single-workgroup scan turns the counts into output offsets and the total.
// Writing (second pass, after the caller has sized the grown map): each selected point's
// position is its workgroup offset plus the popcount of the mask bits before it; it writes the
// per-point planes (mean, scale, DC). The existing Gaussians are copied plane by plane into the
// grown map, whose planes have a larger stride, by the same kernel that fills the new range of
// the constant planes (rotation, opacity, higher SH).
#include <algorithm>
#include <cmath>

#include "gs_internal.hpp"

namespace gs {

namespace {

constexpr int kExpThreads = 256;
constexpr int kExpPer = 4;  // points per lane
constexpr int kExpBlockPts = kExpThreads * kExpPer;
constexpr int kExpWaves = kExpThreads / 64;
constexpr float kY0 = 0.28209479177387814f;  // degree-0 real SH basis value 1 / (2 sqrt(pi))

// The integer decision, in float32 with the projection's operation order (contraction off).
__device__ __forceinline__ bool expand_decide(const ExpandArgs &a, float x, float y, float z, float &pz) {
#pragma clang fp contract(off)
  const float *R = a.R;
  const float px = R[0] * x + R[1] * y + R[2] * z + a.t[0];
  const float py = R[3] * x + R[4] * y + R[5] * z + a.t[1];
  pz = R[6] * x + R[7] * y + R[8] * z + a.t[2];
  if (!(isfinite(x) && isfinite(y) && isfinite(z)) || !(pz > kNear)) return false;
  if (!a.opacity) return true;
  const float u = a.fx * (px / pz) + a.cx;
  const float v = a.fy * (py / pz) + a.cy;
  const float fu = floorf(u + 0.5f), fv = floorf(v + 0.5f);
  if (!(fu >= (float)a.x0 && fu < (float)(a.x0 + a.w) && fv >= (float)a.y0 && fv < (float)(a.y0 + a.h))) return false;
  const int ix = (int)fu - a.x0, iy = (int)fv - a.y0;
  return a.opacity[(int64_t)iy * a.w + ix] < a.tau;
}

}  // namespace

__global__ __launch_bounds__(kExpThreads) void k_expand_select(ExpandArgs a, uint64_t *__restrict__ masks,
                                                                uint32_t *__restrict__ counts) {
  __shared__ uint32_t red[kExpWaves];
  const int64_t base = (int64_t)blockIdx.x * kExpBlockPts;
  const int wave = threadIdx.x >> 6;
  float xs[kExpPer], ys[kExpPer], zs[kExpPer];
#pragma unroll
  for (int j = 0; j < kExpPer; ++j) {  // all loads first
    const int64_t i = base + j * kExpThreads + threadIdx.x;
    const bool in = i < a.n;
    xs[j] = in ? a.xyz[i] : 0.f;
    ys[j] = in ? a.xyz[a.n + i] : 0.f;
    zs[j] = in ? a.xyz[2 * a.n + i] : 0.f;
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kExpPer; ++j) {
    const int64_t i = base + j * kExpThreads + threadIdx.x;
    float pz;
    const bool sel = i < a.n && expand_decide(a, xs[j], ys[j], zs[j], pz);
    const uint64_t m = __ballot(sel);
    if ((threadIdx.x & 63) == 0) masks[(int64_t)blockIdx.x * (kExpPer * kExpWaves) + j * kExpWaves + wave] = m;
    cnt += (uint32_t)__popcll(m);
  }
  if ((threadIdx.x & 63) == 0) red[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Exclusive scan of the workgroup counts into offsets, and the total (one workgroup).
__global__ __launch_bounds__(1024) void k_expand_scan(const uint32_t *__restrict__ counts, int64_t nb,
                                                      uint32_t *__restrict__ offsets, int64_t *__restrict__ total) {
  __shared__ int64_t part[1024];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += counts[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan of the lane sums
    const int64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int64_t b = b0; b < b1; ++b) {
    offsets[b] = (uint32_t)run;
    run += counts[b];
  }
  if (threadIdx.x == 1023 && total) *total = part[1023];
}

// New Gaussians of the selected points at n_old + rank (rank < added, else skipped).
__global__ __launch_bounds__(kExpThreads) void k_expand_write(ExpandArgs a, const uint64_t *__restrict__ masks,
                                                               const uint32_t *__restrict__ offsets,
                                                               ExpandOut o) {
  constexpr int kMasks = kExpPer * kExpWaves;
  __shared__ uint32_t pre[kMasks];
  const int64_t blk = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {  // exclusive scan of the 16 mask popcounts across lanes
    const uint32_t c = lane < kMasks ? (uint32_t)__popcll(masks[blk * kMasks + lane]) : 0u;
    uint32_t incl = c;
#pragma unroll
    for (int off = 1; off < kMasks; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    if (lane < kMasks) pre[lane] = offsets[blk] + incl - c;
  }
  __syncthreads();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t N = o.n;
#pragma unroll
  for (int j = 0; j < kExpPer; ++j) {
    const int k = j * kExpWaves + wave;
    const uint64_t m = masks[blk * kMasks + k];
    if (!((m >> lane) & 1ull)) continue;
    const int64_t rank = (int64_t)pre[k] + __popcll(m & below);
    if (rank >= o.added) continue;
    const int64_t i = blk * kExpBlockPts + j * kExpThreads + threadIdx.x;
    const float x = a.xyz[i], y = a.xyz[a.n + i], z = a.xyz[2 * a.n + i];
    float pz;
    (void)expand_decide(a, x, y, z, pz);
    const int64_t d = o.n_old + rank;
    const float s = pz / a.fx;
    o.mean[d] = x;
    o.mean[N + d] = y;
    o.mean[2 * N + d] = z;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      o.scale[c * N + d] = s;
      o.sh_dc[c * N + d] = (a.rgb[c * a.n + i] - 0.5f) / kY0;
    }
    // rotation, opacity and higher SH are constant planes, filled by k_copy_planes
  }
}

// Plane p of the grown map: elements [0, n_old) copied from the existing map, and on the
// constant planes (rotation, opacity, higher SH) the new elements [n_old, n_new) set to the
// initial value. Each workgroup moves 1024 consecutive elements, every load and store a
// contiguous wavefront run (the plane strides differ, so the runs are not 16-byte aligned in
// general); writing the constant planes here keeps those stores full-width.
__global__ __launch_bounds__(256) void k_copy_planes(PlaneCopy pc, int64_t n_old, int64_t n_new) {
  const int p = blockIdx.y;
  const float *src = pc.src[p] ? pc.src[p] + pc.plane[p] * n_old : nullptr;
  float *dst = pc.dst[p] + pc.plane[p] * n_new;
  const int64_t end = pc.constant[p] ? n_new : n_old;
  const float fill = pc.fill[p];
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  float v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i0 + 256 * k;
    v[k] = i < n_old ? src[i] : fill;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (i0 + 256 * k < end) dst[i0 + 256 * k] = v[k];
}

int64_t expand_blocks(int64_t n) { return (n + kExpBlockPts - 1) / kExpBlockPts; }

size_t expand_scratch_bytes(int64_t n) {
  const int64_t nb = std::max<int64_t>(expand_blocks(n), 1);
  return (size_t)nb * (kExpPer * kExpWaves * sizeof(uint64_t) + 2 * sizeof(uint32_t)) + 256;
}

static void carve(void *scratch, int64_t n, uint64_t *&masks, uint32_t *&counts, uint32_t *&offsets) {
  const int64_t nb = std::max<int64_t>(expand_blocks(n), 1);
  masks = (uint64_t *)scratch;
  counts = (uint32_t *)(masks + nb * kExpPer * kExpWaves);
  offsets = counts + nb;
}

hipError_t launch_expand_select(const ExpandArgs &a, void *scratch, int64_t *total, hipStream_t st) {
  uint64_t *masks;
  uint32_t *counts, *offsets;
  carve(scratch, a.n, masks, counts, offsets);
  const int64_t nb = expand_blocks(a.n);
  if (nb > 0) hipLaunchKernelGGL(k_expand_select, dim3((unsigned)nb), dim3(kExpThreads), 0, st, a, masks, counts);
  hipLaunchKernelGGL(k_expand_scan, dim3(1), dim3(1024), 0, st, counts, nb, offsets, total);
  return hipGetLastError();
}

hipError_t launch_expand_write(const ExpandArgs &a, const void *scratch, const ExpandOut &o, const PlaneCopy &pc,
                               int n_planes, hipStream_t st) {
  uint64_t *masks;
  uint32_t *counts, *offsets;
  carve(const_cast<void *>(scratch), a.n, masks, counts, offsets);
  if (o.n > 0 && n_planes > 0) {
    const dim3 grid((unsigned)((o.n + 1023) / 1024), (unsigned)n_planes);
    hipLaunchKernelGGL(k_copy_planes, grid, dim3(256), 0, st, pc, o.n_old, o.n);
  }
  const int64_t nb = expand_blocks(a.n);
  if (nb > 0 && o.added > 0)
    hipLaunchKernelGGL(k_expand_write, dim3((unsigned)nb), dim3(kExpThreads), 0, st, a, masks, offsets, o);
  return hipGetLastError();
}

}  // namespace gs
