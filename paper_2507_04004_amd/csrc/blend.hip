// Stages a3 and a4 of the rasterizer, load-balanced: front-to-back compositing of colour,
// depth and opacity (eq:alpha, eq:rendered_rgb, eq:rendered_depth, eq:rendered_opacity) and
// its backward.
//
// Per-tile list lengths vary by two orders of magnitude (a tile at the vanishing point of a
// street holds tens of thousands of splats, the median tile a hundred), so one workgroup per
// tile leaves the chip idle behind a few long tiles. Each tile's depth-sorted list is cut
// into chunks of BD records; every (tile, chunk) is a work item of one workgroup (one lane per
// pixel, records staged once through LDS and read as a broadcast).
//
// Compositing is associative: a chunk composited from transmittance 1 gives partial sums
// (C_k, D_k, O_k) and a transmittance product T_k, and the pixel's result is
// sum_k T_in,k * C_k with T_in,k the product of the earlier T_k. Only the early stop (stop
// before a splat that would take the transmittance below 1e-4) needs the true incoming
// transmittance, so:
//   1. k_blend_chunk composites every chunk from T = 1. Chunk 0 is exact. A tile with one
//      chunk writes its pixels directly (the common case).
//   2. k_blend_scan walks the chunk partials of each multi-chunk tile in order per pixel. A
//      chunk whose product keeps the transmittance at or above 1e-4 is accumulated as a whole;
//      at the chunk in which the pixel stops it records the incoming state.
//   Passes 1 and 2 run in three windows of chunks (the first kWin0 splats of every list, up
//   to kWin1, the rest): a window's chunks are composited only for the tiles in which some
//   pixel was still running at the end of the previous window. With a pair capacity too small
//   for long lists one window takes every chunk.
//   3. k_blend_fix (one workgroup per chunk, in parallel) composites each pixel's stop chunk
//      again record by record from the true incoming transmittance, which applies the stop
//      rule exactly.
//   4. k_blend_suffix stores, per chunk and pixel, the transmittance after the chunk and the
//      colour / depth composited behind it (normalised by that transmittance): the backward's
//      starting state.
//   5. k_blend_bwd_chunk runs every chunk back to front in parallel from that state,
//      rebuilding each transmittance by division, exactly as a sequential walk would from the
//      last blended splat.
// The per-pixel checkpoint of the forward stays T_final and the position of the last
// blended splat in the tile list; the per-chunk state is 32 B per (chunk, pixel).
#include <algorithm>

#include "gs_internal.hpp"

namespace gs {

struct ChunkRec {
  float c0, c1, c2, d, o, t;
  uint32_t info;  // bits 0-9: local last + 1 (0 = none); 10-19: contributions; 20: stopped inside
  float pad;
};
static_assert(sizeof(ChunkRec) == 32, "chunk record is 32 B");

__host__ __device__ __forceinline__ uint32_t n_chunks(uint32_t len, int bd) { return (len + bd - 1) / bd; }

// ---- work items: (tile, chunk) pairs --------------------------------------------------------
// Items are listed tile by tile in a locality order: stripes of kStripe tile rows, column by
// column inside a stripe, so that consecutive items are spatial neighbours and share splats.
// Workgroups are dealt to the 8 XCDs round-robin; the launch remaps them so that each XCD
// takes whole groups of kGroup consecutive items (neighbouring tiles share that XCD's L2),
// while the groups themselves are dealt round-robin, which keeps the XCDs evenly loaded
// (the work per image band differs by a large factor).
constexpr int kItemThreads = 64;  // one wavefront per 64 tiles: the item pass spreads over the chip
constexpr int kItemPer = 1;
constexpr int kItemChunk = kItemThreads * kItemPer;
constexpr int kStripe = 4;
constexpr uint32_t kXcds = 8;
constexpr uint32_t kGroup = 16;

// Global tile id at position j of the locality order (a bijection within each view).
__device__ __forceinline__ uint32_t tile_at(const ViewTable &vt, uint32_t j) {
  const int vi = view_of_tile(vt, j);
  const ViewCam &cam = vt.v[vi];
  const uint32_t s = j - cam.tile_base;
  const uint32_t tx_n = (uint32_t)cam.tiles_x, ty_n = (uint32_t)cam.tiles_y;
  const uint32_t stripe = s / (kStripe * tx_n);
  const uint32_t r = s - stripe * kStripe * tx_n;
  const uint32_t h = min((uint32_t)kStripe, ty_n - stripe * kStripe);
  const uint32_t tx = r / h, ty = stripe * kStripe + r % h;
  return cam.tile_base + ty * tx_n + tx;
}

// Work item of this workgroup after the XCD remap; false when out of range. Workgroup b runs
// on XCD b % 8 as its (b / 8)-th workgroup there.
__device__ __forceinline__ bool item_of_block(const uint32_t *n_items, uint32_t &item) {
  const uint32_t x = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
  item = ((k / kGroup) * kXcds + x) * kGroup + k % kGroup;
  return item < *n_items;
}

// Per block of tiles: the number of items and of first-window work items (chunks below w0).
__global__ __launch_bounds__(kItemThreads) void k_items_reduce(ViewTable vt, const uint32_t *__restrict__ range,
                                                                int bd, uint32_t w0, uint32_t *__restrict__ bsum,
                                                                uint32_t *__restrict__ bsum0) {
  __shared__ uint32_t lds[kItemThreads / 64 + 1];
  const uint32_t T = vt.total_tiles;
  uint32_t s = 0, s0 = 0;
#pragma unroll
  for (int r = 0; r < kItemPer; ++r) {
    const uint32_t j = blockIdx.x * kItemChunk + r * kItemThreads + threadIdx.x;
    if (j < T) {
      const uint32_t t = tile_at(vt, j);
      const uint32_t k = n_chunks(range[2 * t + 1] - range[2 * t], bd);
      s += k;
      s0 += min(k, w0);
    }
  }
  uint32_t total, total0;
  block_exclusive_scan<kItemThreads>(s, lds, total);
  block_exclusive_scan<kItemThreads>(s0, lds, total0);
  if (threadIdx.x == 0) {
    bsum[blockIdx.x] = total;
    bsum0[blockIdx.x] = total0;
  }
}

// n_work[0]: the first window's work items; n_work[1] (the second window's) is cleared.
__global__ __launch_bounds__(1024) void k_items_scan(uint32_t *__restrict__ bsum, uint32_t *__restrict__ bsum0,
                                                      uint32_t nb, uint32_t *__restrict__ n_items,
                                                      uint32_t *__restrict__ item_base, uint32_t T,
                                                      uint32_t *__restrict__ n_work) {
  __shared__ uint32_t lds[1024 / 64 + 1];
  uint32_t running = 0, running0 = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    const uint32_t v0 = i < nb ? bsum0[i] : 0u;
    uint32_t total, total0;
    const uint32_t ex = block_exclusive_scan<1024>(v, lds, total);
    const uint32_t ex0 = block_exclusive_scan<1024>(v0, lds, total0);
    if (i < nb) {
      bsum[i] = running + ex;
      bsum0[i] = running0 + ex0;
    }
    running += total;
    running0 += total0;
  }
  if (threadIdx.x == 0) {
    *n_items = running;
    item_base[T] = running;
    n_work[0] = running0;
    n_work[1] = 0u;
  }
}

// The item list (every chunk, tile by tile: the item of chunk c of tile t is item_base[t] + c,
// which also indexes its chunk records) and the first window's work list (its chunks below w0,
// in the same order).
__global__ __launch_bounds__(kItemThreads) void k_items_apply(ViewTable vt, const uint32_t *__restrict__ range, int bd,
                                                               uint32_t w0, const uint32_t *__restrict__ bsum,
                                                               const uint32_t *__restrict__ bsum0,
                                                               uint32_t *__restrict__ item_base,
                                                               uint2 *__restrict__ items, uint2 *__restrict__ work,
                                                               uint32_t *__restrict__ need_fix) {
  __shared__ uint32_t lds[kItemThreads / 64 + 1];
  const uint32_t T = vt.total_tiles;
  uint32_t running = bsum[blockIdx.x], running0 = bsum0[blockIdx.x];
  for (int r = 0; r < kItemPer; ++r) {
    const uint32_t j = blockIdx.x * kItemChunk + r * kItemThreads + threadIdx.x;
    const uint32_t t = j < T ? tile_at(vt, j) : 0u;
    const uint32_t k = j < T ? n_chunks(range[2 * t + 1] - range[2 * t], bd) : 0u;
    const uint32_t k0 = min(k, w0);
    uint32_t total, total0;
    const uint32_t ex = block_exclusive_scan<kItemThreads>(k, lds, total);
    const uint32_t ex0 = block_exclusive_scan<kItemThreads>(k0, lds, total0);
    if (j < T) {
      const uint32_t b = running + ex, b0 = running0 + ex0;
      item_base[t] = b;
      for (uint32_t c = 0; c < k; ++c) {
        items[b + c] = make_uint2(t, c);
        need_fix[b + c] = 0u;  // set again by k_blend_scan where a pixel stops inside
      }
      for (uint32_t c = 0; c < k0; ++c) work[b0 + c] = make_uint2(t, c);
    }
    running += total;
    running0 += total0;
  }
}

// ---- per-lane pixels -------------------------------------------------------------------------
// A workgroup of NT lanes covers a TW x TH tile; lane t owns the PPT = TW*TH/NT pixels
// t, t + NT, t + 2 NT, ... (row-major in the tile), so one wavefront instruction touches a
// 64-pixel block and a splat's per-pixel terms are summed inside the lane first.
template <int TW, int TH, int NT>
struct TileCtx {
  static constexpr int PPT = TW * TH / NT;
  static_assert(NT % TW == 0, "a lane's pixels share a column (pixel k of a lane is k NT further)");
  int vi, tx, ty;
  int64_t npx;
  const ViewCam *cam;

  __device__ __forceinline__ TileCtx(const ViewTable &vt, uint32_t gt) {
    vi = view_of_tile(vt, gt);
    cam = &vt.v[vi];
    const uint32_t lt = gt - cam->tile_base;
    tx = (int)(lt % (uint32_t)cam->tiles_x);
    ty = (int)(lt / (uint32_t)cam->tiles_x);
    npx = (int64_t)cam->w * cam->h;
  }
  __device__ __forceinline__ int pidx(int k) const { return (int)threadIdx.x + k * NT; }
  __device__ __forceinline__ void pixel(int k, bool &inside, float &px, float &py, int64_t &pi) const {
    const int q = pidx(k);
    const int wx = tx * TW + q % TW, wy = ty * TH + q / TW;
    inside = wx < cam->w && wy < cam->h;
    px = (float)(cam->x0 + wx);
    py = (float)(cam->y0 + wy);
    pi = (int64_t)wy * cam->w + wx;
  }
};

// Splats per compositing group (the unit of the early exit and of the last-index bookkeeping).
constexpr int kGroupLen = 8;

// KEEP_ID (the backward kernels): the fourth component of the staged colour holds the record
// index (as bits) in place of the SH clamp bits, which compositing does not read.
template <int BD, int NT, bool KEEP_ID = false>
__device__ __forceinline__ void stage(const uint32_t *__restrict__ vals, uint32_t start, int cnt,
                                      const Card *__restrict__ card, float4 *s_a, float4 *s_b, float4 *s_c) {
  for (int k = threadIdx.x; k < cnt; k += NT) {
    const uint32_t e = vals[start + k];
    const Card &cd = card[e];
    stage_card(cd.a, cd.b, cd.c, s_a[k], s_b[k], s_c[k]);
    if (KEEP_ID) s_c[k].w = __uint_as_float(e);
  }
  // up to the next multiple of kGroupLen: records of opacity 0 (alpha 0, never blended), so
  // the compositing loop runs whole groups
  const int padded = min(BD, (cnt + kGroupLen - 1) / kGroupLen * kGroupLen);
  for (int k = cnt + (int)threadIdx.x; k < padded; k += NT) stage_empty(s_a[k], s_b[k], s_c[k]);
}

__device__ __forceinline__ void write_pixel(const ViewImg &im, const ViewCam &cam, int64_t pi, int64_t npx, float C0,
                                            float C1, float C2, float D, float O, float T, int32_t last, int32_t nc) {
  im.color[pi] = C0 + T * cam.bg[0];
  im.color[npx + pi] = C1 + T * cam.bg[1];
  im.color[2 * npx + pi] = C2 + T * cam.bg[2];
  im.depth[pi] = D;
  im.alpha[pi] = O;
  im.t_final[pi] = T;
  im.last[pi] = last;
  if (im.n_contrib) im.n_contrib[pi] = nc;
}

// Compositing state of one pixel.
// The last blended position is lastg + lastr: lastg is the start of the group that holds it,
// lastr its offset inside the group (a constant per unrolled step).
struct PixState {
  float T, C0, C1, C2, D, O;
  int32_t lastg, lastr, nc;
  bool stopped;
  __device__ __forceinline__ int32_t last() const { return lastg + lastr; }
};

// One staged splat over the lane's PPT pixels, continuing each pixel's state; u is the
// splat's offset inside its group. A splat with alpha < 1/255 is skipped; a pixel stops
// before a splat that would take its T below 1e-4. Selects instead of branches: a skipped
// splat adds an exact zero, so the sums equal those of a branching walk bit for bit.
// CNT: also count the contributors (only when that output is wanted).
template <int PPT, bool CNT>
__device__ __forceinline__ void composite_splat(const float4 &A, const float4 &B, const float4 &Cc, int u,
                                                const float (&px)[PPT], const float (&py)[PPT],
                                                PixState (&st)[PPT], bool (&took)[PPT]) {
  const SplatCol col = splat_col(A, B, px[0] - A.x);  // the lane's pixels share a column
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    PixState &p = st[k];
    const float alpha = fminf(kAlphaMax, splat_e2(splat_p2(B, col, py[k] - A.y)));
    const float wt = alpha * p.T;  // the weight, and T's decrement: T (1 - alpha) = T - alpha T
    const float Tn = p.T - wt;
    // take = !stopped && alpha_ok && !low, written through the updated stop flag so that the
    // one compare of Tn serves both (its negation falls on a lane mask)
    const bool alpha_ok = alpha >= kAlphaMin;
    p.stopped = p.stopped || (alpha_ok && Tn < kTMin);
    const bool take = alpha_ok && !p.stopped;
    const float w = take ? wt : 0.f;
    p.C0 += w * Cc.x;
    p.C1 += w * Cc.y;
    p.C2 += w * Cc.z;
    p.D += w * B.z;
    p.O += w;
    p.T = take ? Tn : p.T;
    p.lastr = take ? u : p.lastr;
    took[k] = took[k] || take;
    if constexpr (CNT) p.nc += take ? 1 : 0;
  }
}

template <int PPT>
__device__ __forceinline__ bool all_stopped(const PixState (&st)[PPT]) {
  bool all = true;
#pragma unroll
  for (int k = 0; k < PPT; ++k) all = all && st[k].stopped;
  return __all(all);
}

// Front-to-back over cnt staged splats (padded to whole groups of kGroupLen by the staging)
// for the lane's PPT pixels; positions are pos0 + index. Returns false once every pixel of
// the wavefront has stopped (the walk then ends early).
template <int PPT, bool CNT, int G = kGroupLen>
__device__ __forceinline__ bool composite_run(const float4 *s_a, const float4 *s_b, const float4 *s_c, int cnt,
                                              const float (&px)[PPT], const float (&py)[PPT], int pos0,
                                              PixState (&st)[PPT]) {
  static_assert(kGroupLen % G == 0, "groups must tile the padding");
  for (int j0 = 0; j0 < cnt; j0 += G) {
    if (all_stopped(st)) return false;
    bool took[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) took[k] = false;
#pragma unroll
    for (int u = 0; u < G; ++u) composite_splat<PPT, CNT>(s_a[j0 + u], s_b[j0 + u], s_c[j0 + u], u, px, py, st, took);
#pragma unroll
    for (int k = 0; k < PPT; ++k) st[k].lastg = took[k] ? pos0 + j0 : st[k].lastg;
  }
  return true;
}

// ---- forward pass 1: every chunk of a window's work list from transmittance 1 -------------
// work / n_work: this window's work items (tile, chunk); n_next, l_next: the next window's
// work and tile counts, cleared here for k_blend_scan to append to. A chunk's records sit at
// item item_base[t] + c. PERSIST: a fixed grid walks the list (the later windows, whose lists
// are short: a grid for the longest list would mostly launch empty workgroups); otherwise one
// item per workgroup in the XCD-grouped order.
template <int TW, int TH, int BD, int NT, bool CNT, bool PERSIST>
__global__ __launch_bounds__(NT) void k_blend_chunk(ViewTable vt, ImgTable it, const Card *__restrict__ card,
                                                    const uint32_t *__restrict__ vals,
                                                    const uint32_t *__restrict__ range,
                                                    const uint2 *__restrict__ work,
                                                    const uint32_t *__restrict__ n_work,
                                                    uint32_t *__restrict__ n_next, uint32_t *__restrict__ l_next,
                                                    const uint32_t *__restrict__ item_base,
                                                    ChunkRec *__restrict__ chunk) {
  using Ctx = TileCtx<TW, TH, NT>;
  constexpr int PPT = Ctx::PPT;
  __shared__ float4 s_a[BD], s_b[BD], s_c[BD];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *n_next = 0u;
    *l_next = 0u;
  }
  uint32_t w;
  if (PERSIST) {
    w = blockIdx.x;
    if (w >= *n_work) return;
  } else if (!item_of_block(n_work, w)) {
    return;
  }
  const uint32_t nw = PERSIST ? *n_work : 0u;
#pragma unroll 1
  for (;;) {
    const uint2 tc = work[w];
    const uint32_t gt = tc.x, c = tc.y;
    const uint32_t item = item_base[gt] + c;
    const Ctx tile(vt, gt);
    const uint32_t s0 = range[2 * gt], e0 = range[2 * gt + 1];
    const uint32_t K = n_chunks(e0 - s0, BD);
    const uint32_t cs = s0 + c * BD;
    const int cnt = (int)min<uint32_t>(BD, e0 - cs);
    stage<BD, NT>(vals, cs, cnt, card, s_a, s_b, s_c);
    __syncthreads();

    float px[PPT], py[PPT];
    bool inside[PPT];
    int64_t pi[PPT];
    PixState st[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      tile.pixel(k, inside[k], px[k], py[k], pi[k]);
      st[k] = PixState{1.f, 0.f, 0.f, 0.f, 0.f, 0.f, -1, 0, 0, !inside[k]};
    }
    composite_run<PPT, CNT>(s_a, s_b, s_c, cnt, px, py, 0, st);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (!inside[k]) continue;
      const PixState &p = st[k];
      if (K == 1) {
        write_pixel(it.v[tile.vi], *tile.cam, pi[k], tile.npx, p.C0, p.C1, p.C2, p.D, p.O, p.T, p.last(), p.nc);
      } else {
        ChunkRec r;
        r.c0 = p.C0; r.c1 = p.C1; r.c2 = p.C2; r.d = p.D; r.o = p.O; r.t = p.T;
        r.info = (uint32_t)(p.last() + 1) | ((uint32_t)p.nc << 10) | ((uint32_t)p.stopped << 20);
        r.pad = 0.f;
        chunk[(int64_t)item * (TW * TH) + tile.pidx(k)] = r;
      }
    }
    if (!PERSIST) return;
    w += gridDim.x;
    if (w >= nw) return;
    __syncthreads();  // the staged splats are read by every wavefront before the next item
  }
}

// ---- forward pass 2: per multi-chunk tile, chunk partials in order ------------------------
// Per pixel, over the chunks in order until the pixel stops: a chunk whose product keeps T at
// or above 1e-4 is accumulated whole (its record then holds the chunk's absolute colour /
// depth and the transmittance after it); at the chunk where the pixel stops the record gets
// the incoming state (colour, depth, opacity, T, last + 1, count) flagged kPending, and the
// item is marked for k_blend_fix. Chunks behind that point are not touched: later passes stop
// at the pixel's last contributor. Chunk records are loaded kScanBatch at a time, so a long
// tile's chain costs one memory latency per batch instead of one per chunk.
//
// The chunks are composited and scanned in windows of increasing length ([0, q_hi), then
// [q_hi, q_next), ...), so that a tile all of whose pixels have stopped in one window has none
// of its later chunks composited (in a street view most long tile lists lie mostly behind
// the point where every pixel of the tile is opaque). This pass scans the window
// [q_lo, q_hi) and, when some pixel is still running, appends the tile's next window
// [q_hi, q_next) to the next work list and the tile to the next tile list. The first window
// takes one workgroup per tile; the later ones walk the tile list with a fixed grid. Between
// windows a running pixel keeps its state in its own output planes: colour without the
// background, depth, opacity, last, count, and the transmittance negated in t_final (a pixel
// whose t_final is not negative is finished or waits for k_blend_fix).
constexpr uint32_t kPending = 1u << 31;
constexpr int kScanBatch = 8;

template <int TW, int TH, int BD>
__device__ __forceinline__ void scan_tile(const ViewTable &vt, const ImgTable &it, const uint32_t *__restrict__ range,
                                          const uint32_t *__restrict__ item_base, ChunkRec *__restrict__ chunk,
                                          uint32_t *__restrict__ need_fix, uint32_t q_lo, uint32_t q_hi,
                                          uint32_t q_next, uint2 *__restrict__ work, uint32_t *__restrict__ n_next,
                                          uint32_t *__restrict__ live_next, uint32_t *__restrict__ l_next,
                                          uint32_t &s_base, uint32_t gt) {
  // one pixel per lane: the per-pixel chain over the chunks is serial, so spread it wide
  using Ctx = TileCtx<TW, TH, TW * TH>;
  constexpr int PPT = Ctx::PPT;
  constexpr int64_t TT = TW * TH;
  const uint32_t s0 = range[2 * gt], e0 = range[2 * gt + 1];
  const uint32_t K = n_chunks(e0 - s0, BD);
  if (K == 1) return;                // written by the chunk pass
  if (q_lo > 0 && K <= q_lo) return;  // finished in an earlier window
  const Ctx tile(vt, gt);
  const ViewImg &im = it.v[tile.vi];
  const uint32_t q_end = min(K, q_hi);
  bool running_any = false;
#pragma unroll 1
  for (int k = 0; k < PPT; ++k) {
    bool inside;
    float pxf, pyf;
    int64_t pi;
    tile.pixel(k, inside, pxf, pyf, pi);
    if (!inside) continue;
    if (K == 0) {
      write_pixel(im, *tile.cam, pi, tile.npx, 0.f, 0.f, 0.f, 0.f, 0.f, 1.f, -1, 0);
      continue;
    }
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, O = 0.f;
    int32_t last = -1, nc = 0;
    if (q_lo > 0) {
      const float tf = im.t_final[pi];
      if (!(tf < 0.f)) continue;  // finished in an earlier window, or waiting for the fix
      T = -tf;
      C0 = im.color[pi];
      C1 = im.color[tile.npx + pi];
      C2 = im.color[2 * tile.npx + pi];
      D = im.depth[pi];
      O = im.alpha[pi];
      last = im.last[pi];
      if (im.n_contrib) nc = im.n_contrib[pi];
    }
    const uint32_t ib = item_base[gt];
    ChunkRec *base = chunk + (int64_t)ib * TT + tile.pidx(k);
    bool done = false, pending = false;
    for (uint32_t q0 = q_lo; q0 < q_end && !done; q0 += kScanBatch) {
      ChunkRec rb[kScanBatch];
#pragma unroll
      for (int i = 0; i < kScanBatch; ++i)
        if (q0 + i < q_end) rb[i] = base[(int64_t)(q0 + i) * TT];
#pragma unroll
      for (int i = 0; i < kScanBatch; ++i) {
        const uint32_t q = q0 + i;
        if (done || q >= q_end) continue;
        const ChunkRec &r = rb[i];
        const int ll = (int)(r.info & 1023u) - 1;
        const int ncl = (int)((r.info >> 10) & 1023u);
        const bool cut = (r.info >> 20) & 1u;
        const float Tafter = T * r.t;
        ChunkRec w;
        w.o = 0.f;
        w.pad = 0.f;
        if (!cut ? (Tafter >= kTMin) : (T == 1.f)) {
          // the whole chunk blends (from T = 1 the chunk pass is exact even when it stops inside)
          w.c0 = T * r.c0; w.c1 = T * r.c1; w.c2 = T * r.c2; w.d = T * r.d;
          C0 += w.c0; C1 += w.c1; C2 += w.c2; D += w.d;
          O += T * r.o;
          if (ll >= 0) last = (int32_t)(q * BD) + ll;
          nc += ncl;
          T = Tafter;
          w.t = T;
          w.info = 0u;
          done = cut;
        } else {
          // the pixel stops inside this chunk: hand the incoming state to k_blend_fix
          w.c0 = C0; w.c1 = C1; w.c2 = C2; w.d = D; w.o = O; w.t = T;
          w.info = kPending | (uint32_t)(last + 1);
          w.pad = __int_as_float(nc);
          pending = done = true;
          need_fix[ib + q] = 1u;  // every writer stores the same value
        }
        base[(int64_t)q * TT] = w;
      }
    }
    if (pending) {
      if (q_hi < K) im.t_final[pi] = 1.f;  // not running (the fix writes the pixel)
    } else if (!done && q_hi < K) {
      // still running: keep the state for the next window
      im.color[pi] = C0;
      im.color[tile.npx + pi] = C1;
      im.color[2 * tile.npx + pi] = C2;
      im.depth[pi] = D;
      im.alpha[pi] = O;
      im.t_final[pi] = -T;
      im.last[pi] = last;
      if (im.n_contrib) im.n_contrib[pi] = nc;
      running_any = true;
    } else {
      write_pixel(im, *tile.cam, pi, tile.npx, C0, C1, C2, D, O, T, last, nc);
    }
  }
  if (__syncthreads_or(running_any) == 0) return;
  // some pixel is still running: the tile's next window goes to the next work list
  const uint32_t n = min(K, q_next) - q_hi;
  if (threadIdx.x == 0) {
    s_base = atomicAdd(n_next, n);
    live_next[atomicAdd(l_next, 1u)] = gt;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += TW * TH) work[s_base + i] = make_uint2(gt, q_hi + i);
}

// live == nullptr: the first window, one workgroup per tile; else the tiles of live[0, *n_live).
template <int TW, int TH, int BD>
__global__ __launch_bounds__(TW * TH) void k_blend_scan(ViewTable vt, ImgTable it, const uint32_t *__restrict__ range,
                                                   const uint32_t *__restrict__ item_base,
                                                   ChunkRec *__restrict__ chunk, uint32_t *__restrict__ need_fix,
                                                   uint32_t q_lo, uint32_t q_hi, uint32_t q_next,
                                                   uint2 *__restrict__ work, uint32_t *__restrict__ n_next,
                                                   const uint32_t *__restrict__ live,
                                                   const uint32_t *__restrict__ n_live,
                                                   uint32_t *__restrict__ live_next, uint32_t *__restrict__ l_next) {
  __shared__ uint32_t s_base;
  if (!live) {
    scan_tile<TW, TH, BD>(vt, it, range, item_base, chunk, need_fix, q_lo, q_hi, q_next, work, n_next, live_next,
                          l_next, s_base, blockIdx.x);
    return;
  }
  const uint32_t nl = *n_live;
  for (uint32_t i = blockIdx.x; i < nl; i += gridDim.x)
    scan_tile<TW, TH, BD>(vt, it, range, item_base, chunk, need_fix, q_lo, q_hi, q_next, work, n_next, live_next,
                          l_next, s_base, live[i]);
}

template <int TW, int TH, int BD, int NT, bool CNT>
__device__ __forceinline__ void fix_item(const ViewTable &vt, const ImgTable &it, const Card *__restrict__ card,
                                         const uint32_t *__restrict__ vals, const uint32_t *__restrict__ range,
                                         const uint2 *__restrict__ items, uint32_t item, ChunkRec *__restrict__ chunk,
                                         float4 *s_a, float4 *s_b, float4 *s_c) {
  using Ctx = TileCtx<TW, TH, NT>;
  constexpr int PPT = Ctx::PPT;
  const uint2 tc = items[item];
  const uint32_t gt = tc.x, c = tc.y;
  const uint32_t s0 = range[2 * gt], e0 = range[2 * gt + 1];
  const Ctx tile(vt, gt);
  float px[PPT], py[PPT];
  bool inside[PPT], pending[PPT];
  int64_t pi[PPT];
  ChunkRec r[PPT];
  PixState st[PPT];
  bool any = false;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    tile.pixel(k, inside[k], px[k], py[k], pi[k]);
    r[k] = ChunkRec{};
    if (inside[k]) r[k] = chunk[(int64_t)item * (TW * TH) + tile.pidx(k)];
    pending[k] = inside[k] && (r[k].info & kPending);
    any = any || pending[k];
    // composite the chunk's splats only (partial sums start at zero; O and the count carry on)
    st[k] = PixState{r[k].t, 0.f, 0.f, 0.f, 0.f, r[k].o, (int32_t)(r[k].info & 0x3FFFFFFFu) - 1, 0,
                     __float_as_int(r[k].pad), !pending[k]};
  }
  if (__syncthreads_count(any) == 0) return;  // uniform
  const uint32_t cs = s0 + c * BD;
  const int cnt = (int)min<uint32_t>(BD, e0 - cs);
  stage<BD, NT>(vals, cs, cnt, card, s_a, s_b, s_c);
  __syncthreads();
  composite_run<PPT, CNT>(s_a, s_b, s_c, cnt, px, py, (int)(c * BD), st);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    if (!pending[k]) continue;
    const PixState &p = st[k];
    write_pixel(it.v[tile.vi], *tile.cam, pi[k], tile.npx, r[k].c0 + p.C0, r[k].c1 + p.C1, r[k].c2 + p.C2,
                r[k].d + p.D, p.O, p.T, p.last(), p.nc);
    ChunkRec w;
    w.c0 = p.C0; w.c1 = p.C1; w.c2 = p.C2; w.d = p.D; w.o = 0.f; w.t = p.T; w.info = 0u; w.pad = 0.f;
    chunk[(int64_t)item * (TW * TH) + tile.pidx(k)] = w;
  }
}

// ---- forward pass 3: exact compositing of each pixel's stop chunk (chunk-parallel) -------
template <int TW, int TH, int BD, int NT, bool CNT>
__global__ __launch_bounds__(NT) void k_blend_fix(ViewTable vt, ImgTable it, const Card *__restrict__ card,
                                                  const uint32_t *__restrict__ vals,
                                                  const uint32_t *__restrict__ range,
                                                  const uint2 *__restrict__ items,
                                                  const uint32_t *__restrict__ n_items,
                                                  const uint32_t *__restrict__ need_fix,
                                                  ChunkRec *__restrict__ chunk) {
  __shared__ float4 s_a[BD], s_b[BD], s_c[BD];
  uint32_t item;
  if (!item_of_block(n_items, item)) return;
  if (!need_fix[item]) return;  // no pixel stops inside this chunk
  fix_item<TW, TH, BD, NT, CNT>(vt, it, card, vals, range, items, item, chunk, s_a, s_b, s_c);
}

// ---- forward passes 1 and 3 for 8x8 tiles: two work items per wavefront ----------------
// With one pixel per lane the broadcast LDS reads of the staged splats (40 B per splat and
// lane) bound the compositing loop. Here lanes 0-31 take item 2p and lanes 32-63 item 2p + 1,
// two pixels each (rows 0-3 and 4-7 of the 8x8 tile): one LDS instruction delivers a splat of
// each item and every lane uses it for two pixels, which halves the LDS bytes per
// evaluation. Each chunk is staged in sub-chunks of kSub splats (the LDS footprint of a
// one-item workgroup); the half with fewer splats runs over opacity-0 padding. The second
// half's arrays start 16 B further into the banks, so the two addresses of a read differ in
// bank.
constexpr int kSub = 64;
constexpr int kPairGroup = 8;  // splats per unrolled group in the two-item loop
constexpr int kHalfStride = kSub + 1;  // float4 entries per half in the staging arrays

// Pair of items of this workgroup after the XCD remap; false when neither exists.
__device__ __forceinline__ bool pair_of_block(const uint32_t *n_items, uint32_t &pair) {
  const uint32_t x = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
  pair = ((k / kGroup) * kXcds + x) * kGroup + k % kGroup;
  return 2 * pair < *n_items;
}

// One half-wavefront's item: its tile, chunk and the lane's two pixels.
template <int BD>
struct HalfItem {
  bool valid;
  uint32_t item, gt, c, K, cs;
  int cnt, vi;
  const ViewCam *cam;
  int64_t npx;
  bool inside[2];
  float px[2], py[2];
  int64_t pi[2];
  int q[2];  // row-major pixel index in the tile

  __device__ __forceinline__ HalfItem(const ViewTable &vt, const uint2 *work, const uint32_t *item_base,
                                      const uint32_t *range, uint32_t nI, uint32_t it, int hl) {
    valid = it < nI;
    const uint2 tc = valid ? work[it] : make_uint2(0u, 0u);
    gt = tc.x;
    c = tc.y;
    item = valid ? item_base[gt] + c : 0u;
    const uint32_t s0 = valid ? range[2 * gt] : 0u, e0 = valid ? range[2 * gt + 1] : 0u;
    K = n_chunks(e0 - s0, BD);
    cs = s0 + c * BD;
    cnt = valid ? (int)min<uint32_t>(BD, e0 - cs) : 0;
    vi = view_of_tile(vt, gt);
    cam = &vt.v[vi];
    npx = (int64_t)cam->w * cam->h;
    const uint32_t lt = gt - cam->tile_base;
    const int tx = (int)(lt % (uint32_t)cam->tiles_x), ty = (int)(lt / (uint32_t)cam->tiles_x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      q[k] = hl + 32 * k;
      const int wx = tx * 8 + (q[k] & 7), wy = ty * 8 + (q[k] >> 3);
      inside[k] = valid && wx < cam->w && wy < cam->h;
      px[k] = (float)(cam->x0 + wx);
      py[k] = (float)(cam->y0 + wy);
      pi[k] = (int64_t)wy * cam->w + wx;
    }
  }
};

// Stage splats [base, base + kSub) of the half's chunk (zero records past cnt) into its half
// of the arrays; 32 lanes, two splats each.
__device__ __forceinline__ void stage_half(const uint32_t *__restrict__ vals, const Card *__restrict__ card,
                                           uint32_t cs, int cnt, int base, int hl, float4 *a, float4 *b, float4 *cc) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int kk = hl + 32 * r;
    float4 sa, sb, sc;
    stage_empty(sa, sb, sc);
    if (base + kk < cnt) {
      const Card &cd = card[vals[cs + base + kk]];
      stage_card(cd.a, cd.b, cd.c, sa, sb, sc);
    }
    a[kk] = sa;
    b[kk] = sb;
    cc[kk] = sc;
  }
}

// Both halves over their chunks, sub-chunk by sub-chunk; positions are relative to the chunk
// start. Leaves early once every pixel of the wavefront has stopped.
template <int BD, bool CNT>
__device__ __forceinline__ void composite_pair(const uint32_t *__restrict__ vals, const Card *__restrict__ card,
                                               const HalfItem<BD> &hi, int hl, float4 *s_a, float4 *s_b, float4 *s_c,
                                               PixState (&st)[2]) {
  const int h = (int)threadIdx.x >> 5;
  float4 *a = s_a + h * kHalfStride, *b = s_b + h * kHalfStride, *cc = s_c + h * kHalfStride;
  const int n_max = max(__builtin_amdgcn_readlane(hi.cnt, 0), __builtin_amdgcn_readlane(hi.cnt, 32));
#pragma unroll 1
  for (int base = 0; base < n_max; base += kSub) {
    if (all_stopped(st)) return;
    __syncthreads();  // the previous sub-chunk's reads are done
    stage_half(vals, card, hi.cs, hi.cnt, base, hl, a, b, cc);
    __syncthreads();
    const int len = min(kSub, n_max - base);
    if (!composite_run<2, CNT, kPairGroup>(a, b, cc, len, hi.px, hi.py, base, st)) return;
  }
}

template <int BD, bool CNT>
__device__ __forceinline__ void pair_item(const ViewTable &vt, const ImgTable &it, const Card *__restrict__ card,
                                          const uint32_t *__restrict__ vals, const uint2 *__restrict__ work,
                                          uint32_t nw, const uint32_t *__restrict__ item_base,
                                          const uint32_t *__restrict__ range, uint32_t pair,
                                          ChunkRec *__restrict__ chunk, float4 *s_a, float4 *s_b, float4 *s_c) {
  const int hl = (int)threadIdx.x & 31;
  const HalfItem<BD> hi(vt, work, item_base, range, nw, 2 * pair + (threadIdx.x >> 5), hl);
  PixState st[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) st[k] = PixState{1.f, 0.f, 0.f, 0.f, 0.f, 0.f, -1, 0, 0, !hi.inside[k]};
  composite_pair<BD, CNT>(vals, card, hi, hl, s_a, s_b, s_c, st);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!hi.inside[k]) continue;
    const PixState &p = st[k];
    if (hi.K == 1) {
      write_pixel(it.v[hi.vi], *hi.cam, hi.pi[k], hi.npx, p.C0, p.C1, p.C2, p.D, p.O, p.T, p.last(), p.nc);
    } else {
      ChunkRec r;
      r.c0 = p.C0; r.c1 = p.C1; r.c2 = p.C2; r.d = p.D; r.o = p.O; r.t = p.T;
      r.info = (uint32_t)(p.last() + 1) | ((uint32_t)p.nc << 10) | ((uint32_t)p.stopped << 20);
      r.pad = 0.f;
      chunk[(int64_t)hi.item * 64 + hi.q[k]] = r;
    }
  }
}

template <int BD, bool CNT>
__global__ __launch_bounds__(64) void k_blend_chunk_pair(ViewTable vt, ImgTable it, const Card *__restrict__ card,
                                                         const uint32_t *__restrict__ vals,
                                                         const uint32_t *__restrict__ range,
                                                         const uint2 *__restrict__ work,
                                                         const uint32_t *__restrict__ n_work,
                                                         uint32_t *__restrict__ n_next,
                                                         uint32_t *__restrict__ l_next,
                                                         const uint32_t *__restrict__ item_base,
                                                         ChunkRec *__restrict__ chunk) {
  __shared__ float4 s_a[2 * kHalfStride], s_b[2 * kHalfStride], s_c[2 * kHalfStride];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *n_next = 0u;
    *l_next = 0u;
  }
  uint32_t pair;
  if (!pair_of_block(n_work, pair)) return;
  pair_item<BD, CNT>(vt, it, card, vals, work, *n_work, item_base, range, pair, chunk, s_a, s_b, s_c);
}

// ---- forward pass 4: backward starting state per chunk (suffix sums, per tile) ------------
// Colour / depth composited behind each chunk, normalised by the transmittance after it, for
// the chunks up to the one holding the pixel's last contributor (the backward reads no
// other). Records are loaded kScanBatch at a time.
template <int TW, int TH, int BD>
__global__ __launch_bounds__(TW * TH) void k_blend_suffix(ViewTable vt, ImgTable it, const uint32_t *__restrict__ range,
                                                     const uint32_t *__restrict__ item_base,
                                                     ChunkRec *__restrict__ chunk) {
  using Ctx = TileCtx<TW, TH, TW * TH>;
  constexpr int PPT = Ctx::PPT;
  constexpr int64_t TT = TW * TH;
  const uint32_t gt = blockIdx.x;
  const uint32_t K = n_chunks(range[2 * gt + 1] - range[2 * gt], BD);
  if (K < 2) return;
  const Ctx tile(vt, gt);
  const ViewImg &im = it.v[tile.vi];
#pragma unroll 1
  for (int k = 0; k < PPT; ++k) {
    bool inside;
    float pxf, pyf;
    int64_t pi;
    tile.pixel(k, inside, pxf, pyf, pi);
    if (!inside) continue;
    const int last = im.last[pi];
    if (last < 0) continue;
    ChunkRec *base = chunk + (int64_t)item_base[gt] * TT + tile.pidx(k);
    float b0 = 0.f, b1 = 0.f, b2 = 0.f, bd = 0.f;
    for (int q0 = last / BD; q0 >= 0; q0 -= kScanBatch) {
      ChunkRec rb[kScanBatch];
#pragma unroll
      for (int i = 0; i < kScanBatch; ++i)
        if (q0 - i >= 0) rb[i] = base[(int64_t)(q0 - i) * TT];
#pragma unroll
      for (int i = 0; i < kScanBatch; ++i) {
        const int q = q0 - i;
        if (q < 0) continue;
        const ChunkRec &r = rb[i];
        const float inv = 1.f / r.t;
        ChunkRec w;
        w.c0 = b0 * inv; w.c1 = b1 * inv; w.c2 = b2 * inv; w.d = bd * inv; w.o = 0.f; w.t = r.t; w.info = 0u;
        w.pad = 0.f;
        base[(int64_t)q * TT] = w;
        b0 += r.c0; b1 += r.c1; b2 += r.c2; bd += r.d;
      }
    }
  }
}

// ---- backward: every chunk back to front ---------------------------------------------------
// Row-local DPP read of a neighbour lane (every pattern used reads inside its own row, so no
// lane sees the bound value); in this form the compiler folds it into the consuming add.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over the wavefront of ten values, transposed so that no lane selects are needed where
// the lane split falls on a DPP bank (4-lane group) boundary:
//   1. row_mirror pairs lane i with 15 - i (bit 3 differs). Two DPP adds per output, each
//      writing half of the banks: lanes with bit 3 clear keep slots 0-4, the others 5-9.
//   2. row_half_mirror pairs i with 7 - i (bit 2 differs): bit 2 clear keeps the first three
//      of its five slots, set keeps the last two (its third output is left unwritten there:
//      the later steps never move it into a lane that holds a result).
//   3. permlane16 swaps add row pairs (0+1, 2+3) of two outputs in one register, and of the
//      third in another; a permlane32 swap adds the halves: row 0 then holds output 0, row 1
//      output 1, row 2 output 2, each summed over the four rows (row 3: nothing of use).
//   4. two quad DPP adds sum the four lanes of a quad (bits 0 and 1).
// Afterwards lane l holds the total of value reduce10_slot(l) (-1: nothing to store).
// The DPP sources are written by ordinary VALU code just before each block, hence the two
// wait states (s_nop 1) that a DPP read of a freshly written register needs.
__device__ __forceinline__ float wave_reduce10(const float (&g)[10]) {
  float a0, a1, a2, a3, a4;
  asm volatile(
      "s_nop 1\n"
      "v_add_f32_dpp %0, %5, %5 row_mirror row_mask:0xf bank_mask:0x3\n"
      "v_add_f32_dpp %0, %10, %10 row_mirror row_mask:0xf bank_mask:0xc\n"
      "v_add_f32_dpp %1, %6, %6 row_mirror row_mask:0xf bank_mask:0x3\n"
      "v_add_f32_dpp %1, %11, %11 row_mirror row_mask:0xf bank_mask:0xc\n"
      "v_add_f32_dpp %2, %7, %7 row_mirror row_mask:0xf bank_mask:0x3\n"
      "v_add_f32_dpp %2, %12, %12 row_mirror row_mask:0xf bank_mask:0xc\n"
      "v_add_f32_dpp %3, %8, %8 row_mirror row_mask:0xf bank_mask:0x3\n"
      "v_add_f32_dpp %3, %13, %13 row_mirror row_mask:0xf bank_mask:0xc\n"
      "v_add_f32_dpp %4, %9, %9 row_mirror row_mask:0xf bank_mask:0x3\n"
      "v_add_f32_dpp %4, %14, %14 row_mirror row_mask:0xf bank_mask:0xc"
      : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4)
      : "v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(g[6]), "v"(g[7]), "v"(g[8]),
        "v"(g[9]));
  float b0, b1, b2;
  asm volatile(
      "s_nop 1\n"
      "v_add_f32_dpp %0, %3, %3 row_half_mirror row_mask:0xf bank_mask:0x5\n"
      "v_add_f32_dpp %0, %6, %6 row_half_mirror row_mask:0xf bank_mask:0xa\n"
      "v_add_f32_dpp %1, %4, %4 row_half_mirror row_mask:0xf bank_mask:0x5\n"
      "v_add_f32_dpp %1, %7, %7 row_half_mirror row_mask:0xf bank_mask:0xa\n"
      "v_add_f32_dpp %2, %5, %5 row_half_mirror row_mask:0xf bank_mask:0x5"
      : "=&v"(b0), "=&v"(b1), "=&v"(b2)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3), "v"(a4));
  const auto p01 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b0), __float_as_uint(b1), false, false);
  const float r01 = __uint_as_float(p01[0]) + __uint_as_float(p01[1]);
  // b2's second operand is a spent register: rows 1 and 3 of the sum then hold its rows, which
  // only reach row 3 of the result, where no value is read
  const auto p22 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b2), __float_as_uint(a0), false, false);
  const float r22 = __uint_as_float(p22[0]) + __uint_as_float(p22[1]);
  const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(r01), __float_as_uint(r22), false, false);
  float v = __uint_as_float(q[0]) + __uint_as_float(q[1]);
  v += dpp<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

// Which of the ten values lane l holds after wave_reduce10, or -1 (one lane per quad; bits 3-2
// pick the slot group {0-2, 3-4, 5-7, 8-9}, the row the member of the group).
__device__ __forceinline__ int reduce10_slot(int lane) {
  const int grp = (lane >> 2) & 3, row = lane >> 4;
  const int base = grp == 0 ? 0 : (grp == 1 ? 3 : (grp == 2 ? 5 : 8));
  const bool ok = (lane & 3) == 0 && (row < 2 || (row == 2 && (grp & 1) == 0));
  return ok ? base + row : -1;
}

// Backward state of one pixel. The colour behind the current splat enters the alpha
// derivative only through dL/dC . (c - C_behind), so the pixel carries the scalar
// S = dL/dC . C_behind (updated as S + alpha (dL/dC . c - S)) instead of the three channels.
constexpr int kBwdSub = 64;  // splats staged at a time by the compositing backward

struct PixGrad {
  float gC0, gC1, gC2, gD, TfG;  // TfG = T_final (dL/dO - dL/dC . bg)
  float T, S, AD;
  int ll;
  float px, py;
};

// Gradient record per splat and view (grad2d, 12 floats), summed over pixels; the geometry
// kernel applies the splat's conic and the constant factors:
//   0: sum dp dx                     -> dL/du = a slot0 + b slot1
//   1: sum dp dy                     -> dL/dv = b slot0 + c slot1
//   2: sum dp dx^2                   -> dL/da = -slot / 2
//   3: sum dp dx dy                  -> dL/db = -slot
//   4: sum dp dy^2                   -> dL/dc = -slot / 2
//   5: sum dp                        -> dL/do = slot / o
//   6-8: dL/d(r, g, b);  9: dL/d(depth)
// with dp = dL/dpower = dL/dalpha * o exp(power) (zero where alpha is clamped at 0.99) and
// (a, b, c) the unscaled conic.
// Splats hi down to lo of the chunk, back to front, for the pixels of this lane; splat j is
// staged at s_a/s_b/s_c[j - lo] (record index in s_c[.].w). DEPTH: some pixel of the
// wavefront has a depth gradient.
template <int PPT, bool DEPTH>
__device__ __forceinline__ void bwd_splats(int hi, int lo, const float4 *s_a, const float4 *s_b, const float4 *s_c,
                                           PixGrad (&pg)[PPT], int slot, float *__restrict__ g2) {
  // the staged record's byte offset lives in a vector register: the LDS reads take their
  // address from one, and a scalar index would be copied over twice per splat
  int off = (hi - lo) * (int)sizeof(float4);
  for (int j = hi; j >= lo; --j, off -= (int)sizeof(float4)) {
    asm volatile("" : "+v"(off));
    const float4 A = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_a) + off);
    const float4 B = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_b) + off);
    const float4 Cc = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_c) + off);
    // alpha at every pixel first; a splat no pixel of the wavefront blends costs only this
    float dxs[PPT], dys[PPT], ars[PPT];
    bool act[PPT];
    bool any = false;
    const SplatCol col = splat_col(A, B, pg[0].px - A.x);  // the lane's pixels share a column
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      dxs[k] = pg[k].px - A.x;
      dys[k] = pg[k].py - A.y;
      ars[k] = splat_e2(splat_p2(B, col, dys[k]));
      act[k] = j <= pg[k].ll && fminf(kAlphaMax, ars[k]) >= kAlphaMin;
      any = any || act[k];
    }
    if (!__any(any)) continue;
    float g[10];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      PixGrad &p = pg[k];
      // a pixel this splat does not reach takes alpha 0: every update below then leaves its
      // state unchanged exactly (T * 1, S + 0 * r) and adds zeros
      const float alpha = act[k] ? fminf(kAlphaMax, ars[k]) : 0.f;
      const float inv = __builtin_amdgcn_rcpf(1.f - alpha);  // 1 ulp; 1 - alpha >= 0.01; exactly 1 at alpha 0
      p.T = p.T * inv;                                       // transmittance in front of this splat
      const float w = alpha * p.T;
      // dL/dC . (c - C_behind), then C_behind <- alpha c + (1 - alpha) C_behind
      float r = (p.gC0 * Cc.x + p.gC1 * Cc.y + p.gC2 * Cc.z) - p.S;
      p.S = fmaf(alpha, r, p.S);
      float t9 = 0.f;
      if (DEPTH) {
        t9 = p.gD * w;
        const float rd = B.z - p.AD;
        r = fmaf(p.gD, rd, r);
        p.AD = fmaf(alpha, rd, p.AD);
      }
      const float dLda = fmaf(p.T, r, inv * p.TfG);
      const float dm = (act[k] && ars[k] < kAlphaMax) ? dLda : 0.f;  // clamped alpha: no power path
      const float dp = dm * ars[k];
      const float dpx = dp * dxs[k], dpy = dp * dys[k];
      const float t[10] = {dpx,          dpy,          dpx * dxs[k], dpx * dys[k], dpy * dys[k],
                           dp,           p.gC0 * w,    p.gC1 * w,    p.gC2 * w,    t9};
#pragma unroll
      for (int v = 0; v < 10; ++v) g[v] = k == 0 ? t[v] : g[v] + t[v];
    }
    const float tot = wave_reduce10(g);
    if (slot >= 0 && tot != 0.f) unsafeAtomicAdd(&g2[(int64_t)__float_as_uint(Cc.w) * 12 + slot], tot);
  }
}

template <int TW, int TH, int BD, int NT>
__global__ __launch_bounds__(NT) void k_blend_bwd_chunk(ViewTable vt, ImgTable it, GradTable gtab,
                                                        const Card *__restrict__ card,
                                                        const uint32_t *__restrict__ vals,
                                                        const uint32_t *__restrict__ range,
                                                        const uint2 *__restrict__ items,
                                                        const uint32_t *__restrict__ n_items,
                                                        const ChunkRec *__restrict__ chunk,
                                                        float *__restrict__ g2 /*[E][12]*/) {
  using Ctx = TileCtx<TW, TH, NT>;
  constexpr int PPT = Ctx::PPT;
  // the chunk is staged kBwdSub splats at a time, back to front: LDS and registers do not
  // grow with the chunk length
  constexpr int SUB = BD < kBwdSub ? BD : kBwdSub;
  __shared__ float4 s_a[SUB], s_b[SUB], s_c[SUB];
  __shared__ int s_max;
  uint32_t item;
  if (!item_of_block(n_items, item)) return;
  const uint2 tc = items[item];
  const uint32_t gt = tc.x, c = tc.y;
  const Ctx tile(vt, gt);
  const ViewCam &cam = *tile.cam;
  const uint32_t s0 = range[2 * gt], e0 = range[2 * gt + 1];
  const uint32_t K = n_chunks(e0 - s0, BD);
  const uint32_t cs = s0 + c * BD;
  const int cnt = (int)min<uint32_t>(BD, e0 - cs);
  const ViewImg &im = it.v[tile.vi];
  const ViewGrad &vg = gtab.v[tile.vi];

  PixGrad pg[PPT];
  int mymax = -1;
  bool depth_any = false;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    PixGrad &p = pg[k];
    bool inside;
    int64_t pi;
    float pxf, pyf;
    tile.pixel(k, inside, pxf, pyf, pi);
    p = PixGrad{0.f, 0.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, -1, pxf, pyf};
    if (inside) {
      const float Tfin = im.t_final[pi];
      p.ll = min(im.last[pi] - (int)(c * BD), cnt - 1);
      p.gC0 = vg.gC[pi];
      p.gC1 = vg.gC[tile.npx + pi];
      p.gC2 = vg.gC[2 * tile.npx + pi];
      if (vg.gD) p.gD = vg.gD[pi];
      const float gO = vg.gO ? vg.gO[pi] : 0.f;
      p.TfG = Tfin * (gO - (p.gC0 * cam.bg[0] + p.gC1 * cam.bg[1] + p.gC2 * cam.bg[2]));
      if (K == 1) {
        p.T = Tfin;
      } else if (p.ll >= 0) {
        const ChunkRec r = chunk[(int64_t)item * (TW * TH) + tile.pidx(k)];
        p.T = r.t;
        p.S = p.gC0 * r.c0 + p.gC1 * r.c1 + p.gC2 * r.c2;
        p.AD = r.d;
      }
    }
    mymax = max(mymax, p.ll);
    depth_any = depth_any || p.gD != 0.f;
  }
  if (threadIdx.x == 0) s_max = -1;
  __syncthreads();
  if (mymax >= 0) atomicMax(&s_max, mymax);
  __syncthreads();
  const int maxll = __builtin_amdgcn_readfirstlane(s_max);  // uniform: the splat loop runs on scalar registers
  if (maxll < 0) return;  // uniform: no pixel has a contributor in this chunk
  const int slot = reduce10_slot(threadIdx.x & 63);
  const bool dep = __any(depth_any);
  for (int lo = maxll / SUB * SUB; lo >= 0; lo -= SUB) {
    const int hi = min(maxll, lo + SUB - 1);
    if (lo != maxll / SUB * SUB) __syncthreads();  // every wavefront is done with the previous sub-chunk
    stage<SUB, NT, true>(vals, cs + lo, hi - lo + 1, card, s_a, s_b, s_c);
    __syncthreads();
    if (dep)
      bwd_splats<PPT, true>(hi, lo, s_a, s_b, s_c, pg, slot, g2);
    else
      bwd_splats<PPT, false>(hi, lo, s_a, s_b, s_c, pg, slot, g2);
  }
}

// ---- per-Gaussian bucketed backward (a second a4 schedule) ---------------------------------
// The backward schedule of Sec. "CUDA-Related Acceleration Strategies" (per-Gaussian
// buckets), for 8x8 and 16x16 tiles: one wavefront per (tile, chunk) item; the chunk's splats,
// back to front, are taken in buckets of 64, lane L owning splat top - L of the bucket. The
// pixels that can have a contributor in the bucket (last contributor at or behind its front
// splat) stream through the lanes: in step s lane L works on the (s - L)-th of them, so every
// such pixel meets the bucket's splats in back-to-front order, one per step. A pixel's running state
// (transmittance and the colour and depth behind) lives in LDS: the lane that takes the pixel
// reads the state its neighbour wrote in the previous step and writes it back (LDS operations
// of one wavefront stay in program order). Per (splat, pixel) the operations are those of
// k_blend_bwd_chunk in the same order, so the pixel states are the same; each lane sums its
// splat's ten terms over the tile's pixels in registers and issues them as atomics once per
// bucket, with no wavefront reduction.
template <int TW, int TH, int BD>
__global__ __launch_bounds__(64) void k_blend_bwd_bucket(ViewTable vt, ImgTable it, GradTable gtab,
                                                         const Card *__restrict__ card,
                                                         const uint32_t *__restrict__ vals,
                                                         const uint32_t *__restrict__ range,
                                                         const uint2 *__restrict__ items,
                                                         const uint32_t *__restrict__ n_items,
                                                         const ChunkRec *__restrict__ chunk,
                                                         float *__restrict__ g2 /*[E][12]*/) {
  constexpr int NPIX = TW * TH;
  constexpr int NT = 64;
  __shared__ float4 s_a[BD], s_b[BD], s_c[BD];
  // pixel tables: running state and constants
  __shared__ float sT[NPIX], sS[NPIX], sAD[NPIX];  // S = dL/dC . colour behind
  __shared__ float sTfG[NPIX], sGC0[NPIX], sGC1[NPIX], sGC2[NPIX], sGD[NPIX];
  __shared__ int sLL[NPIX];
  __shared__ int s_list[NPIX];  // pixels that can have a contributor in the current bucket
  __shared__ float s_g[NT * 10];  // the bucket's ten sums per splat, for the transposed atomics
  __shared__ uint32_t s_rec[NT];
  __shared__ int s_max;
  uint32_t item;
  if (!item_of_block(n_items, item)) return;
  const uint2 tc = items[item];
  const uint32_t gt = tc.x, c = tc.y;
  const TileCtx<TW, TH, NPIX> tile(vt, gt);  // pidx(0) = lane index over the whole tile
  const ViewCam &cam = *tile.cam;
  const uint32_t s0 = range[2 * gt], e0 = range[2 * gt + 1];
  const uint32_t K = n_chunks(e0 - s0, BD);
  const uint32_t cs = s0 + c * BD;
  const int cnt = (int)min<uint32_t>(BD, e0 - cs);
  const ViewImg &im = it.v[tile.vi];
  const ViewGrad &vg = gtab.v[tile.vi];
  const int lane = threadIdx.x;
  if (lane == 0) s_max = -1;
  __syncthreads();
  int mymax = -1;
  for (int q = lane; q < NPIX; q += NT) {
    const int wx = tile.tx * TW + q % TW, wy = tile.ty * TH + q / TW;
    const bool inside = wx < cam.w && wy < cam.h;
    const int64_t pi = (int64_t)wy * cam.w + wx;
    float T = 1.f, S = 0.f, AD = 0.f, TfG = 0.f, gC0 = 0.f, gC1 = 0.f, gC2 = 0.f, gD = 0.f;
    int ll = -1;
    if (inside) {
      const float Tfin = im.t_final[pi];
      ll = min(im.last[pi] - (int)(c * BD), cnt - 1);
      gC0 = vg.gC[pi];
      gC1 = vg.gC[tile.npx + pi];
      gC2 = vg.gC[2 * tile.npx + pi];
      if (vg.gD) gD = vg.gD[pi];
      const float gO = vg.gO ? vg.gO[pi] : 0.f;
      TfG = Tfin * (gO - (gC0 * cam.bg[0] + gC1 * cam.bg[1] + gC2 * cam.bg[2]));
      if (K == 1) {
        T = Tfin;
      } else if (ll >= 0) {
        const ChunkRec r = chunk[(int64_t)item * NPIX + q];
        T = r.t;
        S = gC0 * r.c0 + gC1 * r.c1 + gC2 * r.c2;
        AD = r.d;
      }
    }
    sT[q] = T; sS[q] = S; sAD[q] = AD;
    sTfG[q] = TfG; sGC0[q] = gC0; sGC1[q] = gC1; sGC2[q] = gC2; sGD[q] = gD;
    sLL[q] = ll;
    mymax = max(mymax, ll);
  }
  if (mymax >= 0) atomicMax(&s_max, mymax);
  __syncthreads();
  const int maxll = __builtin_amdgcn_readfirstlane(s_max);
  if (maxll < 0) return;  // uniform: no pixel has a contributor in this chunk
  stage<BD, NT, true>(vals, cs, maxll + 1, card, s_a, s_b, s_c);
  __syncthreads();
  const float x0 = (float)(cam.x0 + tile.tx * TW), y0 = (float)(cam.y0 + tile.ty * TH);
  for (int top = maxll; top >= 0; top -= NT) {
    const int j = top - lane;  // this lane's splat (j < 0: idle)
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A, Cc = A;
    if (j >= 0) {
      A = s_a[j];
      B = s_b[j];
      Cc = s_c[j];
    }
    float g[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) g[v] = 0.f;
    // only pixels whose last contributor is at or behind the bucket's front splat pass through
    // it (the others keep their state); they are listed in tile order with wavefront ballots
    const int lo = max(top - (NT - 1), 0);
    int nact = 0;
#pragma unroll
    for (int k = 0; k < NPIX / NT; ++k) {
      const int q = lane + NT * k;
      const bool a = sLL[q] >= lo;
      const uint64_t m = __ballot(a);
      if (a) s_list[nact + __popcll(m & lanemask_lt())] = q;
      nact += __popcll(m);
    }
    const int steps = nact > 0 ? nact + (top - lo) : 0;  // no listed pixel: the bucket adds nothing
    for (int st = 0; st < steps; ++st) {
      // pixel r's state is written in step st by lane L and read in step st + 1 by lane L + 1:
      // the wave barrier keeps each step's LDS accesses in program order across the wavefront
      __builtin_amdgcn_wave_barrier();
      const int r = st - lane;
      if (j < 0 || r < 0 || r >= nact) continue;
      const int q = s_list[r];
      const float px = x0 + (float)(q % TW), py = y0 + (float)(q / TW);
      const float dx = px - A.x, dy = py - A.y;
      const float ar = splat_e2(splat_p2(B, splat_col(A, B, dx), dy));
      const bool act = j <= sLL[q] && fminf(kAlphaMax, ar) >= kAlphaMin;
      // a pixel this splat does not reach takes alpha 0 and its state stays as it is
      if (!act) continue;
      const float alpha = fminf(kAlphaMax, ar);
      const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
      const float T = sT[q] * inv;
      const float w = alpha * T;
      const float gC0 = sGC0[q], gC1 = sGC1[q], gC2 = sGC2[q], gD = sGD[q];
      const float S = sS[q], AD = sAD[q];
      g[6] += gC0 * w;
      g[7] += gC1 * w;
      g[8] += gC2 * w;
      g[9] += gD * w;
      const float rc = (gC0 * Cc.x + gC1 * Cc.y + gC2 * Cc.z) - S, rd = B.z - AD;
      sS[q] = fmaf(alpha, rc, S);
      sAD[q] = fmaf(alpha, rd, AD);
      sT[q] = T;
      const float dLda = fmaf(T, fmaf(gD, rd, rc), inv * sTfG[q]);
      const float dm = ar < kAlphaMax ? dLda : 0.f;  // clamped alpha: no power path
      const float dp = dm * ar;
      g[5] += dp;
      const float dpx = dp * dx, dpy = dp * dy;
      g[0] += dpx;
      g[1] += dpy;
      g[2] += dpx * dx;
      g[3] += dpx * dy;
      g[4] += dpy * dy;
    }
    // the lanes' sums leave through LDS, transposed: each atomic instruction then covers the
    // ten consecutive values of six or seven splats' records instead of one value in each of
    // 64 records, so its updates fall on a few memory lines
    __syncthreads();  // the previous bucket's reads of s_g are done
#pragma unroll
    for (int v = 0; v < 10; ++v) s_g[lane * 10 + v] = g[v];
    s_rec[lane] = j >= 0 ? __float_as_uint(Cc.w) : 0xFFFFFFFFu;
    __syncthreads();
#pragma unroll
    for (int i = lane; i < NT * 10; i += NT) {
      const int sl = i / 10, v = i - sl * 10;
      const uint32_t rec = s_rec[sl];
      const float val = s_g[i];
      if (rec != 0xFFFFFFFFu && val != 0.f) unsafeAtomicAdd(&g2[(int64_t)rec * 12 + v], val);
    }
  }
}

// ---- scratch layout and dispatch -----------------------------------------------------------
static inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Upper bound on items, rounded up to whole rounds of the XCD remap (kXcds * kGroup), so the
// launch of max_items workgroups reaches every item.
int64_t max_items(int64_t total_tiles, int64_t cap, int bd) {
  const int64_t m = total_tiles + (cap + bd - 1) / bd + 1;
  const int64_t r = (int64_t)kXcds * kGroup;
  return (m + r - 1) / r * r;
}

size_t blend_state_bytes(int64_t total_tiles, int64_t cap, int tw, int th, int bd) {
  const int64_t T = std::max<int64_t>(total_tiles, 1);
  const int64_t I = max_items(T, cap, bd);
  size_t s = a256(4 * (T + 1));                                     // item_base
  s += a256(8 * I);                                                 // items
  s += a256(4 * ((T + kItemChunk - 1) / kItemChunk + 1));          // block sums
  s += a256(16);                                                    // n_items, work list counts
  s += a256(sizeof(ChunkRec) * (size_t)I * tw * th);                // chunk records
  s += a256(4 * (size_t)I);                                         // fix-needed flags
  s += a256(8 * I);                                                 // window work list
  s += a256(4 * ((T + kItemChunk - 1) / kItemChunk + 1));          // first-window block sums
  s += 2 * a256(4 * (size_t)T);                                     // window tile lists
  return s;
}

struct BlendState {
  uint32_t *item_base;
  uint2 *items;
  uint32_t *bsum;
  uint32_t *n_items;  // [0] items; [1], [2] work and [3], [4] tile list counts of alternating windows
  ChunkRec *chunk;
  uint32_t *need_fix;
  uint2 *work;
  uint32_t *bsum0;
  uint32_t *live[2];
  int64_t I, cap;
};

static BlendState carve_state(void *base, int64_t total_tiles, int64_t cap, int tw, int th, int bd) {
  const int64_t T = std::max<int64_t>(total_tiles, 1);
  BlendState s;
  s.I = max_items(T, cap, bd);
  s.cap = cap;
  char *p = (char *)base;
  s.item_base = (uint32_t *)p;
  p += a256(4 * (T + 1));
  s.items = (uint2 *)p;
  p += a256(8 * s.I);
  s.bsum = (uint32_t *)p;
  p += a256(4 * ((T + kItemChunk - 1) / kItemChunk + 1));
  s.n_items = (uint32_t *)p;
  p += a256(16);
  s.chunk = (ChunkRec *)p;
  p += a256(sizeof(ChunkRec) * (size_t)s.I * tw * th);
  s.need_fix = (uint32_t *)p;
  p += a256(4 * (size_t)s.I);
  s.work = (uint2 *)p;
  p += a256(8 * s.I);
  s.bsum0 = (uint32_t *)p;
  p += a256(4 * ((T + kItemChunk - 1) / kItemChunk + 1));
  s.live[0] = (uint32_t *)p;
  p += a256(4 * (size_t)T);
  s.live[1] = (uint32_t *)p;
  return s;
}

// Compositing windows, in splats: chunks below kWin0 / BD first, then up to kWin1 / BD, then
// the rest (each at least one chunk longer than the one before).
constexpr uint32_t kWin0 = 512, kWin1 = 2048;
constexpr unsigned kLateChunkGrid = 4096, kLateScanGrid = 2048;  // fixed grids of the later windows

template <int TW, int TH, int BD, int NT, bool CNT>
static hipError_t fwd_impl_cnt(const ViewTable &vt, const ImgTable &it, const gs_projected &p, const uint32_t *vals,
                               const uint32_t *range, const BlendState &s, hipStream_t st) {
  const uint32_t T = vt.total_tiles;
  const uint32_t nb = (T + kItemChunk - 1) / kItemChunk;
  // the later windows cost four more launches: they are enqueued only when the pair capacity
  // allows tile lists that average more than kWin0 / 2 splats (else one window takes all)
  const int n_win = s.cap > (int64_t)T * (kWin0 / 2) ? 3 : 1;
  const uint32_t w0 = n_win == 1 ? 0xFFFFFFFFu : std::max<uint32_t>(1, kWin0 / BD);
  const uint32_t w1 = n_win == 1 ? 0xFFFFFFFFu : std::max<uint32_t>(w0 + 1, kWin1 / BD);
  const uint32_t q_bounds[4] = {0u, w0, w1, 0xFFFFFFFFu};
  uint32_t *n_work = s.n_items + 1;  // the first window's count is written by k_items_scan
  hipLaunchKernelGGL(k_items_reduce, dim3(nb), dim3(kItemThreads), 0, st, vt, range, BD, w0, s.bsum, s.bsum0);
  hipLaunchKernelGGL(k_items_scan, dim3(1), dim3(1024), 0, st, s.bsum, s.bsum0, nb, s.n_items, s.item_base, T,
                     n_work);
  hipLaunchKernelGGL(k_items_apply, dim3(nb), dim3(kItemThreads), 0, st, vt, range, BD, w0, (const uint32_t *)s.bsum,
                     (const uint32_t *)s.bsum0, s.item_base, s.items, s.work, s.need_fix);
  // 8x8 tiles: two items per wavefront (rounded up to whole rounds of the XCD remap)
  constexpr bool kPair = TW == 8 && TH == 8;
  const int64_t r = (int64_t)kXcds * kGroup;
  const unsigned pairs = (unsigned)(((s.I + 1) / 2 + r - 1) / r * r);
  uint32_t *ctr = s.n_items;  // [1], [2]: work list counts; [3], [4]: tile list counts
  for (int win = 0; win < n_win; ++win) {
    const int cur = win & 1, nxt = cur ^ 1;
    if (win == 0 && kPair)
      hipLaunchKernelGGL((k_blend_chunk_pair<BD, CNT>), dim3(pairs), dim3(64), 0, st, vt, it, (const Card *)p.card,
                         vals, range, (const uint2 *)s.work, (const uint32_t *)(ctr + 1 + cur), ctr + 1 + nxt,
                         ctr + 3 + nxt, (const uint32_t *)s.item_base, s.chunk);
    else if (win == 0)
      hipLaunchKernelGGL((k_blend_chunk<TW, TH, BD, NT, CNT, false>), dim3((unsigned)s.I), dim3(NT), 0, st, vt, it,
                         (const Card *)p.card, vals, range, (const uint2 *)s.work, (const uint32_t *)(ctr + 1 + cur),
                         ctr + 1 + nxt, ctr + 3 + nxt, (const uint32_t *)s.item_base, s.chunk);
    else  // the later windows hold far fewer items: one item per workgroup (the latency of a
          // two-item wavefront is not hidden there), walked by a fixed grid
      hipLaunchKernelGGL((k_blend_chunk<TW, TH, BD, NT, CNT, true>), dim3(kLateChunkGrid), dim3(NT), 0, st, vt, it,
                         (const Card *)p.card, vals, range, (const uint2 *)s.work, (const uint32_t *)(ctr + 1 + cur),
                         ctr + 1 + nxt, ctr + 3 + nxt, (const uint32_t *)s.item_base, s.chunk);
    hipLaunchKernelGGL((k_blend_scan<TW, TH, BD>), dim3(win == 0 ? T : kLateScanGrid), dim3(TW * TH), 0, st, vt, it,
                       range, (const uint32_t *)s.item_base, s.chunk, s.need_fix, q_bounds[win], q_bounds[win + 1],
                       q_bounds[std::min(win + 2, 3)], s.work, ctr + 1 + nxt,
                       win == 0 ? (const uint32_t *)nullptr : (const uint32_t *)s.live[cur],
                       (const uint32_t *)(ctr + 3 + cur), s.live[nxt], ctr + 3 + nxt);
  }
  hipLaunchKernelGGL((k_blend_fix<TW, TH, BD, NT, CNT>), dim3((unsigned)s.I), dim3(NT), 0, st, vt, it,
                     (const Card *)p.card, vals, range, (const uint2 *)s.items, (const uint32_t *)s.n_items,
                     (const uint32_t *)s.need_fix, s.chunk);
  hipLaunchKernelGGL((k_blend_suffix<TW, TH, BD>), dim3(T), dim3(TW * TH), 0, st, vt, it, range,
                     (const uint32_t *)s.item_base, s.chunk);
  return hipGetLastError();
}

// Contributor counting only when some view asks for that plane.
template <int TW, int TH, int BD, int NT>
static hipError_t fwd_impl(const ViewTable &vt, const ImgTable &it, const gs_projected &p, const uint32_t *vals,
                           const uint32_t *range, const BlendState &s, hipStream_t st) {
  bool cnt = false;
  for (int i = 0; i < vt.n_views; ++i) cnt = cnt || it.v[i].n_contrib != nullptr;
  return cnt ? fwd_impl_cnt<TW, TH, BD, NT, true>(vt, it, p, vals, range, s, st)
             : fwd_impl_cnt<TW, TH, BD, NT, false>(vt, it, p, vals, range, s, st);
}

template <int TW, int TH, int BD, int NT>
static hipError_t bwd_bucket_impl(const ViewTable &vt, const ImgTable &it, const GradTable &gtab,
                                  const gs_projected &p, const uint32_t *vals, const uint32_t *range,
                                  const BlendState &s, float *g2, hipStream_t st) {
  if constexpr (TW * TH > 256) {
    return hipErrorInvalidValue;  // the pixel tables of tiles over 256 pixels do not fit beside the staged splats
  } else {
    hipLaunchKernelGGL((k_blend_bwd_bucket<TW, TH, BD>), dim3((unsigned)s.I), dim3(64), 0, st, vt, it, gtab,
                       (const Card *)p.card, vals, range, (const uint2 *)s.items, (const uint32_t *)s.n_items,
                       (const ChunkRec *)s.chunk, g2);
    return hipGetLastError();
  }
}

template <int TW, int TH, int BD, int NT>
static hipError_t bwd_impl(const ViewTable &vt, const ImgTable &it, const GradTable &gtab, const gs_projected &p,
                           const uint32_t *vals, const uint32_t *range, const BlendState &s, float *g2,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_blend_bwd_chunk<TW, TH, BD, NT>), dim3((unsigned)s.I), dim3(NT), 0, st, vt, it, gtab,
                     (const Card *)p.card, vals, range,
                     (const uint2 *)s.items, (const uint32_t *)s.n_items, (const ChunkRec *)s.chunk, g2);
  return hipGetLastError();
}

// Lanes per workgroup by tile size: tiles of up to 256 pixels -> one wavefront (8x8: one pixel
// per lane; 8x16, 16x8: two; 16x16, 8x32, 32x8: four), larger ones -> 256 lanes (16x32, 32x16:
// two pixels per lane; 32x32: four). Chunk lengths 32, 64, 128 and 256.
#define GS_BLEND_DEPTHS(FN, TW, TH, NT, ...)                                                   \
  do {                                                                                         \
    if (bd == 32) return FN<TW, TH, 32, NT>(__VA_ARGS__);                                      \
    if (bd == 64) return FN<TW, TH, 64, NT>(__VA_ARGS__);                                      \
    if (bd == 128) return FN<TW, TH, 128, NT>(__VA_ARGS__);                                    \
    if (bd == 256) return FN<TW, TH, 256, NT>(__VA_ARGS__);                                    \
    return hipErrorInvalidValue;                                                               \
  } while (0)
#define GS_BLEND_DISPATCH(FN, ...)                                                             \
  do {                                                                                         \
    const int tw = vt.tile_w, th = vt.tile_h;                                                  \
    if (tw == 8 && th == 8) GS_BLEND_DEPTHS(FN, 8, 8, 64, __VA_ARGS__);                        \
    if (tw == 8 && th == 16) GS_BLEND_DEPTHS(FN, 8, 16, 64, __VA_ARGS__);                      \
    if (tw == 16 && th == 8) GS_BLEND_DEPTHS(FN, 16, 8, 64, __VA_ARGS__);                      \
    if (tw == 16 && th == 16) GS_BLEND_DEPTHS(FN, 16, 16, 64, __VA_ARGS__);                    \
    if (tw == 8 && th == 32) GS_BLEND_DEPTHS(FN, 8, 32, 64, __VA_ARGS__);                      \
    if (tw == 32 && th == 8) GS_BLEND_DEPTHS(FN, 32, 8, 64, __VA_ARGS__);                      \
    if (tw == 16 && th == 32) GS_BLEND_DEPTHS(FN, 16, 32, 256, __VA_ARGS__);                   \
    if (tw == 32 && th == 16) GS_BLEND_DEPTHS(FN, 32, 16, 256, __VA_ARGS__);                   \
    if (tw == 32 && th == 32) GS_BLEND_DEPTHS(FN, 32, 32, 256, __VA_ARGS__);                   \
    return hipErrorInvalidValue;                                                               \
  } while (0)

hipError_t launch_blend_fwd(int bd, const ViewTable &vt, const ImgTable &it, const gs_projected &p,
                            const uint32_t *vals, const uint32_t *range, void *state, int64_t cap, hipStream_t st) {
  if (vt.total_tiles == 0) return hipSuccess;
  const BlendState s = carve_state(state, vt.total_tiles, cap, vt.tile_w, vt.tile_h, bd);
  GS_BLEND_DISPATCH(fwd_impl, vt, it, p, vals, range, s, st);
}

hipError_t launch_blend_bwd(int bd, const ViewTable &vt, const ImgTable &it, const GradTable &gtab,
                            const gs_projected &p, const uint32_t *vals, const uint32_t *range, void *state,
                            int64_t cap, float *g2, hipStream_t st, int schedule) {
  if (vt.total_tiles == 0) return hipSuccess;
  const BlendState s = carve_state(state, vt.total_tiles, cap, vt.tile_w, vt.tile_h, bd);
  if (schedule == GS_BWD_BUCKETS) GS_BLEND_DISPATCH(bwd_bucket_impl, vt, it, gtab, p, vals, range, s, g2, st);
  GS_BLEND_DISPATCH(bwd_impl, vt, it, gtab, p, vals, range, s, g2, st);
}

}  // namespace gs
