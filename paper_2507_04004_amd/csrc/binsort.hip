// Stage a2 of the rasterizer: (tile, Gaussian) pairs with the alpha-max tile cull, sorted so
// that each tile's list is in depth order (Sec. "3D Gaussian Splatting Representation": the
// splats are arranged in depth order before alpha-blending; Sec. "CUDA-Related Acceleration
// Strategies": tiles whose largest weight is below 1/255 are culled).
//
// Order: one total order (tile, depth bits, record index). Built as
//   1. a stable LSD radix sort of the visible records by depth key (the first pass drops the
//      invisible ones, whose key is all ones, and stores how many remain on the device),
//   2. an exclusive scan of the per-record tile counts in that order,
//   3. emission of (global tile id, record) pairs in depth order, repeating the cull test on
//      the stored float32 splat record so the decisions equal those of the projection stage,
//   4. a stable LSD radix sort of the pairs by tile id, which keeps depth order inside a tile,
//   5. per-tile [begin, end) ranges.
// Radix passes use digits of at most 8 bits (the tile sort splits the tile-id bits evenly over
// its passes). Ranks inside a block come from wave64 ballots (peer masks of equal digits), so
// the sort is stable without per-item atomics. The pair count lives on the
// device; every kernel after the scan reads it, so no host synchronisation is needed.
#include <algorithm>

#include "gs_internal.hpp"

namespace gs {

constexpr int kRadixBits = 8;  // widest digit
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kRadixThreads = 256;  // one thread per digit of the widest digit
static_assert(kRadixThreads == kRadixDigits, "a radix block owns one digit per thread");
// Elements per block: the depth sort (one record per Gaussian and view) uses smaller blocks
// so that a 1M-record pass still spreads over the whole chip; the pair sort uses larger
// blocks, whose longer per-digit runs make the stores more contiguous.
constexpr int kItemsDepth = 4;
constexpr int kItemsPairs = 8;
constexpr int kRadixMinChunk = kRadixThreads * (kItemsDepth < kItemsPairs ? kItemsDepth : kItemsPairs);
constexpr int kScanThreads = 256;
constexpr int kScanItems = 1;
constexpr int kScanChunk = kScanThreads * kScanItems;
constexpr int kEmitStage = 4096;  // pairs staged in LDS per emission block (32 KB)

// Workgroups are dealt to the 8 XCDs round-robin. A radix pass gives each XCD groups of
// kChunkGroup consecutive chunks, so the histogram lines and the digit runs that neighbouring
// chunks share are completed inside one L2 instead of being written back in pieces by eight.
// The launch is rounded up to whole rounds (kChunkRound); workgroups past the last chunk exit.
constexpr int kXcdCount = 8;
constexpr int kChunkGroup = 16;
constexpr int kChunkRound = kXcdCount * kChunkGroup;
__device__ __forceinline__ int chunk_of_block() {
  const int x = (int)blockIdx.x % kXcdCount, k = (int)blockIdx.x / kXcdCount;
  return ((k / kChunkGroup) * kXcdCount + x) * kChunkGroup + k % kChunkGroup;
}

__device__ __forceinline__ int64_t live_count(int64_t n_static, const int64_t *n_dev, int64_t cap) {
  if (!n_dev) return n_static;
  int64_t v = *n_dev;
  return v < cap ? v : cap;
}

// Lanes of this wavefront whose BITS-bit digit equals this lane's digit (only valid lanes).
template <int BITS>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// ---- radix passes --------------------------------------------------------------------------
// drop: keys equal to kDropKey are left out (not counted here, not written by the scatter).
constexpr uint32_t kDropKey = 0xFFFFFFFFu;

template <int ITEMS, int BITS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n_static,
                                                              const int64_t *n_dev, int64_t cap, int shift,
                                                              uint32_t *__restrict__ hist, int nblocks, int stride,
                                                              bool drop) {
  constexpr int D = 1 << BITS;
  __shared__ uint32_t h[D];
  const int chunk = chunk_of_block();
  if (chunk >= nblocks) return;  // uniform per block
  const int64_t n = live_count(n_static, n_dev, cap);
  if (threadIdx.x < D) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)chunk * (kRadixThreads * ITEMS);
  if (base < n) {
    // every key of the block is requested before the first is ranked
    uint32_t kr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int64_t i = base + r * kRadixThreads + threadIdx.x;
      kr[r] = i < n ? keys[i] : 0u;
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = base + r * kRadixThreads + threadIdx.x < n && !(drop && kr[r] == kDropKey);
      const uint32_t d = (kr[r] >> shift) & (D - 1);
      const uint64_t peers = digit_peers<BITS>(d, valid);
      if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  if (threadIdx.x < D) hist[(int64_t)threadIdx.x * stride + chunk] = h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of that digit's counts over the chunks, in place;
// the digit total goes to tot[digit]. Each thread owns kScanRun consecutive counts, so a row
// of up to kRadixThreads * kScanRun blocks takes a single block-wide scan.
constexpr int kScanRun = 16;
__global__ __launch_bounds__(kRadixThreads) void k_radix_scan(uint32_t *__restrict__ hist, int nblocks, int stride,
                                                              uint32_t *__restrict__ tot) {
  __shared__ uint32_t lds[kRadixThreads / 64 + 1];
  uint32_t *row = hist + (int64_t)blockIdx.x * stride;
  uint32_t running = 0;
  for (int base = 0; base < nblocks; base += kRadixThreads * kScanRun) {
    const int i0 = base + threadIdx.x * kScanRun;
    uint32_t v[kScanRun];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      v[j] = i0 + j < nblocks ? row[i0 + j] : 0u;
      sum += v[j];
    }
    uint32_t total;
    uint32_t ex = running + block_exclusive_scan<kRadixThreads>(sum, lds, total);
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      if (i0 + j < nblocks) row[i0 + j] = ex;
      ex += v[j];
    }
    running += total;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = running;
}

// Stable scatter. vin == nullptr means the values are the input positions; kout may be null.
// The block first orders its chunk by digit in LDS (stable: round, then wavefront, then lane
// rank), then writes each digit's run to consecutive global positions, so the stores leave
// as contiguous runs instead of one scattered element per lane.
template <int ITEMS, int BITS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                 const uint32_t *__restrict__ vin,
                                                                 uint32_t *__restrict__ kout,
                                                                 uint32_t *__restrict__ vout, int64_t n_static,
                                                                 const int64_t *n_dev, int64_t cap, int shift,
                                                                 const uint32_t *__restrict__ hist,
                                                                 const uint32_t *__restrict__ tot, int nblocks,
                                                                 int stride, bool drop, int64_t *kept_total) {
  constexpr int NW = kRadixThreads / 64;
  constexpr int CHUNK = kRadixThreads * ITEMS;
  constexpr int D = 1 << BITS;
  __shared__ uint32_t s_k[CHUNK], s_v[CHUNK];
  __shared__ uint32_t s_glob[D];  // global start of this block's run of each digit
  __shared__ uint32_t s_loc[D];   // start of each digit's run inside the block
  __shared__ uint32_t s_run[D];
  __shared__ uint32_t s_wcnt[NW][D];
  __shared__ uint32_t lds[NW + 1];
  const int chunk = chunk_of_block();
  if (chunk >= nblocks) return;  // uniform per block
  const int64_t n = live_count(n_static, n_dev, cap);
  const int64_t base = (int64_t)chunk * CHUNK;
  if (base >= n) return;  // uniform per block
  const int cnt = (int)min<int64_t>(CHUNK, n - base);
  const int t = threadIdx.x;
  // the block's keys and values are requested before the digit offsets are computed
  uint32_t kr[ITEMS], vr[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = r * kRadixThreads + t;
    kr[r] = li < cnt ? kin[base + li] : 0u;
    vr[r] = li < cnt ? (vin ? vin[base + li] : (uint32_t)(base + li)) : 0u;
  }
  uint32_t total;
  const bool own = t < D;  // this thread owns digit t
  const uint32_t tt = own ? tot[t] : 0u;
  const uint32_t pre = block_exclusive_scan<kRadixThreads>(tt, lds, total);
  // the number of keys the pass keeps (all of them unless drop) for the passes and kernels after it
  if (kept_total && chunk == 0 && t == 0) *kept_total = (int64_t)total;
  const uint32_t h0 = own ? hist[(int64_t)t * stride + chunk] : 0u;
  const uint32_t h1 = !own ? 0u : (chunk + 1 < nblocks ? hist[(int64_t)t * stride + chunk + 1] : tt);
  uint32_t kept;  // keys of this block that the pass keeps
  const uint32_t loc = block_exclusive_scan<kRadixThreads>(h1 - h0, lds, kept);
  if (own) {
    s_glob[t] = pre + h0;
    s_loc[t] = loc;
    s_run[t] = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s_wcnt[w][t] = 0;
  }
  __syncthreads();
  const int wave = t >> 6;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = r * kRadixThreads + t;
    const uint32_t k = kr[r];
    const bool valid = li < cnt && !(drop && k == kDropKey);
    const uint32_t d = (k >> shift) & (D - 1);
    const uint64_t peers = digit_peers<BITS>(d, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = s_loc[d] + s_run[d];
      for (int w = 0; w < wave; ++w) off += s_wcnt[w][d];
      s_k[off + rank] = k;
      s_v[off + rank] = vr[r];
    }
    __syncthreads();
    if (own) {
      uint32_t add = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        add += s_wcnt[w][t];
        s_wcnt[w][t] = 0;
      }
      s_run[t] += add;
    }
    __syncthreads();
  }
  // the chunk's kept keys are in digit order in LDS: element j goes to its digit's global run
  for (int j = t; j < (int)kept; j += kRadixThreads) {
    const uint32_t k = s_k[j];
    const uint32_t d = (k >> shift) & (D - 1);
    const uint32_t pos = s_glob[d] + (uint32_t)j - s_loc[d];
    if (kout) kout[pos] = k;
    vout[pos] = s_v[j];
  }
}

// ---- pair counts, scan, emission -----------------------------------------------------------
// Also clears the tile ranges (an empty tile keeps [0, 0)).
// n_vis: the number of records in depth order (the visible ones), on the device.
__global__ __launch_bounds__(kScanThreads) void k_count_reduce(const uint32_t *__restrict__ order,
                                                               const uint32_t *__restrict__ n_tiles,
                                                               const int64_t *__restrict__ n_vis,
                                                               uint32_t *__restrict__ bsum,
                                                               uint32_t *__restrict__ tile_range, int64_t n_range) {
  __shared__ uint32_t lds[kScanThreads / 64 + 1];
  const int64_t n = *n_vis;
  for (int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; i < n_range;
       i += (int64_t)gridDim.x * kScanThreads)
    tile_range[i] = 0u;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + r * kScanThreads + threadIdx.x;
    if (i < n) s += n_tiles[order[i]];
  }
  uint32_t total;
  block_exclusive_scan<kScanThreads>(s, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the block sums; total pair count (int64) to *num_pairs.
// Also clears the length of the large-rectangle list that the emission appends to.
__global__ __launch_bounds__(1024) void k_count_scan_bsums(uint32_t *__restrict__ bsum, int64_t nb,
                                                           int64_t *__restrict__ num_pairs,
                                                           uint32_t *__restrict__ big_n) {
  __shared__ uint32_t lds[1024 / 64 + 1];
  uint64_t running = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<1024>(v, lds, total);
    if (i < nb) bsum[i] = (uint32_t)(running + ex);
    running += total;
  }
  if (threadIdx.x == 0) {
    *num_pairs = (int64_t)running;
    *big_n = 0u;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_emit_pairs(ViewTable vt, const uint32_t *__restrict__ order,
                                                             const int64_t *__restrict__ n_vis,
                                                             const Card *__restrict__ card,
                                                             const uint32_t *__restrict__ bsum, int64_t cap,
                                                             uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
                                                             uint32_t *__restrict__ big_e, uint32_t *__restrict__ big_off,
                                                             uint32_t *__restrict__ big_n) {
  __shared__ uint32_t lds[kScanThreads / 64 + 1];
  __shared__ uint32_t s_key[kEmitStage], s_val[kEmitStage];
  const int64_t i = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
  const int64_t n = *n_vis;
  // one card gather per record (a single memory line) supplies the count, centre, conic and
  // rectangle together
  uint32_t e = 0, cnt = 0;
  float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
  uint4 d = make_uint4(0u, 0u, 0u, 0u);
  if (i < n) {
    e = order[i];
    const Card &cd = card[e];
    A = cd.a;
    B = cd.b;
    d = cd.d;
    cnt = d.z;
  }
  uint32_t total;
  const uint32_t blk0 = bsum[blockIdx.x];
  const uint32_t off = blk0 + block_exclusive_scan<kScanThreads>(cnt, lds, total);
  // the block's pairs occupy one contiguous output range: stage it in LDS and store it as
  // whole lines (the ranges of large rectangles are left as holes, which k_emit_big fills
  // later in stream order)
  const bool staged = total <= (uint32_t)kEmitStage;
  short4 rc = make_short4(0, 0, -1, -1);
  int vi = 0;
  if (cnt) {
    vi = (int)(e / (uint32_t)vt.n);
    rc = make_short4((short)lo_i16(d.x), (short)hi_i16(d.x), (short)lo_i16(d.y), (short)hi_i16(d.y));
  }
  const int area = cnt ? (rc.z - rc.x + 1) * (rc.w - rc.y + 1) : 0;
  // small rectangles: one lane each, walking the kept-tile mask the projection stage stored
  if (cnt && area <= kCoopArea) {
    const ViewCam &cam = vt.v[vi];
    const int rw = rc.z - rc.x + 1;
    const float inv_rw = 1.0f / (float)rw;  // exact row for t < 32: (t + 1/2) / rw is never near an integer
    uint32_t mask = d.w;
    for (uint32_t j = 0; mask; ++j, mask &= mask - 1) {
      const int t = __ffs(mask) - 1;
      const int r = (int)(((float)t + 0.5f) * inv_rw);
      const uint32_t lt = (uint32_t)((rc.y + r) * cam.tiles_x + rc.x + (t - r * rw));
      if (staged) {
        s_key[off - blk0 + j] = cam.tile_base + lt;
        s_val[off - blk0 + j] = e;
      } else {
        const int64_t pos = (int64_t)off + j;
        if (pos < cap) {
          pkey[pos] = cam.tile_base + lt;
          pval[pos] = e;
        }
      }
    }
  }
  if (staged) {
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < total; k += kScanThreads) {
      const int64_t pos = (int64_t)blk0 + k;
      if (pos < cap) {
        pkey[pos] = s_key[k];
        pval[pos] = s_val[k];
      }
    }
  }
  // large rectangles go to a list that k_emit_big spreads over the whole chip: in depth order
  // the near (large) splats are neighbours, so visiting them here would leave a few
  // wavefronts with most of the work
  const bool is_big = cnt && area > kCoopArea;
  const uint64_t big = __ballot(is_big);
  if (big) {
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == __ffsll((unsigned long long)big) - 1) base = atomicAdd(big_n, (uint32_t)__popcll(big));
    base = __shfl(base, __ffsll((unsigned long long)big) - 1);
    if (is_big) {
      const uint32_t slot = base + (uint32_t)__popcll(big & lanemask_lt());
      big_e[slot] = e;
      big_off[slot] = off;
    }
  }
}

// One wavefront per large rectangle (grid-stride over the list): the wavefront tests 64
// tiles per step and compacts the kept ones with a ballot.
constexpr int kBigBlocks = 8192;  // more wavefronts than large rectangles at the headline view (32 k, 18.8 k)
__global__ __launch_bounds__(kScanThreads) void k_emit_big(ViewTable vt, const Card *__restrict__ card,
                                                           const uint32_t *__restrict__ big_e,
                                                           const uint32_t *__restrict__ big_off,
                                                           const uint32_t *__restrict__ big_n, int64_t cap,
                                                           uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval) {
  const uint32_t waves = gridDim.x * (kScanThreads / 64);
  const uint32_t nbig = *big_n;
  for (uint32_t it = blockIdx.x * (kScanThreads / 64) + threadIdx.x / 64; it < nbig; it += waves) {
    const uint32_t e = big_e[it], boff = big_off[it];
    const Card &cd = card[e];
    const float4 A = cd.a, B = cd.b;
    const uint4 d = cd.d;
    const ViewCam &cam = vt.v[e / (uint32_t)vt.n];
    wave_visit_kept_tiles(cam, vt.tile_w, vt.tile_h, A.x, A.y, B.x, B.y, B.z, B.w, lo_i16(d.x), hi_i16(d.x),
                          lo_i16(d.y), hi_i16(d.y), [&](uint32_t lt, uint32_t j, uint32_t) {
                            const int64_t pos = (int64_t)boff + j;
                            if (pos < cap) {
                              pkey[pos] = cam.tile_base + lt;
                              pval[pos] = e;
                            }
                          });
  }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Four consecutive sorted keys per thread (one 16-B load and the two neighbours): a tile's
// range starts where the key differs from the one before and ends where it differs from the
// one after. keys must be 16-B aligned.
__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, const int64_t *num_pairs, int64_t cap,
                              uint32_t *__restrict__ range) {
  const int64_t n = live_count(0, num_pairs, cap);
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= n) return;
  uint32_t k[6];  // keys i0 - 1 .. i0 + 4
  if (i0 + 4 <= n) {
    const uint4 q = *reinterpret_cast<const uint4 *>(keys + i0);
    k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) k[1 + u] = i0 + u < n ? keys[i0 + u] : 0xFFFFFFFFu;
  }
  k[0] = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
  k[5] = i0 + 4 < n ? keys[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + u;
    if (i >= n) break;
    if (i == 0 || k[u] != k[u + 1]) range[2 * (int64_t)k[u + 1]] = (uint32_t)i;
    if (i == n - 1 || k[u + 2] != k[u + 1]) range[2 * (int64_t)k[u + 1] + 1] = (uint32_t)(i + 1);
  }
}

// ---- host-side orchestration ---------------------------------------------------------------
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }
static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BinScratch {
  uint32_t *dk_a, *dv_a, *dk_b, *dv_b;  // depth sort ping-pong [n]
  uint32_t *bsum;                       // [ceil(n / kScanChunk)]
  uint32_t *pk_a, *pv_a, *pk_b, *pv_b;  // pair sort ping-pong [cap]
  uint32_t *hist;                       // [256][row stride: chunks rounded to kChunkRound]
  uint32_t *tot;                        // [256]
  uint32_t *big_n;                      // [1] length of the large-rectangle list
  int64_t *n_vis;                       // [1] visible records (kept by the first depth pass)
};

size_t bin_scratch_bytes(int64_t n, int64_t cap) {
  const int64_t nb_max = round_up(std::max<int64_t>(cdiv(std::max<int64_t>(n, 1), kRadixMinChunk),
                                                    cdiv(std::max<int64_t>(cap, 1), kRadixMinChunk)),
                                   kChunkRound);
  size_t s = 0;
  s += 4 * align256(sizeof(uint32_t) * std::max<int64_t>(n, 1));
  s += align256(sizeof(uint32_t) * cdiv(std::max<int64_t>(n, 1), kScanChunk));
  s += 4 * align256(sizeof(uint32_t) * std::max<int64_t>(cap, 1));
  s += align256(sizeof(uint32_t) * kRadixDigits * nb_max);
  s += align256(sizeof(uint32_t) * kRadixDigits);
  s += align256(16);
  s += align256(16);
  return s;
}

static BinScratch carve(void *base, int64_t n, int64_t cap) {
  const int64_t nb_max = round_up(std::max<int64_t>(cdiv(std::max<int64_t>(n, 1), kRadixMinChunk),
                                                    cdiv(std::max<int64_t>(cap, 1), kRadixMinChunk)),
                                   kChunkRound);
  char *p = (char *)base;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += align256(bytes);
    return (uint32_t *)r;
  };
  BinScratch s;
  const size_t nn = sizeof(uint32_t) * std::max<int64_t>(n, 1);
  const size_t cc = sizeof(uint32_t) * std::max<int64_t>(cap, 1);
  s.dk_a = take(nn); s.dv_a = take(nn); s.dk_b = take(nn); s.dv_b = take(nn);
  s.bsum = take(sizeof(uint32_t) * cdiv(std::max<int64_t>(n, 1), kScanChunk));
  s.pk_a = take(cc); s.pv_a = take(cc); s.pk_b = take(cc); s.pv_b = take(cc);
  s.hist = take(sizeof(uint32_t) * kRadixDigits * nb_max);
  s.tot = take(sizeof(uint32_t) * kRadixDigits);
  s.big_n = take(16);
  s.n_vis = (int64_t *)take(16);
  return s;
}

template <int ITEMS, int BITS>
static hipError_t radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_static,
                             const int64_t *n_dev, int64_t cap, int shift, const BinScratch &s, hipStream_t st,
                             bool drop = false, int64_t *kept_total = nullptr) {
  static_assert(BITS >= 1 && BITS <= kRadixBits, "digit width");
  const int64_t nmax = n_dev ? cap : n_static;
  const int nb = (int)std::max<int64_t>(cdiv(nmax, kRadixThreads * ITEMS), 1);
  const int grid = (int)round_up(nb, kChunkRound);  // also the histogram's row stride
  hipLaunchKernelGGL((k_radix_hist<ITEMS, BITS>), dim3(grid), dim3(kRadixThreads), 0, st, kin, n_static, n_dev, cap,
                     shift, s.hist, nb, grid, drop);
  hipLaunchKernelGGL(k_radix_scan, dim3(1 << BITS), dim3(kRadixThreads), 0, st, s.hist, nb, grid, s.tot);
  hipLaunchKernelGGL((k_radix_scatter<ITEMS, BITS>), dim3(grid), dim3(kRadixThreads), 0, st, kin, vin, kout, vout,
                     n_static, n_dev, cap, shift, s.hist, s.tot, nb, grid, drop, kept_total);
  return hipGetLastError();
}

// One pass of the tile sort with digits of `bits` bits (5 to 8).
static hipError_t tile_pass(int bits, const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                            const int64_t *n_dev, int64_t cap, int shift, const BinScratch &s, hipStream_t st) {
  switch (bits) {
    case 5: return radix_pass<kItemsPairs, 5>(kin, vin, kout, vout, 0, n_dev, cap, shift, s, st);
    case 6: return radix_pass<kItemsPairs, 6>(kin, vin, kout, vout, 0, n_dev, cap, shift, s, st);
    case 7: return radix_pass<kItemsPairs, 7>(kin, vin, kout, vout, 0, n_dev, cap, shift, s, st);
    default: return radix_pass<kItemsPairs, 8>(kin, vin, kout, vout, 0, n_dev, cap, shift, s, st);
  }
}

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// n: number of records (views x Gaussians); cap: pair capacity; total_tiles over all views.
hipError_t launch_bin_sort(const ViewTable &vt, const gs_projected &p, int64_t n, int64_t cap, uint32_t *vals,
                           uint32_t *tile_range, int64_t *num_pairs, void *scratch, hipStream_t st) {
  BinScratch s = carve(scratch, n, cap);
  hipError_t err;
  if (n == 0) {
    if ((err = fill_u32(tile_range, 2 * (int64_t)vt.total_tiles, 0u, st)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)num_pairs, 2, 0u);
    return hipGetLastError();
  }
  // 1. depth order of the visible records (stable; the record index breaks ties). The first
  // pass drops the invisible records and leaves their number in s.n_vis; the later passes
  // run over that many.
  const uint32_t *kin = p.dkey;
  const uint32_t *vin = nullptr;
  uint32_t *kb[2] = {s.dk_a, s.dk_b}, *vb[2] = {s.dv_a, s.dv_b};
  for (int pass = 0; pass < 4; ++pass) {
    uint32_t *ko = pass == 3 ? nullptr : kb[pass & 1];
    uint32_t *vo = vb[pass & 1];
    err = pass == 0 ? radix_pass<kItemsDepth, kRadixBits>(kin, vin, ko, vo, n, nullptr, 0, 0, s, st, true, s.n_vis)
                    : radix_pass<kItemsDepth, kRadixBits>(kin, vin, ko, vo, 0, s.n_vis, n, pass * kRadixBits, s, st);
    if (err != hipSuccess) return err;
    kin = ko;
    vin = vo;
  }
  const uint32_t *order = vin;  // == s.dv_b, s.n_vis entries
  // 2. exclusive scan of tile counts in depth order; total -> num_pairs
  const int64_t nbs = cdiv(n, kScanChunk);
  hipLaunchKernelGGL(k_count_reduce, dim3((unsigned)nbs), dim3(kScanThreads), 0, st, order, p.n_tiles,
                     (const int64_t *)s.n_vis, s.bsum, tile_range, 2 * (int64_t)vt.total_tiles);
  hipLaunchKernelGGL(k_count_scan_bsums, dim3(1), dim3(1024), 0, st, s.bsum, nbs, num_pairs, s.big_n);
  // 3. emission in depth order
  // the depth keys' ping-pong buffers are free now: they hold the large-rectangle list
  hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)nbs), dim3(kScanThreads), 0, st, vt, order,
                     (const int64_t *)s.n_vis,
                     (const Card *)p.card, s.bsum, cap, s.pk_a, s.pv_a, s.dk_a, s.dk_b, s.big_n);
  hipLaunchKernelGGL(k_emit_big, dim3(kBigBlocks), dim3(kScanThreads), 0, st, vt, (const Card *)p.card,
                     (const uint32_t *)s.dk_a, (const uint32_t *)s.dk_b, (const uint32_t *)s.big_n, cap, s.pk_a,
                     s.pv_a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  // 4. stable sort by global tile id; the id bits are split evenly over the passes (narrower
  // digits: fewer ballot rounds per key and longer runs per digit)
  int tile_bits = 1;
  while ((1ull << tile_bits) < (uint64_t)vt.total_tiles) ++tile_bits;
  const int passes = (int)cdiv(tile_bits, kRadixBits);
  const int digit_bits = std::max(5, (int)cdiv(tile_bits, passes));
  const uint32_t *pk = s.pk_a, *pv = s.pv_a;
  uint32_t *pkb[2] = {s.pk_b, s.pk_a}, *pvb[2] = {s.pv_b, s.pv_a};
  for (int pass = 0; pass < passes; ++pass) {
    uint32_t *ko = pkb[pass & 1];
    uint32_t *vo = pass == passes - 1 ? vals : pvb[pass & 1];
    if ((err = tile_pass(digit_bits, pk, pv, ko, vo, num_pairs, cap, pass * digit_bits, s, st)) != hipSuccess)
      return err;
    pk = ko;
    pv = vo;
  }
  // 5. tile ranges
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)cdiv(std::max<int64_t>(cap, 1), 1024)), dim3(256), 0, st, pk,
                     num_pairs, cap, tile_range);
  return hipGetLastError();
}

}  // namespace gs
