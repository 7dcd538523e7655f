// Binning of projected Gaussians into per-tile lists in depth order
// (Sec. 3.3: every Gaussian joins the list of each tile its 3-sigma box
// touches, and a tile blends its list front to back).
//
// Order of work (integer only):
//   1. count: a workgroup takes 1024 consecutive Gaussians, counts the pairs
//      it adds to every tile in LDS and reserves its share of each tile it
//      touches with one global atomic; it also sums its Gaussians' pair
//      counts and counts its visible Gaussians;
//   2. offsets (one workgroup): the visible and key totals (plain stores:
//      thousands of atomics on one report word from every wave of the
//      projection would serialise), the capacity check, tile
//      starts (exclusive scan of the tile counts -> [start, end) ranges) and
//      workgroup starts in the emit order (exclusive scan of the sums);
//   3. place: the pair of Gaussian g and tile t gets the 64-bit key
//      (depth bits << 32 | e), where e, its emit position, is g's first
//      position (the exclusive prefix of the pair counts in index order)
//      plus t's row-major place in g's tile rectangle; the key goes to a free
//      slot of t's segment and gofe[e] = g;
//   4. sort: one workgroup per tile sorts its segment (a counting sort on
//      depth buckets and each key's rank inside its bucket, or a merge sort
//      when buckets are crowded or the list is long) and writes the Gaussian
//      index and the emit position of every sorted pair.
// A tile holds at most one pair per Gaussian and emit positions increase
// with the Gaussian index, so ascending keys are ascending (depth bits,
// index): the order of the keys (tile, depth, index) within each tile.  The
// order in which slots are taken in step 3 does not matter.  Item counts
// stay on the device, so nothing here synchronises with the host.
#include "fe_common.h"

namespace fe {
namespace {

__global__ void zero_u32_kernel(uint32_t* p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = 0u;
}

// ---- block-wide exclusive scan (NW waves of 64 lanes) ----
template <int NW>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_warp, uint32_t& total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_warp[wave] = x;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = s_warp[w];
    if (w < wave) wave_off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return wave_off + x - v;
}

// ---- exclusive scan of u32 values (one workgroup; sizes here are per-tile
// arrays, a few thousand entries) ----
constexpr int kScanWg = 1024;

__device__ __forceinline__ void scan_small(const uint32_t* in, uint32_t* out, int64_t n) {
  __shared__ uint32_t s_warp[kScanWg / 64];
  constexpr int per = 4;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += kScanWg * per) {
    const int64_t i0 = base + (int64_t)threadIdx.x * per;
    uint32_t c[per], sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      c[k] = i0 + k < n ? in[i0 + k] : 0u;
      sum += c[k];
    }
    uint32_t step;
    uint32_t o = carry + block_exclusive_scan<kScanWg / 64>(sum, s_warp, step);
#pragma unroll
    for (int k = 0; k < per; ++k) {
      if (i0 + k < n) out[i0 + k] = o;
      o += c[k];
    }
    carry += step;
  }
}

// Backward preparation in one launch: workgroup 0 clears the backward's
// status word, scans the per-tile walk lengths into row offsets and orders
// the tiles for the compositing backward by walk length, longest first (at
// row_base + tiles + 1; classes by the two leading bits of the length, so a
// class spans a factor of at most sqrt 2, and Z order inside a class), so
// that the longest walks start in the first round; the others
// clear the row index of every key of the frame (min(report keys, cap) words,
// 16 bytes per store; nothing reads the words past the key count).
__global__ __launch_bounds__(kScanWg) void backward_prep_kernel(const uint32_t* walk, uint32_t* row_base, int64_t tiles, int64_t tiles_x,
                                                                uint4* rowidx, unsigned long long* report,
                                                                int64_t cap) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) report[kRepBwdStatus] = 0ull;
    scan_small(walk, row_base, tiles);
    constexpr int kCls = 128;
    __shared__ uint32_t s_cls[kCls];
    auto wclass = [](uint32_t w) {
      if (w < 4u) return (int)w;
      const int lz = 31 - __builtin_clz(w);
      return 2 * lz + (int)((w >> (lz - 1)) & 1u);
    };
    if (threadIdx.x < kCls) s_cls[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < tiles; t += kScanWg) atomicAdd(&s_cls[wclass(walk[t])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (int c = kCls - 1; c >= 0; --c) {
        const uint32_t n = s_cls[c];
        s_cls[c] = acc;
        acc += n;
      }
    }
    __syncthreads();
    uint32_t* order = row_base + tiles + 1;
    // inside a class the tiles are taken in Z order, so that the runs of
    // consecutive positions one XCD receives are compact blocks of tiles
    // that share Gaussians in that XCD's L2
    int lg = 0;
    const int64_t tiles_y = tiles_x > 0 ? (tiles + tiles_x - 1) / tiles_x : tiles;
    while (((int64_t)1 << lg) < tiles_x || ((int64_t)1 << lg) < tiles_y) ++lg;
    const int64_t zn = (int64_t)1 << (2 * lg);
    if (tiles_x > 0 && lg <= 15 && zn <= 8 * tiles) {
      auto unz = [](uint32_t v) {
        v &= 0x55555555u;
        v = (v | (v >> 1)) & 0x33333333u;
        v = (v | (v >> 2)) & 0x0f0f0f0fu;
        v = (v | (v >> 4)) & 0x00ff00ffu;
        return (int64_t)((v | (v >> 8)) & 0x0000ffffu);
      };
      for (int64_t z = threadIdx.x; z < zn; z += kScanWg) {
        const int64_t x = unz((uint32_t)z), y = unz((uint32_t)z >> 1);
        const int64_t t = y * tiles_x + x;
        if (x < tiles_x && t < tiles) order[atomicAdd(&s_cls[wclass(walk[t])], 1u)] = (uint32_t)t;
      }
    } else {
      for (int64_t t = threadIdx.x; t < tiles; t += kScanWg) order[atomicAdd(&s_cls[wclass(walk[t])], 1u)] = (uint32_t)t;
    }
    return;
  }
  const unsigned long long k = report[kRepKeys];
  const size_t n4 = ((k > (unsigned long long)cap ? 0 : (size_t)k) + 3) / 4;
  size_t i = (size_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)(gridDim.x - 1) * blockDim.x;
  for (; i < n4; i += stride) rowidx[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---- binning ----
struct BinArgs {
  const uint32_t* count;        // [n] tiles touched per Gaussian
  const short4* box;            // [n] pixel box (i0, j0, i1, j1)
  const uint32_t* dkey;         // [n] float32 depth bits
  uint32_t* tile_cnt;           // [tiles] pairs per tile (zeroed), then the next free slot
  uint32_t* rel;                // [nblk][tiles] a workgroup's first slot in a tile, from the tile start
  uint32_t* blk_sum;            // [nblk] pairs of a workgroup's Gaussians
  uint32_t* blk_off;            // [nblk] their first emit position
  uint32_t* blk_vis;            // [nblk] their Gaussians with at least one pair
  uint32_t* tile_order;         // [tiles] tiles by list length, longest first
  uint2* ranges;                // [tiles]
  unsigned long long* report;
  unsigned long long* keys;     // [cap]
  uint32_t* gofe;               // [cap] Gaussian of each emit position
  uint32_t* eoff;               // [n] first emit position of each Gaussian
  int64_t n, cap;
  int32_t tiles, tiles_x, tile_w, tile_h, nblk;
};

// The Gaussians of a binning workgroup in LDS: exclusive prefix of their
// pair counts (entry kBinChunk holds the total) and their tile rectangles
// (x0 | x1 << 16, y0 | y1 << 16).  Returns the workgroup's pair total.
__device__ __forceinline__ uint32_t bin_stage(const BinArgs& a, uint32_t* s_off, uint32_t* s_rx, uint32_t* s_ry,
                                              uint32_t* s_warp, uint32_t (&c)[kBinItems], int chunk) {
  const int64_t g0 = (int64_t)chunk * kBinChunk + (int64_t)threadIdx.x * kBinItems;
  uint32_t pre[kBinItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) {
    c[k] = g0 + k < a.n ? a.count[g0 + k] : 0u;
    pre[k] = sum;
    sum += c[k];
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan<kBinThreads / 64>(sum, s_warp, total);
  const int j0 = (int)threadIdx.x * kBinItems;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) {
    s_off[j0 + k] = off + pre[k];
    uint32_t rx = 0u, ry = 0u;
    if (c[k]) {
      const short4 b = a.box[g0 + k];
      rx = (uint32_t)(b.x / a.tile_w) | ((uint32_t)(b.z / a.tile_w) << 16);
      ry = (uint32_t)(b.y / a.tile_h) | ((uint32_t)(b.w / a.tile_h) << 16);
    }
    s_rx[j0 + k] = rx;
    s_ry[j0 + k] = ry;
  }
  if (threadIdx.x == 0) s_off[kBinChunk] = total;
  __syncthreads();
  return total;
}

// Every lane takes an equal run of the workgroup's pairs (in emit order) and
// calls f(Gaussian slot, tile, pair index) for each, so that large and small
// Gaussians cost the same per pair.
template <class F>
__device__ __forceinline__ void bin_walk(const uint32_t* s_off, const uint32_t* s_rx, const uint32_t* s_ry,
                                         uint32_t total, int tiles_x, F&& f) {
  const uint32_t q0 = (uint32_t)(((uint64_t)total * threadIdx.x) / kBinThreads);
  const uint32_t q1 = (uint32_t)(((uint64_t)total * (threadIdx.x + 1)) / kBinThreads);
  if (q0 >= q1) return;
  // the last Gaussian whose prefix is <= q0 holds pair q0 (one without pairs
  // shares its prefix with the next)
  int lo = 0, hi = kBinChunk;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_off[mid] <= q0) lo = mid; else hi = mid;
  }
  int j = lo;
  const uint32_t li = q0 - s_off[j];
  uint32_t rx = s_rx[j], ry = s_ry[j];
  int tx0 = (int)(rx & 0xFFFFu), tx1 = (int)(rx >> 16), ty1 = (int)(ry >> 16);
  const int w = tx1 - tx0 + 1;
  int ty = (int)(ry & 0xFFFFu) + (int)(li / (uint32_t)w);
  int tx = tx0 + (int)(li % (uint32_t)w);
  for (uint32_t q = q0; q < q1; ++q) {
    f(j, ty * tiles_x + tx, q);
    if (++tx > tx1) {
      ++ty;
      if (ty > ty1 && q + 1 < q1) {
        do { ++j; } while (s_off[j + 1] == s_off[j]);
        rx = s_rx[j];
        ry = s_ry[j];
        tx0 = (int)(rx & 0xFFFFu);
        tx1 = (int)(rx >> 16);
        ty = (int)(ry & 0xFFFFu);
        ty1 = (int)(ry >> 16);
      }
      tx = tx0;
    }
  }
}

// Step 1.  kLds: per-tile counters in LDS (dynamic, 4 bytes per tile) and one
// global atomic per touched tile; otherwise one global atomic per pair.
template <bool kLds>
__global__ __launch_bounds__(kBinThreads) void bin_count_kernel(BinArgs a) {
  extern __shared__ uint32_t s_tile[];
  __shared__ uint32_t s_off[kBinChunk + 1], s_rx[kBinChunk], s_ry[kBinChunk];
  __shared__ uint32_t s_warp[kBinThreads / 64];
  if constexpr (kLds)
    for (int t = threadIdx.x; t < a.tiles; t += kBinThreads) s_tile[t] = 0u;
  uint32_t c[kBinItems];
  const uint32_t total = bin_stage(a, s_off, s_rx, s_ry, s_warp, c, (int)blockIdx.x);   // its barriers order the zeroing
  uint32_t nvis = 0;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) nvis += (uint32_t)__syncthreads_count(c[k] != 0u);
  if (threadIdx.x == 0) {
    a.blk_sum[blockIdx.x] = total;
    a.blk_vis[blockIdx.x] = nvis;
  }
  bin_walk(s_off, s_rx, s_ry, total, a.tiles_x, [&](int, int t, uint32_t) {
    if constexpr (kLds)
      atomicAdd(&s_tile[t], 1u);
    else
      atomicAdd(&a.tile_cnt[t], 1u);
  });
  if constexpr (kLds) {
    // eight reservations in flight per lane: each returns only after a trip
    // to the device-wide atomic unit
    __syncthreads();
    uint32_t* rel = a.rel + (size_t)blockIdx.x * a.tiles;
    constexpr int kF = 8;
    for (int base = 0; base < a.tiles; base += kBinThreads * kF) {
      uint32_t cnt[kF], r[kF];
#pragma unroll
      for (int k = 0; k < kF; ++k) {
        const int t = base + k * kBinThreads + (int)threadIdx.x;
        cnt[k] = t < a.tiles ? s_tile[t] : 0u;
        r[k] = cnt[k] ? atomicAdd(&a.tile_cnt[t], cnt[k]) : 0u;
      }
#pragma unroll
      for (int k = 0; k < kF; ++k)
        if (cnt[k]) rel[base + k * kBinThreads + (int)threadIdx.x] = r[k];
    }
  }
}

// Step 2: one workgroup.
__global__ __launch_bounds__(kBinOffThreads) void bin_offsets_kernel(BinArgs a) {
  constexpr int NW = kBinOffThreads / 64;
  __shared__ uint32_t s_warp[NW];
  __shared__ unsigned long long s_part[NW], s_vpart[NW];
  // key total over the tiles, in 64 bits (a tile count is at most n), and
  // the visible Gaussians over the binning workgroups
  unsigned long long part = 0, vpart = 0;
  for (int t = threadIdx.x; t < a.tiles; t += kBinOffThreads) part += a.tile_cnt[t];
  for (int b = threadIdx.x; b < a.nblk; b += kBinOffThreads) vpart += a.blk_vis[b];
  for (int o = 32; o > 0; o >>= 1) {
    part += __shfl_xor(part, o, 64);
    vpart += __shfl_xor(vpart, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_part[threadIdx.x >> 6] = part;
    s_vpart[threadIdx.x >> 6] = vpart;
  }
  __syncthreads();
  unsigned long long tot64 = 0, vis64 = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    tot64 += s_part[w];
    vis64 += s_vpart[w];
  }
  tot64 = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(tot64 >> 32)) << 32) |
          __builtin_amdgcn_readfirstlane((uint32_t)tot64);
  if (threadIdx.x == 0) {
    a.report[kRepVisible] = vis64;
    a.report[kRepKeys] = tot64;
    if (tot64 > (unsigned long long)a.cap) a.report[kRepStatus] = (unsigned long long)FE_ERR_KEY_OVERFLOW;
  }
  if (tot64 > (unsigned long long)a.cap) {
    // ranges stay empty and nothing is placed; the compositing still takes
    // its tiles through the order
    for (int t = threadIdx.x; t < a.tiles; t += kBinOffThreads) a.tile_order[t] = (uint32_t)t;
    return;
  }
  // tile ranges; the tile counts become the tiles' first free slots.  The
  // lengths are also counted by class (class 0: empty; then the two leading
  // bits of the length, a factor of at most sqrt 2 per class) for the launch
  // order of the per-tile sort and the forward compositing
  __shared__ uint32_t s_cls[65];
  if (threadIdx.x < 65) s_cls[threadIdx.x] = 0u;
  __syncthreads();
  auto len_class = [](uint32_t c) {
    if (c == 0u) return 0;
    const int lz = 31 - __builtin_clz(c);
    return 1 + 2 * lz + (lz > 0 ? (int)((c >> (lz - 1)) & 1u) : 0);
  };
  constexpr int per = 4;
  uint32_t carry = 0;
  for (int base = 0; base < a.tiles; base += kBinOffThreads * per) {
    const int i0 = base + (int)threadIdx.x * per;
    uint32_t c[per], s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      c[k] = i0 + k < a.tiles ? a.tile_cnt[i0 + k] : 0u;
      s += c[k];
    }
    uint32_t step;
    uint32_t o = carry + block_exclusive_scan<NW>(s, s_warp, step);
#pragma unroll
    for (int k = 0; k < per; ++k) {
      if (i0 + k < a.tiles) {
        a.ranges[i0 + k] = make_uint2(o, o + c[k]);
        a.tile_cnt[i0 + k] = o;
        atomicAdd(&s_cls[len_class(c[k])], 1u);
      }
      o += c[k];
    }
    carry += step;
  }
  // longest class first: a class's first slot is the count of the longer classes
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 64; b >= 0; --b) {
      const uint32_t cb = s_cls[b];
      s_cls[b] = acc;
      acc += cb;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < a.tiles; t += kBinOffThreads) {
    const uint2 r = a.ranges[t];   // written above by this workgroup
    a.tile_order[atomicAdd(&s_cls[len_class(r.y - r.x)], 1u)] = (uint32_t)t;
  }
  // first emit position of each workgroup's Gaussians
  carry = 0;
  for (int base = 0; base < a.nblk; base += kBinOffThreads * per) {
    const int i0 = base + (int)threadIdx.x * per;
    uint32_t c[per], s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
      c[k] = i0 + k < a.nblk ? a.blk_sum[i0 + k] : 0u;
      s += c[k];
    }
    uint32_t step;
    uint32_t o = carry + block_exclusive_scan<NW>(s, s_warp, step);
#pragma unroll
    for (int k = 0; k < per; ++k) {
      if (i0 + k < a.nblk) a.blk_off[i0 + k] = o;
      o += c[k];
    }
    carry += step;
  }
}

// Step 3, with the same Gaussians per workgroup as step 1.
template <bool kLds>
__global__ __launch_bounds__(kBinThreads) void bin_place_kernel(BinArgs a) {
  extern __shared__ uint32_t s_next[];          // [tiles] next free slot of this workgroup (kLds)
  __shared__ uint32_t s_off[kBinChunk + 1], s_rx[kBinChunk], s_ry[kBinChunk], s_dk[kBinChunk];
  __shared__ uint32_t s_warp[kBinThreads / 64];
  if (a.report[kRepKeys] > (unsigned long long)a.cap) return;
  if constexpr (kLds) {
    // tiles this workgroup does not touch read words step 1 left unwritten;
    // their slots are never used
    const uint32_t* rel = a.rel + (size_t)blockIdx.x * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += kBinThreads) s_next[t] = a.tile_cnt[t] + rel[t];
  }
  const int64_t gb = (int64_t)blockIdx.x * kBinChunk;
  const int j0 = (int)threadIdx.x * kBinItems;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) s_dk[j0 + k] = gb + j0 + k < a.n ? a.dkey[gb + j0 + k] : 0u;
  uint32_t c[kBinItems];
  const uint32_t total = bin_stage(a, s_off, s_rx, s_ry, s_warp, c, (int)blockIdx.x);
  const uint32_t e0 = a.blk_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kBinItems; ++k)
    if (c[k]) a.eoff[gb + j0 + k] = e0 + s_off[j0 + k];
  const uint32_t cap = (uint32_t)a.cap;
  bin_walk(s_off, s_rx, s_ry, total, a.tiles_x, [&](int j, int t, uint32_t q) {
    uint32_t slot;
    if constexpr (kLds)
      slot = atomicAdd(&s_next[t], 1u);
    else
      slot = atomicAdd(&a.tile_cnt[t], 1u);
    const uint32_t e = e0 + q;
    if (slot < cap && e < cap) {   // always true for consistent counts
      a.keys[slot] = ((unsigned long long)s_dk[j] << 32) | e;
      a.gofe[e] = (uint32_t)(gb + j);
    }
  });
}

// ---- step 4: per-tile merge sort ----
constexpr int kTsThreads = 512;
constexpr int kTsItems = 16;
constexpr int kTsCap = kTsThreads * kTsItems;   // keys sorted in LDS at once
constexpr unsigned long long kKeyPad = ~0ull;   // above every key (a depth key is never all ones)

// LDS index with one unused word after every 16 keys, so that the 16
// consecutive keys of neighbouring lanes start in different banks
__device__ __forceinline__ int ts_ix(int i) { return i + (i >> 4); }

template <bool kPad>
__device__ __forceinline__ unsigned long long ts_load(const unsigned long long* p, int i) {
  return p[kPad ? ts_ix(i) : i];
}

// ascending bitonic network over the registers of one lane
template <int M>
__device__ __forceinline__ void sort_regs(unsigned long long (&v)[M]) {
#pragma unroll
  for (int k = 2; k <= M; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned long long x = v[i], y = v[l];
          const bool sw = (i & k) == 0 ? x > y : x < y;
          v[i] = sw ? y : x;
          v[l] = sw ? x : y;
        }
      }
}

// M outputs, starting at output d, of the merge of the ascending runs
// src[a0, a0 + la) and src[b0, b0 + lb) (equal keys: the first run first)
template <int M, bool kPad>
__device__ __forceinline__ void merge_at(const unsigned long long* src, int a0, int la, int b0, int lb, int d,
                                         unsigned long long (&v)[M]) {
  // merge path: i keys of the first run among the first d outputs
  int lo = max(0, d - lb), hi = min(d, la);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ts_load<kPad>(src, a0 + mid) <= ts_load<kPad>(src, b0 + d - 1 - mid))
      lo = mid + 1;
    else
      hi = mid;
  }
  int i = lo, j = d - lo;
  unsigned long long ua = i < la ? ts_load<kPad>(src, a0 + i) : kKeyPad;
  unsigned long long ub = j < lb ? ts_load<kPad>(src, b0 + j) : kKeyPad;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const bool ta = ua <= ub;
    v[k] = ta ? ua : ub;
    i += ta ? 1 : 0;
    j += ta ? 0 : 1;
    const bool ok = ta ? i < la : j < lb;
    const int at = ok ? (ta ? a0 + i : b0 + j) : a0;   // a0 is in range: the load may be issued either way
    const unsigned long long nx = ok ? ts_load<kPad>(src, at) : kKeyPad;
    ua = ta ? nx : ua;
    ub = ta ? ub : nx;
  }
}

// Sorts src[0, m) (m <= kTsCap) with the whole workgroup.  np is the padded
// length (a power of two, kTsItems <= np <= kTsCap, uniform); lane t ends
// with outputs t*kTsItems .. t*kTsItems + kTsItems - 1 in v.
__device__ __forceinline__ void block_sort(const unsigned long long* src, int m, int np, unsigned long long* s_k,
                                           unsigned long long (&v)[kTsItems]) {
  const int o = (int)threadIdx.x * kTsItems;
  const bool act = o < np;
#pragma unroll
  for (int k = 0; k < kTsItems; ++k) v[k] = (act && o + k < m) ? src[o + k] : kKeyPad;
  sort_regs(v);
  for (int run = kTsItems; run < np; run <<= 1) {
    if (act) {
#pragma unroll
      for (int k = 0; k < kTsItems; ++k) s_k[ts_ix(o + k)] = v[k];
    }
    __syncthreads();
    if (act) {
      const int a0 = o & ~(2 * run - 1);
      merge_at<kTsItems, true>(s_k, a0, run, a0 + run, run, o - a0, v);
    }
    __syncthreads();
  }
}

struct TileSortArgs {
  unsigned long long* keys;     // [cap] per-tile segments, unsorted
  unsigned long long* keys_b;   // [cap] merge buffer for lists longer than kTsCap
  const uint32_t* gofe;
  const uint2* ranges;
  const uint32_t* order;        // [tiles] launch order (longest lists first)
  const unsigned long long* report;
  uint32_t* gauss;              // [cap] Gaussian index of each sorted pair
  uint32_t* epos;               // [cap] its emit position
  int64_t cap;
};

// Counting sort on depth buckets, then each key's exact place inside its
// bucket by counting the smaller keys there.  The bucket of a key is
// (depth bits - smallest depth bits) >> sh, with sh chosen so that the
// tile's span of depth bits fills at most np/4 buckets: a bucket is a
// contiguous range of keys, so the result is the sorted order for any
// bucket sizes; a few keys per bucket keep the counting short.  Returns false
// (the same in every lane, nothing written) when a bucket holds more than
// kTsMaxBucket keys, e.g. when many depths are equal.  THREADS lanes hold
// PER_LANE keys each in registers; s_k holds THREADS * PER_LANE keys.
constexpr int kTsMaxBucket = 64;

__device__ __forceinline__ int pow2_at_least(int m);

template <int THREADS, int PER_LANE>
__device__ __forceinline__ bool bucket_rank_sort(const TileSortArgs& a, uint32_t start, int n, unsigned long long* s_k,
                                                 uint32_t* s_b, uint32_t* s_red) {
  constexpr int NW = THREADS / 64;
  constexpr int BPL = PER_LANE / 4;              // bucket counters per lane (np/4 <= THREADS * BPL)
  const int t = threadIdx.x;
  unsigned long long v[PER_LANE];
  uint32_t dmin = 0xFFFFFFFFu, dmax = 0u;
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j) {
    const int p = t + j * THREADS;
    v[j] = p < n ? a.keys[start + p] : 0ull;
    if (p < n) {
      const uint32_t d = (uint32_t)(v[j] >> 32);
      dmin = min(dmin, d);
      dmax = max(dmax, d);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmin = min(dmin, (uint32_t)__shfl_xor((int)dmin, o, 64));
    dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, o, 64));
  }
  const int wave = t >> 6;
  if ((t & 63) == 0) {
    s_red[wave] = dmin;
    s_red[NW + wave] = dmax;
  }
  const int np = pow2_at_least(n);
  const int nb = np >> 2;                       // buckets (a power of two, >= 4)
  for (int b = t; b < nb; b += THREADS) s_b[b] = 0u;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    dmin = min(dmin, s_red[w]);
    dmax = max(dmax, s_red[NW + w]);
  }
  dmin = __builtin_amdgcn_readfirstlane(dmin);
  dmax = __builtin_amdgcn_readfirstlane(dmax);
  const int span_bits = 32 - __clz((int)(dmax - dmin));
  const int sh = max(span_bits - (31 - __clz(nb)), 0);
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j)
    if (t + j * THREADS < n) atomicAdd(&s_b[((uint32_t)(v[j] >> 32) - dmin) >> sh], 1u);
  __syncthreads();
  // bucket starts and the largest bucket
  const int b0 = t * BPL;
  uint32_t c[BPL], sum = 0, big = 0;
#pragma unroll
  for (int k = 0; k < BPL; ++k) {
    c[k] = b0 + k < nb ? s_b[b0 + k] : 0u;
    big = max(big, c[k]);
  }
  for (int o = 32; o > 0; o >>= 1) big = max(big, (uint32_t)__shfl_xor((int)big, o, 64));
  if ((t & 63) == 0) s_red[2 * NW + wave] = big;
#pragma unroll
  for (int k = 0; k < BPL; ++k) sum += c[k];
  uint32_t tot;
  uint32_t off = block_exclusive_scan<NW>(sum, s_red + 3 * NW, tot);   // its barriers publish the maxima
#pragma unroll
  for (int w = 0; w < NW; ++w) big = max(big, s_red[2 * NW + w]);
  if ((uint32_t)__builtin_amdgcn_readfirstlane(big) > (uint32_t)kTsMaxBucket) return false;
#pragma unroll
  for (int k = 0; k < BPL; ++k) {
    if (b0 + k < nb) s_b[b0 + k] = off;
    off += c[k];
  }
  __syncthreads();
  // counting-sort placement; afterwards s_b[b] is the end of bucket b
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j)
    if (t + j * THREADS < n) s_k[atomicAdd(&s_b[((uint32_t)(v[j] >> 32) - dmin) >> sh], 1u)] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PER_LANE; ++j) {
    const int p = t + j * THREADS;
    if (p < n) {
      const unsigned long long key = s_k[p];
      const uint32_t b = ((uint32_t)(key >> 32) - dmin) >> sh;
      const uint32_t lo = b ? s_b[b - 1] : 0u, hi = s_b[b];
      uint32_t r = lo;
      for (uint32_t q = lo; q < hi; ++q) r += s_k[q] < key ? 1u : 0u;
      const uint32_t e = (uint32_t)key;
      a.gauss[start + r] = a.gofe[e];
      a.epos[start + r] = e;
    }
  }
  return true;
}

__device__ __forceinline__ int pow2_at_least(int m) {
  int p = kTsItems;
  while (p < m) p <<= 1;
  return p;
}

// One workgroup per tile: the bucket sort for lists of up to kTsCap keys
// whose buckets stay small; otherwise the merge sort, in LDS up to kTsCap
// keys, and for longer lists as sorted chunks of kTsCap keys merged through
// global memory.
__global__ __launch_bounds__(kTsThreads, 4) void tile_sort_kernel(TileSortArgs a) {
  __shared__ unsigned long long s_k[kTsCap + kTsCap / 16];
  __shared__ uint32_t s_b[kTsCap / 4];
  __shared__ uint32_t s_red[4 * (kTsThreads / 64)];
  if (a.report[kRepKeys] > (unsigned long long)a.cap) return;
  // the longest lists are sorted first, so that they do not start last
  const uint32_t tile = __builtin_amdgcn_readfirstlane(a.order[blockIdx.x]);
  const uint2 rg = uniform_u2(a.ranges[tile]);
  const int n = (int)(rg.y - rg.x);
  if (n <= 0) return;
  unsigned long long* seg = a.keys + rg.x;
  unsigned long long v[kTsItems];
  const int o = (int)threadIdx.x * kTsItems;
  if (n <= kTsCap) {
    if (bucket_rank_sort<kTsThreads, kTsCap / kTsThreads>(a, rg.x, n, s_k, s_b, s_red)) return;
    block_sort(seg, n, __builtin_amdgcn_readfirstlane(pow2_at_least(n)), s_k, v);
#pragma unroll
    for (int k = 0; k < kTsItems; ++k)
      if (o + k < n) {
        const uint32_t e = (uint32_t)v[k];
        a.gauss[rg.x + o + k] = a.gofe[e];
        a.epos[rg.x + o + k] = e;
      }
    return;
  }
  // longer lists: sorted chunks of kTsCap keys, then merge rounds through
  // global memory (every step of a round covers kTsCap outputs)
  const int nch = (n + kTsCap - 1) / kTsCap;
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = ch * kTsCap;
    const int m = min(kTsCap, n - c0);
    block_sort(seg + c0, m, __builtin_amdgcn_readfirstlane(pow2_at_least(m)), s_k, v);
#pragma unroll
    for (int k = 0; k < kTsItems; ++k)
      if (o + k < m) seg[c0 + o + k] = v[k];
    __syncthreads();
  }
  unsigned long long* src = seg;
  unsigned long long* dst = a.keys_b + rg.x;
  for (int run = kTsCap; run < n; run <<= 1) {
    for (int ob = 0; ob < n; ob += kTsCap) {
      const int p = ob + o;
      if (p < n) {
        const int a0 = p & ~(2 * run - 1);
        const int la = min(run, n - a0);
        const int b0 = a0 + la;
        const int lb = min(run, n - b0);
        merge_at<kTsItems, false>(src, a0, la, b0, lb, p - a0, v);
#pragma unroll
        for (int k = 0; k < kTsItems; ++k)
          if (p + k < n) dst[p + k] = v[k];
      }
    }
    __syncthreads();
    unsigned long long* t = src;
    src = dst;
    dst = t;
  }
  for (int p = o; p < n; p += kTsCap)
#pragma unroll
    for (int k = 0; k < kTsItems; ++k)
      if (p + k < n) {
        const uint32_t e = (uint32_t)src[p + k];
        a.gauss[rg.x + p + k] = a.gofe[e];
        a.epos[rg.x + p + k] = e;
      }
}

// ---- work queue of (frame, tile) items, longest first ----
// One workgroup: every item gets the bucket 1 + floor(log2(length)) (0 for
// an empty tile), buckets are laid out from the longest down, and items are
// placed in their bucket by LDS counters (the order inside a bucket is
// arbitrary: every item is processed by exactly one workgroup, so the
// results do not depend on it).  Backward queues leave out tiles with no
// walk.  The kernel also sets the count and clears the head counter.
constexpr int kQueueBuckets = 33;

__device__ __forceinline__ uint32_t queue_item_length(const TileQueueBuild& b, int f, int t) {
  const uint2 rg = b.ranges[f][t];
  const uint32_t len = rg.y - rg.x;
  return b.walk ? min(b.walk[f][t], len) : len;
}

__device__ __forceinline__ int queue_bucket(uint32_t len) { return len == 0 ? 0 : 32 - __clz(len); }

__global__ __launch_bounds__(1024) void build_tile_queue_kernel(TileQueueBuild b) {
  __shared__ uint32_t s_n[kQueueBuckets], s_pos[kQueueBuckets];
  const int total = b.frames * b.tiles;
  if (threadIdx.x < kQueueBuckets) s_n[threadIdx.x] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const uint32_t len = queue_item_length(b, e / b.tiles, e % b.tiles);
    if (b.walk && len == 0) continue;
    atomicAdd(&s_n[queue_bucket(len)], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t o = 0;
    for (int k = kQueueBuckets - 1; k >= 0; --k) {
      s_pos[k] = o;
      o += s_n[k];
    }
    *b.count = o;
    *b.head = 0u;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int f = e / b.tiles, t = e % b.tiles;
    const uint32_t len = queue_item_length(b, f, t);
    if (b.walk && len == 0) continue;
    const uint32_t pos = atomicAdd(&s_pos[queue_bucket(len)], 1u);
    b.items[pos] = make_uint2((uint32_t)f, (uint32_t)t);
  }
}

}  // namespace

hipError_t launch_backward_prep(const uint32_t* walk, uint32_t* row_base, int64_t tiles, int64_t tiles_x, uint32_t* rowidx,
                                unsigned long long* report, int64_t cap, hipStream_t s) {
  // clearing workgroups: one 16-byte group per thread over ceil(cap / 4)
  // groups, at least one whenever there is any key slot
  const size_t groups = ((size_t)(cap > 0 ? cap : 0) + 3) / 4;
  size_t zb = (groups + kScanWg - 1) / kScanWg;
  if (zb > 512) zb = 512;
  hipLaunchKernelGGL(backward_prep_kernel, dim3((unsigned)(1 + zb)), dim3(kScanWg), 0, s, walk, row_base, tiles, tiles_x,
                     reinterpret_cast<uint4*>(rowidx), report, cap);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_sort_and_bin(const fe_config* cfg, const StateView& v, hipStream_t s) {
  if (v.n == 0) return hipSuccess;
  BinArgs a;
  a.count = v.count;
  a.box = v.box;
  a.dkey = v.dkey;
  a.tile_cnt = v.tile_cnt;
  a.rel = v.rel;
  a.blk_sum = v.blk_sum;
  a.blk_off = v.blk_off;
  a.blk_vis = v.blk_vis;
  a.tile_order = v.tile_order;
  a.ranges = v.ranges;
  a.report = v.report;
  a.keys = v.keys;
  a.gofe = v.gofe;
  a.eoff = v.eoff;
  a.n = v.n;
  a.cap = v.cap;
  a.tiles = v.tiles;
  a.tiles_x = v.tiles_x;
  a.tile_w = cfg->tile_w;
  a.tile_h = cfg->tile_h;
  a.nblk = v.nblk;
  const bool lds = v.tiles <= kBinLdsTiles;
  const size_t lds_bytes = lds ? sizeof(uint32_t) * (size_t)v.tiles : 0;
  if (lds)
    hipLaunchKernelGGL(bin_count_kernel<true>, dim3(v.nblk), dim3(kBinThreads), lds_bytes, s, a);
  else
    hipLaunchKernelGGL(bin_count_kernel<false>, dim3(v.nblk), dim3(kBinThreads), 0, s, a);
  hipLaunchKernelGGL(bin_offsets_kernel, dim3(1), dim3(kBinOffThreads), 0, s, a);
  if (lds)
    hipLaunchKernelGGL(bin_place_kernel<true>, dim3(v.nblk), dim3(kBinThreads), lds_bytes, s, a);
  else
    hipLaunchKernelGGL(bin_place_kernel<false>, dim3(v.nblk), dim3(kBinThreads), 0, s, a);
  TileSortArgs t{v.keys, v.keys_b, v.gofe, v.ranges, v.tile_order, v.report, v.gauss, v.epos, v.cap};
  hipLaunchKernelGGL(tile_sort_kernel, dim3(v.tiles), dim3(kTsThreads), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_build_tile_queue(const TileQueueBuild& b, hipStream_t s) {
  if (b.frames < 1 || b.tiles < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(build_tile_queue_kernel, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

}  // namespace fe
