// Binning of projected Gaussians into per-tile lists in depth order
// (Sec. 3.4: every Gaussian joins the list of each tile its 3-sigma box
// touches, and a tile blends its list front to back).
//
// Order of work (integer only):
//   1. count: a workgroup takes 2048 consecutive Gaussians, counts the pairs
//      it adds to every tile in LDS and reserves its share of each tile it
//      touches with one global atomic; it also sums its Gaussians' pair
//      counts;
//   2. offsets (one workgroup): the key total and the capacity check, tile
//      starts (exclusive scan of the tile counts -> [start, end) ranges) and
//      workgroup starts in the emit order (exclusive scan of the sums);
//   3. place: the pair of Gaussian g and tile t gets the 64-bit key
//      (depth bits << 32 | e), where e, its emit position, is g's first
//      position (the exclusive prefix of the pair counts in index order)
//      plus t's row-major place in g's tile rectangle; the key goes to a free
//      slot of t's segment and gofe[e] = g;
//   4. sort: one workgroup per tile merge-sorts its segment and writes the
//      Gaussian index and the emit position of every sorted pair.
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

// ---- exclusive scan of u32 values ----
struct ScanArgs {
  const uint32_t* in;       // values
  uint32_t* out;            // exclusive prefix
  uint32_t* block_sums;     // [nblocks]
  int64_t n;
};

__global__ __launch_bounds__(kScanThreads) void scan_local_kernel(ScanArgs a) {
  __shared__ uint32_t s_warp[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    const uint32_t x = i < a.n ? a.in[i] : 0u;
    v[k] = sum;
    sum += x;
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan<kScanThreads / 64>(sum, s_warp, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < a.n) a.out[i] = off + v[k];
  }
  if (threadIdx.x == 0) a.block_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(uint32_t* sums, int nblocks) {
  __shared__ uint32_t s_warp[kScanThreads / 64];
  constexpr int per = kScanTopMax / kScanThreads;   // 16
  uint32_t v[per];
  uint32_t sum = 0;
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x * per + k;
    const uint32_t x = i < nblocks ? sums[i] : 0u;
    v[k] = sum;
    sum += x;
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan<kScanThreads / 64>(sum, s_warp, total);
  for (int k = 0; k < per; ++k) {
    const int i = threadIdx.x * per + k;
    if (i < nblocks) sums[i] = off + v[k];
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(uint32_t* out, const uint32_t* sums, int64_t n) {
  const uint32_t add = sums[blockIdx.x];
  if (add == 0) return;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads) {
    const int64_t i = base + k;
    if (i < n) out[i] += add;
  }
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
  uint2* ranges;                // [tiles]
  unsigned long long* report;
  unsigned long long* keys;     // [cap]
  uint32_t* gofe;               // [cap] Gaussian of each emit position
  uint32_t* eoff;               // [n] first emit position of each Gaussian
  int64_t n, cap;
  int32_t tiles, tiles_x, tile_w, tile_h, nblk;
};

// Step 1.  kLds: per-tile counters in LDS (dynamic, 4 bytes per tile) and one
// global atomic per touched tile; otherwise one global atomic per pair.
template <bool kLds>
__global__ __launch_bounds__(kBinThreads) void bin_count_kernel(BinArgs a) {
  extern __shared__ uint32_t s_tile[];
  __shared__ uint32_t s_warp[kBinThreads / 64];
  if constexpr (kLds) {
    for (int t = threadIdx.x; t < a.tiles; t += kBinThreads) s_tile[t] = 0u;
    __syncthreads();
  }
  const int64_t g0 = (int64_t)blockIdx.x * kBinChunk + (int64_t)threadIdx.x * kBinItems;
  uint32_t sum = 0;
  for (int k = 0; k < kBinItems; ++k) {
    const int64_t g = g0 + k;
    if (g >= a.n) break;
    const uint32_t c = a.count[g];
    if (c == 0u) continue;
    sum += c;
    const short4 b = a.box[g];
    const int tx0 = b.x / a.tile_w, tx1 = b.z / a.tile_w;
    const int ty0 = b.y / a.tile_h, ty1 = b.w / a.tile_h;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        const int t = ty * a.tiles_x + tx;
        if constexpr (kLds)
          atomicAdd(&s_tile[t], 1u);
        else
          atomicAdd(&a.tile_cnt[t], 1u);
      }
  }
  uint32_t total;
  block_exclusive_scan<kBinThreads / 64>(sum, s_warp, total);   // its barriers also order the LDS counts
  if (threadIdx.x == 0) a.blk_sum[blockIdx.x] = total;
  if constexpr (kLds) {
    uint32_t* rel = a.rel + (size_t)blockIdx.x * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += kBinThreads) {
      const uint32_t c = s_tile[t];
      if (c) rel[t] = atomicAdd(&a.tile_cnt[t], c);
    }
  }
}

// Step 2: one workgroup.
__global__ __launch_bounds__(kBinOffThreads) void bin_offsets_kernel(BinArgs a) {
  constexpr int NW = kBinOffThreads / 64;
  __shared__ uint32_t s_warp[NW];
  __shared__ unsigned long long s_part[NW];
  // key total over the tiles, in 64 bits (a tile count is at most n)
  unsigned long long part = 0;
  for (int t = threadIdx.x; t < a.tiles; t += kBinOffThreads) part += a.tile_cnt[t];
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  unsigned long long tot64 = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) tot64 += s_part[w];
  tot64 = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(tot64 >> 32)) << 32) |
          __builtin_amdgcn_readfirstlane((uint32_t)tot64);
  if (threadIdx.x == 0) {
    a.report[kRepKeys] = tot64;
    if (tot64 > (unsigned long long)a.cap) a.report[kRepStatus] = (unsigned long long)FE_ERR_KEY_OVERFLOW;
  }
  if (tot64 > (unsigned long long)a.cap) return;   // ranges stay empty; nothing is placed
  // tile ranges; the tile counts become the tiles' first free slots
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
      }
      o += c[k];
    }
    carry += step;
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
  __shared__ uint32_t s_warp[kBinThreads / 64];
  if (a.report[kRepKeys] > (unsigned long long)a.cap) return;
  if constexpr (kLds) {
    // tiles this workgroup does not touch read words step 1 left unwritten;
    // their slots are never used
    const uint32_t* rel = a.rel + (size_t)blockIdx.x * a.tiles;
    for (int t = threadIdx.x; t < a.tiles; t += kBinThreads) s_next[t] = a.tile_cnt[t] + rel[t];
  }
  const int64_t g0 = (int64_t)blockIdx.x * kBinChunk + (int64_t)threadIdx.x * kBinItems;
  uint32_t c[kBinItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kBinItems; ++k) {
    c[k] = g0 + k < a.n ? a.count[g0 + k] : 0u;
    sum += c[k];
  }
  uint32_t total;
  uint32_t e = a.blk_off[blockIdx.x] + block_exclusive_scan<kBinThreads / 64>(sum, s_warp, total);
  const uint32_t cap = (uint32_t)a.cap;
  for (int k = 0; k < kBinItems; ++k) {
    if (c[k] == 0u) continue;
    const int64_t g = g0 + k;
    a.eoff[g] = e;
    const unsigned long long hi = (unsigned long long)a.dkey[g] << 32;
    const short4 b = a.box[g];
    const int tx0 = b.x / a.tile_w, tx1 = b.z / a.tile_w;
    const int ty0 = b.y / a.tile_h, ty1 = b.w / a.tile_h;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        const int t = ty * a.tiles_x + tx;
        uint32_t slot;
        if constexpr (kLds)
          slot = atomicAdd(&s_next[t], 1u);
        else
          slot = atomicAdd(&a.tile_cnt[t], 1u);
        if (slot < cap && e < cap) {   // always true for consistent counts
          a.keys[slot] = hi | e;
          a.gofe[e] = (uint32_t)g;
        }
        ++e;
      }
  }
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
  const unsigned long long* report;
  uint32_t* gauss;              // [cap] Gaussian index of each sorted pair
  uint32_t* epos;               // [cap] its emit position
  int64_t cap;
};

__device__ __forceinline__ int pow2_at_least(int m) {
  int p = kTsItems;
  while (p < m) p <<= 1;
  return p;
}

__global__ __launch_bounds__(kTsThreads) void tile_sort_kernel(TileSortArgs a) {
  __shared__ unsigned long long s_k[kTsCap + kTsCap / 16];
  if (a.report[kRepKeys] > (unsigned long long)a.cap) return;
  const uint2 rg = uniform_u2(a.ranges[blockIdx.x]);
  const int n = (int)(rg.y - rg.x);
  if (n <= 0) return;
  unsigned long long* seg = a.keys + rg.x;
  unsigned long long v[kTsItems];
  const int o = (int)threadIdx.x * kTsItems;
  if (n <= kTsCap) {
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

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint32_t* sums, int64_t n, hipStream_t s) {
  ScanArgs a{in, out, sums, n};
  const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_local_kernel, dim3(nb), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanThreads), 0, s, out, (const uint32_t*)sums, n);
  return hipGetLastError();
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

hipError_t launch_scan_u32(const uint32_t* in, uint32_t* out, uint32_t* sums, int64_t n, hipStream_t s) {
  return scan_u32(in, out, sums, n, s);
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
  TileSortArgs t{v.keys, v.keys_b, v.gofe, v.ranges, v.report, v.gauss, v.epos, v.cap};
  hipLaunchKernelGGL(tile_sort_kernel, dim3(v.tiles), dim3(kTsThreads), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_build_tile_queue(const TileQueueBuild& b, hipStream_t s) {
  if (b.frames < 1 || b.tiles < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(build_tile_queue_kernel, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

}  // namespace fe
