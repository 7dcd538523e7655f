// Binning of projected Gaussians into depth-ordered per-tile lists.
//
// Order of work (all integer, HBM-bound):
//   1. stable LSD radix sort of the Gaussians by the bits of their float32
//      view-space depth (3 passes of 11 bits; culled Gaussians carry the key
//      0xFFFFFFFF and emit nothing);
//   2. exclusive scan of the per-Gaussian tile counts taken in depth order;
//   3. emit one (tile id, Gaussian index) pair per tile of each Gaussian's
//      tile rectangle, in depth order;
//   4. stable LSD radix passes on the tile id (8 bits each), which leaves
//      every tile's pairs in (depth, index) order -- the order of the key
//      (tile << 32 | depth bits) with ties broken by index;
//   5. per-tile [start, end) ranges.
// Sorting N Gaussians by depth once and then only the tile digits of the K
// pairs moves about three times fewer bytes than sorting 64-bit keys.
//
// Every radix pass is deterministic: a chunk histogram per (digit, chunk), an
// exclusive scan over the digit-major matrix, then a scatter that ranks equal
// digits inside each wavefront with ballot masks (stable by position).
// Item counts that live on the device (the number of pairs) are read by the
// kernels themselves, so nothing here synchronises with the host.
#include "fe_common.h"

namespace fe {
namespace {

__device__ __forceinline__ uint32_t lane_rank(unsigned long long mask) {
  // number of set bits of `mask` below this lane
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ void zero_u32_kernel(uint32_t* p, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = 0u;
}

// ---- block-wide exclusive scan helpers (256 threads) ----
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
  for (int w = 0; w < 4; ++w) {
    const uint32_t t = s_warp[w];
    if (w < wave) wave_off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return wave_off + x - v;
}

// ---- exclusive scan of u32 values, optionally gathered through an index ----
struct ScanArgs {
  const uint32_t* in;       // values
  const uint32_t* gather;   // optional: value i = in[gather[i]]
  uint32_t* out;            // exclusive prefix
  uint32_t* block_sums;     // [nblocks]
  unsigned long long* total;  // optional: 64-bit grand total
  int64_t n;
};

__global__ __launch_bounds__(kScanThreads) void scan_local_kernel(ScanArgs a) {
  __shared__ uint32_t s_warp[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
  unsigned long long sum64 = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    uint32_t x = 0;
    if (i < a.n) x = a.gather ? a.in[a.gather[i]] : a.in[i];
    v[k] = sum;
    sum += x;
    sum64 += x;
  }
  uint32_t total;
  const uint32_t off = block_exclusive_scan(sum, s_warp, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < a.n) a.out[i] = off + v[k];
  }
  if (threadIdx.x == 0) a.block_sums[blockIdx.x] = total;
  if (a.total) {
    // 64-bit grand total (the 32-bit prefix may wrap only when the total
    // exceeds any key capacity, which the emit step then rejects)
    unsigned long long w = sum64;
    for (int o = 32; o > 0; o >>= 1) w += __shfl_down(w, o, 64);
    if ((threadIdx.x & 63) == 0 && w) atomicAdd(a.total, w);
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(uint32_t* sums, int nblocks) {
  __shared__ uint32_t s_warp[4];
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
  const uint32_t off = block_exclusive_scan(sum, s_warp, total);
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

// ---- radix pass ----
struct RadixArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;           // NULL: the value is the item's input position
  uint32_t* keys_out;
  uint32_t* vals_out;
  const uint32_t* gather;            // optional: write gather[val] instead of val ...
  uint32_t* epos;                    // ... and epos[output position] = val
  const unsigned long long* n_dev;   // item count on the device (may be NULL)
  int64_t n_const;                   // used when n_dev is NULL
  int64_t cap;                       // upper bound on the item count
  uint32_t* hist;                    // [bins][nchunks]
  uint32_t* totals;                  // [bins], zeroed
  int32_t nchunks;
  int32_t shift;
};

__device__ __forceinline__ int64_t radix_count(const RadixArgs& a) {
  if (!a.n_dev) return a.n_const;
  const unsigned long long k = *a.n_dev;
  return k > (unsigned long long)a.cap ? 0 : (int64_t)k;   // overflow: nothing is valid
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(RadixArgs a) {
  constexpr int BINS = 1 << BITS;
  __shared__ uint32_t h[BINS];
  const int64_t n = radix_count(a);
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  if (base >= n) return;   // chunks past the item count are never read
  for (int b = threadIdx.x; b < BINS; b += kSortThreads) h[b] = 0;
  __syncthreads();
  // each thread counts kSortItems consecutive keys and adds runs of equal
  // digits with one LDS atomic each: emitted tile ids come in runs (a
  // Gaussian's tiles, neighbouring Gaussians), and one atomic per key would
  // make the lanes of a wave collide on the same bin
  const int64_t i0 = base + (int64_t)threadIdx.x * kSortItems;
  uint32_t kv[kSortItems];
  if (i0 + kSortItems <= n) {
    const uint4* p4 = reinterpret_cast<const uint4*>(a.keys_in + i0);
#pragma unroll
    for (int k = 0; k < kSortItems / 4; ++k) {
      const uint4 v = p4[k];
      kv[4 * k] = v.x;
      kv[4 * k + 1] = v.y;
      kv[4 * k + 2] = v.z;
      kv[4 * k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) kv[k] = i0 + k < n ? a.keys_in[i0 + k] : 0u;
  }
  const int valid = (int)max((int64_t)0, min((int64_t)kSortItems, n - i0));
  uint32_t prev = 0u, run = 0u;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    if (k >= valid) break;
    const uint32_t d = (kv[k] >> a.shift) & (BINS - 1);
    if (run != 0u && d != prev) {
      atomicAdd(&h[prev], run);
      run = 0u;
    }
    prev = d;
    ++run;
  }
  if (run != 0u) atomicAdd(&h[prev], run);
  __syncthreads();
  for (int b = threadIdx.x; b < BINS; b += kSortThreads) {
    const uint32_t c = h[b];
    a.hist[(size_t)b * a.nchunks + blockIdx.x] = c;
    if (c) atomicAdd(&a.totals[b], c);
  }
}

// one block per digit: exclusive scan of its row over the chunks in use,
// offset by the digit's base (sum of the totals of the smaller digits)
template <int BITS>
__global__ __launch_bounds__(kScanThreads) void radix_scan_kernel(RadixArgs a) {
  __shared__ uint32_t s_warp[4];
  __shared__ uint32_t s_carry;
  const int bin = blockIdx.x;
  const int64_t n = radix_count(a);
  const int used = (int)((n + kSortChunk - 1) / kSortChunk);
  uint32_t t = 0;
  for (int b = threadIdx.x; b < bin; b += kScanThreads) t += a.totals[b];
  uint32_t tot;
  (void)block_exclusive_scan(t, s_warp, tot);
  if (threadIdx.x == 0) s_carry = tot;
  __syncthreads();
  uint32_t* row = a.hist + (size_t)bin * a.nchunks;
  for (int start = 0; start < used; start += kScanThreads) {
    const int i = start + threadIdx.x;
    const uint32_t x = i < used ? row[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(x, s_warp, total);
    const uint32_t carry = s_carry;
    if (i < used) row[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
}

// Scatter of one chunk: rank equal digits inside each wavefront with ballot
// masks (stable by position), turn the ranks into the chunk's local digit
// order, stage key / value / destination in LDS in that order, and write them
// out so that consecutive threads store consecutive destinations of the same
// digit run (runs of equal digits are contiguous in the output).
template <int BITS>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(RadixArgs a) {
  constexpr int BINS = 1 << BITS;
  __shared__ uint32_t cnt[4][BINS];
  __shared__ uint32_t lbase[BINS];          // exclusive prefix of the chunk's digit counts
  __shared__ uint32_t s_key[kSortChunk];
  __shared__ uint32_t s_val[kSortChunk];
  __shared__ uint32_t s_pos[kSortChunk];
  __shared__ uint32_t s_warp[4];
  const int64_t n = radix_count(a);
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  if (base >= n) return;   // uniform per block
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < 4 * BINS; k += kSortThreads) (&cnt[0][0])[k] = 0u;
  __syncthreads();
  uint32_t key[kSortItems], val[kSortItems], rank[kSortItems], dig[kSortItems];
  const int64_t wbase = base + (int64_t)wave * (kSortChunk / 4);
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = wbase + (int64_t)j * 64 + lane;
    const bool valid = i < n;
    key[j] = valid ? a.keys_in[i] : 0u;
    val[j] = valid ? (a.vals_in ? a.vals_in[i] : (uint32_t)i) : 0u;
  }
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = wbase + (int64_t)j * 64 + lane;
    const bool valid = i < n;
    const uint32_t d = (key[j] >> a.shift) & (BINS - 1);
    dig[j] = d;
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t below = lane_rank(m);
    uint32_t run = 0;
    if (valid) run = cnt[wave][d];
    rank[j] = run + below;
    // the lowest lane of each equal-digit group advances the running count
    if (valid && below == 0) cnt[wave][d] = run + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }
  __syncthreads();
  // per digit: global offsets of the four wavefronts' sub-chunks, and the
  // chunk's local digit order (exclusive scan of the digit counts)
  constexpr int DPT = (BINS + kSortThreads - 1) / kSortThreads;   // digits per thread
  uint32_t tot[DPT];
  uint32_t mysum = 0;
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = threadIdx.x * DPT + k;
    uint32_t t = 0;
    if (d < BINS) {
      uint32_t o = a.hist[(size_t)d * a.nchunks + blockIdx.x];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t c = cnt[w][d];
        cnt[w][d] = o;         // global start of wave w's run of digit d
        o += c;
        t += c;
      }
    }
    tot[k] = t;
    mysum += t;
  }
  uint32_t total;
  uint32_t lo = block_exclusive_scan(mysum, s_warp, total);
#pragma unroll
  for (int k = 0; k < DPT; ++k) {
    const int d = threadIdx.x * DPT + k;
    if (d < BINS) lbase[d] = lo;
    lo += tot[k];
  }
  __syncthreads();
  // local position of an item: digit base + items of the same digit in
  // earlier wavefronts + its rank; global position: wave run start + rank
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = wbase + (int64_t)j * 64 + lane;
    if (i < n) {
      const uint32_t d = dig[j];
      const uint32_t pos = cnt[wave][d] + rank[j];
      const uint32_t lpos = lbase[d] + (cnt[wave][d] - cnt[0][d]) + rank[j];
      s_key[lpos] = key[j];
      s_val[lpos] = val[j];
      s_pos[lpos] = pos;
    }
  }
  __syncthreads();
  const int cnt_here = (int)min((int64_t)kSortChunk, n - base);
  for (int t = threadIdx.x; t < cnt_here; t += kSortThreads) {
    const uint32_t pos = s_pos[t];
    if (pos < (uint64_t)n) {   // always true for a consistent histogram; guards the write
      const uint32_t v = s_val[t];
      if (a.keys_out) a.keys_out[pos] = s_key[t];
      if (a.gather) {
        a.vals_out[pos] = a.gather[v];
        a.epos[pos] = v;
      } else {
        a.vals_out[pos] = v;
      }
    }
  }
}

// ---- emit (tile, Gaussian) pairs in depth order ----
struct EmitArgs {
  const uint32_t* didx;      // depth-sorted Gaussian indices
  const uint32_t* count;     // per Gaussian
  const uint32_t* offsets;   // exclusive scan of count in depth order
  const short4* box;
  const unsigned long long* total;
  unsigned long long* report;
  uint32_t* tile_out;
  uint32_t* gauss_out;
  uint32_t* eoff;            // [n] first emit position of each Gaussian
  int64_t n;
  int64_t cap;
  int32_t tile_w, tile_h, tiles_x;
};

__global__ __launch_bounds__(256) void emit_kernel(EmitArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long total = *a.total;
  if (s == 0) {
    a.report[kRepKeys] = total;
    if (total > (unsigned long long)a.cap) a.report[kRepStatus] = (unsigned long long)FE_ERR_KEY_OVERFLOW;
  }
  if (s >= a.n || total > (unsigned long long)a.cap) return;
  const uint32_t g = a.didx[s];
  const uint32_t c = a.count[g];
  if (c == 0) return;
  uint32_t off = a.offsets[s];
  if ((uint64_t)off + c > (uint64_t)a.cap) return;
  a.eoff[g] = off;
  const short4 b = a.box[g];
  const int tx0 = b.x / a.tile_w, tx1 = b.z / a.tile_w;
  const int ty0 = b.y / a.tile_h, ty1 = b.w / a.tile_h;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      a.tile_out[off] = (uint32_t)(ty * a.tiles_x + tx);
      a.gauss_out[off] = g;
      ++off;
    }
}

__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* tiles, const unsigned long long* total,
                                                     int64_t cap, uint2* ranges, uint32_t ntiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long kt = *total;
  const int64_t k = kt > (unsigned long long)cap ? 0 : (int64_t)kt;
  if (i >= k) return;
  const uint32_t t = tiles[i];
  if (t >= ntiles) return;
  if (i == 0 || tiles[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i == k - 1 || tiles[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

hipError_t scan_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, uint32_t* sums,
                    unsigned long long* total, int64_t n, hipStream_t s) {
  ScanArgs a{in, gather, out, sums, total, n};
  const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_local_kernel, dim3(nb), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanThreads), 0, s, out, (const uint32_t*)sums, n);
  return hipGetLastError();
}

template <int BITS>
hipError_t radix_pass(RadixArgs a, hipStream_t s) {
  if (a.nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(radix_hist_kernel<BITS>, dim3(a.nchunks), dim3(kSortThreads), 0, s, a);
  hipLaunchKernelGGL(radix_scan_kernel<BITS>, dim3(1 << BITS), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(radix_scatter_kernel<BITS>, dim3(a.nchunks), dim3(kSortThreads), 0, s, a);
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
  return scan_u32(in, nullptr, out, sums, nullptr, n, s);
}

hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_sort_and_bin(const fe_config* cfg, const StateView& v, hipStream_t s) {
  hipError_t e;
  if (v.n == 0) return hipSuccess;
  // 1. depth sort of all n Gaussians: three 11-bit passes (A -> B -> A -> B);
  //    the first pass takes the implicit index as value
  {
    RadixArgs a0{v.dkey_a, nullptr, v.dkey_b, v.didx_b, nullptr, nullptr, nullptr, v.n, v.n, v.hist_n,
                 v.totals, v.nchunks_n, 0};
    if ((e = radix_pass<11>(a0, s)) != hipSuccess) return e;
    RadixArgs a1{v.dkey_b, v.didx_b, v.dkey_a, v.didx_a, nullptr, nullptr, nullptr, v.n, v.n, v.hist_n,
                 v.totals + kRadixBinsMax, v.nchunks_n, 11};
    if ((e = radix_pass<11>(a1, s)) != hipSuccess) return e;
    RadixArgs a2{v.dkey_a, v.didx_a, v.dkey_b, v.didx_b, nullptr, nullptr, nullptr, v.n, v.n, v.hist_n,
                 v.totals + 2 * kRadixBinsMax, v.nchunks_n, 22};
    if ((e = radix_pass<11>(a2, s)) != hipSuccess) return e;
  }
  // 2. offsets of each Gaussian's pairs, in depth order; 64-bit total -> report
  unsigned long long* total = v.report + kRepWords;   // scratch word after the report
  if ((e = scan_u32(v.count, v.didx_b, v.offsets, v.scan_sums, total, v.n, s)) != hipSuccess) return e;
  // 3. emit (tile id, Gaussian) pairs: tile ids into the buffer from which the
  //    last tile pass ends in tile_a, Gaussian ids into gofe (or straight into
  //    gauss_a when there is a single tile and no pass)
  const bool odd = (v.tile_passes & 1) != 0;
  EmitArgs ea;
  ea.didx = v.didx_b;
  ea.count = v.count;
  ea.offsets = v.offsets;
  ea.box = v.box;
  ea.total = total;
  ea.report = v.report;
  ea.tile_out = odd ? v.tile_b : v.tile_a;
  ea.gauss_out = v.tile_passes == 0 ? v.gauss_a : v.gofe;
  ea.eoff = v.eoff;
  ea.n = v.n;
  ea.cap = v.cap;
  ea.tile_w = cfg->tile_w;
  ea.tile_h = cfg->tile_h;
  ea.tiles_x = v.tiles_x;
  hipLaunchKernelGGL(emit_kernel, dim3((unsigned)((v.n + 255) / 256)), dim3(256), 0, s, ea);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4. stable passes on the tile digits.  The value carried is the emit
  //    position; the last pass writes the Gaussian index it maps to and the
  //    map sorted position -> emit position.
  uint32_t* tk_in = ea.tile_out;
  uint32_t* tk_out = odd ? v.tile_a : v.tile_b;
  const uint32_t* tv_in = nullptr;
  for (int p = 0; p < v.tile_passes; ++p) {
    const bool final_pass = p == v.tile_passes - 1;
    uint32_t* tv_out = final_pass ? v.gauss_a : v.gauss_b;
    RadixArgs a{tk_in, tv_in, tk_out, tv_out, final_pass ? v.gofe : nullptr, final_pass ? v.epos : nullptr,
                total, 0, v.cap, v.hist_k, v.totals + (3 + p) * kRadixBinsMax,
                v.nchunks_k, p * v.tile_bits};
    if ((e = (v.tile_bits == 11 ? radix_pass<11>(a, s) : radix_pass<8>(a, s))) != hipSuccess) return e;
    uint32_t* t = tk_in; tk_in = tk_out; tk_out = t;
    tv_in = tv_out;
  }
  // 5. per-tile ranges (ranges were zeroed with the state's counters)
  const unsigned rb = (unsigned)((v.cap + 255) / 256);
  if (rb) hipLaunchKernelGGL(ranges_kernel, dim3(rb), dim3(256), 0, s, (const uint32_t*)v.tile_a,
                             (const unsigned long long*)total, v.cap, v.ranges, (uint32_t)v.tiles);
  return hipGetLastError();
}

hipError_t launch_build_tile_queue(const TileQueueBuild& b, hipStream_t s) {
  if (b.frames < 1 || b.tiles < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(build_tile_queue_kernel, dim3(1), dim3(1024), 0, s, b);
  return hipGetLastError();
}

}  // namespace fe
