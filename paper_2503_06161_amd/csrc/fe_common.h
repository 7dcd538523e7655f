// Internal declarations shared by the HIP sources of libfe4dgs_rast.so.
// Not part of the ABI (the ABI is include/fe4dgs_rast.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/fe4dgs_rast.h"

namespace fe {

// Blending rules (Sec. 3.3, eqs. 7-8, with the alpha thresholds of this rasterizer).
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;
constexpr float kQMax = 9.0f;

// The matrix-core kernels evaluate the falloff G = exp(-q/2) of eq. (1) as
// exp2(qs) with qs = -log2(e)/2 * q, from the conic scaled once per Gaussian
// (kQScale A, 2 kQScale B, kQScale C); the cut q <= 9 becomes qs >= kQsMin.
// Forward and backward use the same expression, so they take the same blend
// decisions.
constexpr float kQScale = -0.72134752044448170368f;   // -log2(e) / 2
constexpr float kQsMin = kQMax * kQScale;
__device__ __forceinline__ float4 scale_conic(float4 co) {
  return make_float4(kQScale * co.x, (2.0f * kQScale) * co.y, kQScale * co.z, co.w);
}
__device__ __forceinline__ float scaled_q(float4 cs, float dx, float dy) {
  return __builtin_fmaf(cs.x * dx, dx, __builtin_fmaf(cs.z * dy, dy, cs.y * dx * dy));
}
// Both cuts of a pair, q <= 9 and alpha = min(0.99, o G) >= 1/255, as one
// bound on qs, staged per Gaussian: o 2^qs >= 1/255 <=> qs >= -log2(255 o).
// Opacity 0 (padding) gives +inf: never blended.
__device__ __forceinline__ float blend_cut(float o) { return fmaxf(kQsMin, -__log2f(255.0f * o)); }

// Pixel box test on packed 16-bit coordinates: box = (x0 | y0 << 16,
// (x1 - x0) | (y1 - y0) << 16), p = px | py << 16.  p - origin wraps below
// the origin; the saturating subtraction of the extent is 0 on an axis iff
// the offset is within the extent.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 pack_box(short4 b) {
  return make_uint2((uint32_t)(uint16_t)b.x | ((uint32_t)(uint16_t)b.y << 16),
                    (uint32_t)(uint16_t)(b.z - b.x) | ((uint32_t)(uint16_t)(b.w - b.y) << 16));
}
__device__ __forceinline__ bool in_box(u16x2 p, uint2 box) {
  const u16x2 d = p - __builtin_bit_cast(u16x2, box.x);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(d, __builtin_bit_cast(u16x2, box.y))) == 0u;
}

// Binning: 1024 threads x 1 Gaussian per workgroup (16 waves, so that the
// LDS-atomic -> store chains of the pair loop overlap); per-tile counters in
// LDS up to kBinLdsTiles tiles; one workgroup of kBinOffThreads for the
// offsets.
constexpr int kBinThreads = 1024;
constexpr int kBinItems = 1;
constexpr int kBinChunk = kBinThreads * kBinItems;      // 1024
constexpr int kBinLdsTiles = 12288;
constexpr int kBinOffThreads = 1024;

// Largest supported Gaussian count.
constexpr int64_t kMaxGaussians = int64_t(1) << 23;

// Report words (unsigned long long) at StateView::report.
// kRepStatus is the forward's status (key overflow); kRepBwdStatus the last
// backward's (row overflow), cleared when a backward starts.
enum ReportWord {
  kRepStatus = 0, kRepKeys = 1, kRepVisible = 2, kRepNonFinite = 3, kRepRows = 4, kRepBwdStatus = 5, kRepWords = 8
};

// Device pointers into one frame's forward state plus its derived sizes.
struct StateView {
  float2* xy;
  float4* conic_o;
  float4* rgb;
  short4* box;
  uint32_t* dkey;           // [n] float32 depth bits (culled: all ones)
  uint32_t* count;          // [n] tiles touched
  uint32_t* tile_cnt;       // [tiles] pairs per tile, then placement cursors
  uint32_t* rel;            // [nblk][tiles] (LDS binning only)
  uint32_t* blk_sum;        // [nblk]
  uint32_t* blk_off;        // [nblk]
  uint32_t* blk_vis;        // [nblk] Gaussians of a binning workgroup with at least one key
  uint32_t* tile_order;     // [tiles] tiles by list length, longest first (the per-tile sort's launch order)
  unsigned long long* keys;     // [cap] depth bits << 32 | emit position
  unsigned long long* keys_b;   // [cap] merge buffer of the per-tile sort
  uint32_t* gauss;          // [cap] Gaussian index of each sorted pair
  uint2* ranges;
  uint32_t* tile_maxlast;   // [tiles] largest n_contrib per tile (compositing walk length)
  uint32_t* gofe;           // [cap] Gaussian of each emit position
  uint32_t* epos;           // [cap] emit position of each sorted pair
  uint32_t* eoff;           // [n] first emit position of each Gaussian
  unsigned long long* report;
  // sizes
  int64_t n;
  int64_t cap;
  int32_t tiles_x, tiles_y, tiles;
  int32_t nblk;             // binning workgroups (kBinChunk Gaussians each)
};

struct Layout {
  size_t total;
  size_t report, tile_cnt, ranges, xy, conic_o, rgb, box, dkey, count, rel, blk_sum, blk_off, blk_vis;
  size_t keys, keys_b, gauss, tile_maxlast, gofe, epos, eoff, tile_order;
  int64_t n, cap;
  int32_t tiles_x, tiles_y, tiles, nblk;
};

// Host helpers (fe_api.cpp).
bool compute_layout(const fe_config* cfg, const fe_camera* cam, int64_t n, Layout* L);
StateView make_view(const Layout& L, void* base);

// Per-frame projection constants, computed on the host in float64.
struct CamConst {
  double R[9];       // world -> camera rotation, row-major
  double t[3];
  double campos[3];  // -R^T t
  double fx, fy, cx, cy;
  double limx, limy; // Jacobian clamp limits on tx/tz, ty/tz (<= 0: none)
  double near_plane;
  double dilation;
  int32_t width, height;
};
CamConst make_cam_const(const fe_camera* cam, const fe_config* cfg);

// ---- launchers (each enqueues on `stream`, returns hipError_t) ----
hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t s);
// row offsets per tile (exclusive scan of the walk lengths) and cleared row
// indices for the frame's keys; rowidx 16-byte aligned with room for cap
// rounded up to 4 words
hipError_t launch_backward_prep(const uint32_t* walk, uint32_t* row_base, int64_t tiles, int64_t tiles_x, uint32_t* rowidx,
                                unsigned long long* report, int64_t cap, hipStream_t s);
hipError_t launch_project_fwd(const CamConst& cc, const fe_config* cfg, const fe_gaussians* g,
                              const StateView& v, hipStream_t s);
hipError_t launch_sort_and_bin(const fe_config* cfg, const StateView& v, hipStream_t s);
hipError_t launch_composite_fwd(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                const StateView& v, const fe_images* out, hipStream_t s);
hipError_t launch_composite_fwd_mfma(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                     const StateView& v, const fe_images* out, hipStream_t s);
hipError_t launch_composite_bwd(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                const StateView& v, const fe_images* fwd, const float* d_rgb,
                                const float* d_feat, const float* d_depth, float* grad2d, float* grad_feat,
                                hipStream_t s);
int backward_row_stride(int D);
hipError_t launch_composite_bwd_mfma(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                     const StateView& v, const fe_images* fwd, const float* d_rgb,
                                     const float* d_feat, const float* d_depth, const uint32_t* row_base, float* rows,
                                     int64_t row_cap, uint32_t* rowidx, hipStream_t s);
hipError_t launch_reduce_rows(const fe_config* cfg, const StateView& v, const uint32_t* rowidx,
                              const float* rows, float* grad2d, float* grad_feat, hipStream_t s);
hipError_t launch_project_bwd(const CamConst& cc, const fe_config* cfg, const fe_gaussians* g,
                              const StateView& v, const float* grad2d, const fe_grads* out,
                              hipStream_t s);

// Threads per tile of the matrix-core compositing kernels: one per pixel
// (every wave walks its pixels and runs the contractions) or two per pixel
// (wave-specialized: walker waves and matrix-core waves); threads_per_tile 0
// takes the wave-specialized kernel wherever it exists.
bool forward_wave_specialized(const fe_config* cfg);
bool backward_wave_specialized(const fe_config* cfg);

// ---- compositing of many frames from one work queue ----
// Items are (frame, tile) pairs.  The queue builder writes them longest first
// (by the tile's list length, or by its backward walk length), stores their
// number and sets the head counter, from which the workgroups of a persistent
// compositing kernel take items, to zero.
struct TileQueue {
  const uint2* items;
  const uint32_t* count;
  uint32_t* head;
};
struct TileQueueBuild {
  int32_t frames, tiles;               // tiles per frame
  const uint2* const* ranges;          // [frames] device pointers to each frame's tile ranges
  const uint32_t* const* walk;         // [frames] tile walk lengths (backward), or null (forward)
  uint2* items;                        // [frames * tiles]
  uint32_t* count;
  uint32_t* head;
};
hipError_t launch_build_tile_queue(const TileQueueBuild& b, hipStream_t s);
// Frame records are the argument blocks of the per-frame kernels, kept in
// device memory, one per frame.
bool composite_persistent_supported(const fe_config* cfg);
size_t composite_fwd_record_bytes();
void composite_fwd_record(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                          const fe_images* out, void* dst);
int composite_fwd_persistent_grid(const fe_config* cfg);
hipError_t launch_composite_fwd_persistent(const fe_config* cfg, const void* records, const TileQueue& q,
                                           int grid, hipStream_t s);
size_t composite_bwd_record_bytes();
void composite_bwd_record(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                          const fe_images* fwd, const float* d_rgb, const float* d_feat, const float* d_depth,
                          const uint32_t* row_base, float* rows, int64_t row_cap, uint32_t* rowidx, void* dst);
int composite_bwd_persistent_grid(const fe_config* cfg);
hipError_t launch_composite_bwd_persistent(const fe_config* cfg, const void* records, const TileQueue& q,
                                           int grid, hipStream_t s);

// ---- semantic decoder + feature loss ----
int decoder_grid_size(int in_dim, int target_dtype);
size_t decoder_partial_floats(int in_dim);
size_t decoder_sign_bytes(int64_t pixels);
hipError_t launch_decoder_l1(const fe_decoder* d, int grid, float* partial, void* signs, hipStream_t s);

// ---- small device helpers ----
// Workgroups of a launch are handed to the eight XCDs in turn (workgroup b
// runs on XCD b % 8), and each XCD has its own L2.  Tiles are dealt to the
// XCDs in runs of kXcdRun consecutive positions of the launch order (tile
// order, or the order by work with Z order inside a class), so that neighbouring
// tiles, which share 128-byte lines of the planar images (a 16-pixel tile row
// is half a line) and many Gaussians, are processed by one L2 one after the
// other, while every XCD still gets tiles from the whole image.  Workgroups
// past the last whole round keep their own index.
constexpr int kXcds = 8;
constexpr int kXcdRun = 8;   // 2, 4 and 8 measured alike, 16 1% and 32 3% slower per frame
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int round = kXcds * kXcdRun;
  if (b >= n - n % round) return b;
  const int x = b % kXcds, j = b / kXcds;
  return ((j / kXcdRun) * kXcds + x) * kXcdRun + j % kXcdRun;
}

// Per-tile quantities that steer loops containing barriers are read back as
// scalars: the compiler then treats them as uniform and never lowers such a
// loop (or an early exit around it) with a per-lane exit mask.
__device__ __forceinline__ uint2 uniform_u2(uint2 v) {
  return make_uint2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y));
}
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

template <typename T>
__device__ __forceinline__ float load_as_float(const void* p, int64_t i);

template <>
__device__ __forceinline__ float load_as_float<float>(const void* p, int64_t i) {
  return static_cast<const float*>(p)[i];
}

template <>
__device__ __forceinline__ float load_as_float<uint16_t>(const void* p, int64_t i) {
  return bf16_bits_to_float(static_cast<const uint16_t*>(p)[i]);
}

// Four consecutive channels of a feature row, kept in their storage form
// while in flight (two registers for bf16).  `vec` (uniform) says the row
// start and the channel group are aligned for one vector load.
template <typename FT>
struct FeatGroup;
template <>
struct FeatGroup<float> {
  float4 v;
  __device__ __forceinline__ void clear() { v = make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ __forceinline__ void load(const void* p, int64_t base, int c, int D, bool vec) {
    const float* f = static_cast<const float*>(p) + base + c;
    if (vec) {
      v = *reinterpret_cast<const float4*>(f);
    } else {
      v.x = c < D ? f[0] : 0.f;
      v.y = c + 1 < D ? f[1] : 0.f;
      v.z = c + 2 < D ? f[2] : 0.f;
      v.w = c + 3 < D ? f[3] : 0.f;
    }
  }
  __device__ __forceinline__ float get(int j) const { return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w; }
};
template <>
struct FeatGroup<uint16_t> {
  uint2 v;
  __device__ __forceinline__ void clear() { v = make_uint2(0u, 0u); }
  __device__ __forceinline__ void load(const void* p, int64_t base, int c, int D, bool vec) {
    const uint16_t* f = static_cast<const uint16_t*>(p) + base + c;
    if (vec) {
      v = *reinterpret_cast<const uint2*>(f);
    } else {
      const uint32_t e0 = c < D ? f[0] : 0u, e1 = c + 1 < D ? f[1] : 0u;
      const uint32_t e2 = c + 2 < D ? f[2] : 0u, e3 = c + 3 < D ? f[3] : 0u;
      v = make_uint2(e0 | (e1 << 16), e2 | (e3 << 16));
    }
  }
  __device__ __forceinline__ float get(int j) const {
    const uint32_t w = j < 2 ? v.x : v.y;
    return __uint_as_float((j & 1) ? (w & 0xFFFF0000u) : (w << 16));
  }
};

}  // namespace fe
