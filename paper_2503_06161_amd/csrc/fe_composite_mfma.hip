// Per-tile blending with the D-channel contraction on the matrix cores.
//
// For one tile and one batch of NB Gaussians in depth order, eq. (8) is a
// dense contraction: Z[p][c] += sum_i w_i(p) f_i[c], with w_i(p) =
// alpha_i(p) T_i(p) (zero for skipped or stopped pairs).  The weights are
// computed per pixel on the vector ALUs, sequentially over the batch (the
// transmittance recurrence), then the contraction runs as
// v_mfma_f32_32x32x16_bf16 with the feature matrix as A (channels x
// Gaussians) and the weights as B (Gaussians x pixels).
//
// Exactness: a float32 weight is split without error into three bf16 parts
// (w = hi + mid + lo; each part carries the next 8 significant bits, so the
// 24-bit significand is covered exactly).  BF16-stored features are exact
// bf16; float32 features are split the same way and the six products of
// combined order <= 2 are accumulated.  Every product of two bf16 values is
// exact in float32, so the result differs from a float32 dot product only in
// the order of the float32 additions.
//
// Layout: wave w of the workgroup owns tile pixels [64 w, 64 w + 64) in
// row-major tile order, lane l pixel 64 w + l during the weight pass.  The
// MFMA B operand wants, per lane l, pixel l % 32 of a 32-pixel block and
// Gaussians 8 (l / 32) + j; v_permlane32_swap of the weight registers for
// Gaussians j and 8 + j produces that layout for both pixel blocks at once.
#include "fe_common.h"

#include <cstring>
#include <type_traits>

#pragma clang fp contract(off)

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNB = 32;            // Gaussians per batch
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct MfmaArgs {
  const uint2* ranges;
  const uint32_t* gauss;
  const float2* xy;
  const float4* conic_o;
  const float4* rgb;
  const short4* box;
  const void* feat;
  float* out_rgb;
  float* out_feat;
  float* out_T;
  int32_t* out_n;
  float* out_depth;              // [H][W] or null
  uint32_t* tile_maxlast;        // [tiles] largest n_contrib of the tile
  const uint32_t* order;         // [tiles] tiles by list length, longest first (null: tile order)
  unsigned long long* report;
  float bg[3];
  int32_t W, H, tile_w, tiles_x;
  int32_t D;
  bool vec;                      // feature rows allow aligned 4-channel vector loads
};

__device__ __forceinline__ float bf16_to_f32(__bf16 h) { return (float)h; }

// The tile of a per-frame launch's workgroup: the binning's order (longest
// lists first, so that they do not start in the last round), dealt to the
// XCDs in runs as everywhere else.
__device__ __forceinline__ int fwd_tile(const MfmaArgs& a) {
  const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  return a.order ? (int)__builtin_amdgcn_readfirstlane(a.order[b]) : b;
}

// float32 -> three bf16 parts, hi + mid + lo == x exactly
__device__ __forceinline__ void split3(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  hi = (__bf16)x;
  const float r1 = x - bf16_to_f32(hi);
  mid = (__bf16)r1;
  const float r2 = r1 - bf16_to_f32(mid);
  lo = (__bf16)r2;
}

// Two float32 values -> three packed bf16 pairs (hi, mid, lo), each pair
// holding (value 0, value 1) in its (low, high) half.  Truncation splitting:
// hi keeps the top 8 significant bits, mid the next 8 significant bits of the
// (exact) remainder and lo the rest, so hi + mid + lo == x exactly for every
// normal x.  One byte permute packs the high halves of two values.
__device__ __forceinline__ void split3_pair(float x0, float x1, uint32_t& hi, uint32_t& mid, uint32_t& lo) {
  constexpr uint32_t kTop = 0xFFFF0000u, kSel = 0x07060302u;   // high halves of (x1, x0)
  const uint32_t u0 = __float_as_uint(x0), u1 = __float_as_uint(x1);
  hi = __builtin_amdgcn_perm(u1, u0, kSel);
  const float r0 = x0 - __uint_as_float(u0 & kTop), r1 = x1 - __uint_as_float(u1 & kTop);
  const uint32_t v0 = __float_as_uint(r0), v1 = __float_as_uint(r1);
  mid = __builtin_amdgcn_perm(v1, v0, kSel);
  const float t0 = r0 - __uint_as_float(v0 & kTop), t1 = r1 - __uint_as_float(v1 & kTop);
  lo = __builtin_amdgcn_perm(__float_as_uint(t1), __float_as_uint(t0), kSel);
}

// bf16 bits of four channels, packed two per register
__device__ __forceinline__ uint2 pack_bf16x4(__bf16 a0, __bf16 a1, __bf16 a2, __bf16 a3) {
  auto bits = [](__bf16 h) { return (uint32_t)__builtin_bit_cast(uint16_t, h); };
  return make_uint2(bits(a0) | (bits(a1) << 16), bits(a2) | (bits(a3) << 16));
}

// MFMA A operand (channels x Gaussians) from the Gaussian-major feature
// tile with two LDS transpose loads.  ds_read_b64_tr_b16 works on groups of
// 16 lanes: lane m of a group receives element m % 4 of the 4-element chunks
// addressed by lanes m / 4 + 4 j (j = 0..3) of its group.  Lane L therefore
// addresses row 8 (L / 32) + (L % 16) / 4 (+ 4 for the second load), column
// 16 ((L / 16) % 2) + 4 (L % 4) of the 32-channel block, and receives
// channel L % 32 of Gaussians 8 (L / 32) + 0..7.
template <int FROW>
__device__ __forceinline__ bf16x8 load_a_tr(const __bf16* plane, int krow0, int c0, int lane) {
  const int r = krow0 + 8 * (lane >> 5) + ((lane & 15) >> 2);
  const int c = c0 + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
  typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
  const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)(plane + r * FROW + c));
  const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)(plane + (r + 4) * FROW + c));
  // whole-register reinterpretation: per-element bf16 casts of the loaded
  // vectors were mis-compiled (elements 1..3 replaced by element 0)
  const u32x2 l2 = __builtin_bit_cast(u32x2, lo), h2 = __builtin_bit_cast(u32x2, hi);
  const u32x4 q = {l2[0], l2[1], h2[0], h2[1]};
  return __builtin_bit_cast(bf16x8, q);
}

// occupancy target: two waves per SIMD where everything fits without spills
// (D <= 32); wider feature rows need the whole register file
template <int DP>
constexpr int fwd_waves_per_eu() { return DP <= 32 ? 2 : 1; }

template <int DP, typename FT, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(fwd_waves_per_eu<DP>())))
void composite_fwd_mfma_kernel(MfmaArgs a) {
  constexpr int NPL = std::is_same<FT, float>::value ? 3 : 1;   // feature planes (hi, mid, lo)
  constexpr int CB = DP / 32;                                    // channel blocks
  // Gaussian-major feature rows; a stride of 16 banks mod 64 keeps the
  // transpose loads of 32 lanes (4 rows x 2 column halves) conflict-free
  constexpr int FROW = DP + 32;
  __shared__ float2 s_xy[kNB];
  __shared__ float4 s_co[kNB];
  __shared__ float s_tg[kNB];
  __shared__ float4 s_rgb[kNB];
  __shared__ int4 s_box[kNB];
  __shared__ __attribute__((aligned(16))) __bf16 s_f[NPL][kNB][FROW];
  __shared__ int s_maxlast;

  const int tile = fwd_tile(a);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tile_h = NT / a.tile_w;
  const int lp = threadIdx.x;                       // pixel of this lane in the weight pass
  const int px = (tile % a.tiles_x) * a.tile_w + lp % a.tile_w;
  const int py = (tile / a.tiles_x) * tile_h + lp / a.tile_w;
  const bool inside = (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const uint2 rg = a.ranges[tile];

  float T = 1.0f;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, C3 = 0.f;   // colour, depth
  int last = 0;
  bool done = !inside;
  f32x16 acc[2][CB];
#pragma unroll
  for (int pb = 0; pb < 2; ++pb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[pb][cb] = f32x16{};
  if (threadIdx.x == 0) s_maxlast = 0;

  // Staging is software-pipelined: the Gaussian ids of batch b+2 and the
  // records / feature rows of batch b+1 are loaded into registers while batch
  // b is blended, so the global-memory latency overlaps the compute.
  constexpr int FQ = DP / 4;                               // 4-channel groups per row
  constexpr int FI = (kNB * FQ + NT - 1) / NT;             // feature groups per thread
  uint32_t id_n[FI + 1];                                   // ids of the next batch to load
  FeatGroup<FT> fv[FI];                                    // prefetched feature groups
  float2 p_xy = make_float2(0.f, 0.f);
  float4 p_co = make_float4(0.f, 0.f, 0.f, 0.f), p_rgb = p_co;
  short4 p_box = make_short4(1, 1, 0, 0);
  auto load_ids = [&](uint32_t b0) {
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int i = (threadIdx.x + k * NT) / FQ;
      id_n[k] = (k * NT + (int)threadIdx.x < kNB * FQ && b0 + i < rg.y) ? a.gauss[b0 + i] : 0xFFFFFFFFu;
    }
    id_n[FI] = ((int)threadIdx.x < kNB && b0 + threadIdx.x < rg.y) ? a.gauss[b0 + threadIdx.x] : 0xFFFFFFFFu;
  };
  auto load_data = [&]() {
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int c = ((threadIdx.x + k * NT) % FQ) * 4;
      fv[k].clear();
      if (id_n[k] != 0xFFFFFFFFu && c < a.D) fv[k].load(a.feat, (int64_t)id_n[k] * a.D, c, a.D, a.vec);
    }
    if (id_n[FI] != 0xFFFFFFFFu) {
      const uint32_t g = id_n[FI];
      p_xy = a.xy[g];
      p_co = a.conic_o[g];
      p_rgb = a.rgb[g];
      p_box = a.box[g];
    }
  };
  if (rg.x < rg.y) {
    load_ids(rg.x);
    load_data();
    load_ids(rg.x + kNB);
  }
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kNB) {
    const int nb = (int)min((uint32_t)kNB, rg.y - b0);
    if (__syncthreads_count(!done) == 0) break;
    // ---- stage the batch from registers ----
    if ((int)threadIdx.x < kNB) {
      s_xy[threadIdx.x] = p_xy;
      s_co[threadIdx.x] = scale_conic(p_co);
      s_tg[threadIdx.x] = blend_cut(p_co.w);
      s_rgb[threadIdx.x] = p_rgb;
      s_box[threadIdx.x] = make_int4(p_box.x, p_box.y, p_box.z, p_box.w);
    }
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < kNB * FQ) {
        const int i = e / FQ;
        const int c = (e % FQ) * 4;
        __bf16 pl[NPL][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = i < nb ? fv[k].get(j) : 0.f;
          if constexpr (NPL == 1) {
            pl[0][j] = (__bf16)v;   // exact: the value is a bf16
          } else {
            split3(v, pl[0][j], pl[1][j], pl[2][j]);
          }
        }
#pragma unroll
        for (int p = 0; p < NPL; ++p)
          *reinterpret_cast<uint2*>(&s_f[p][i][c]) = pack_bf16x4(pl[p][0], pl[p][1], pl[p][2], pl[p][3]);
      }
    }
    // ---- issue the next batch's loads ----
    load_data();
    load_ids(b0 + 2 * kNB);
    __syncthreads();
    // ---- weights of this lane's pixel, front to back ----
    const bool wave_live = __ballot(!done) != 0ull;
    if (!wave_live) continue;
    // Per 16 Gaussians (one MFMA k-step): weights branch-free in groups of 8
    // (the per-pair alphas are independent, only the transmittance recurrence
    // is serial), then the contraction on the matrix cores.
    constexpr int GR = 8;
#pragma unroll
    for (int s = 0; s < kNB / 16; ++s) {
      float wv[16];
#pragma unroll
      for (int gi = 0; gi < 16 / GR; ++gi) {
        float al[GR];
        bool act[GR];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int i = 16 * s + gi * GR + u;
          const float2 m = s_xy[i];
          const float4 co = s_co[i];                // scaled conic, opacity
          const int4 b = s_box[i];
          const float dx = fpx - m.x, dy = fpy - m.y;
          const float qs = scaled_q(co, dx, dy);
          const bool inb = (px >= b.x) & (px <= b.z) & (py >= b.y) & (py <= b.w);
          const float alpha = fminf(kAlphaMax, co.w * __builtin_amdgcn_exp2f(qs));
          act[u] = (i < nb) & inb & (qs >= s_tg[i]);
          al[u] = alpha;
        }
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int i = 16 * s + gi * GR + u;
          const float Tn = T * (1.0f - al[u]);
          const bool live = act[u] & !done;
          const bool stop = live & (Tn < kTStop);
          const bool take = live & !stop;
          done = done | stop;
          const float w = take ? al[u] * T : 0.f;
          const float4 c = s_rgb[i];
          C0 = __builtin_fmaf(w, c.x, C0);
          C1 = __builtin_fmaf(w, c.y, C1);
          C2 = __builtin_fmaf(w, c.z, C2);
          C3 = __builtin_fmaf(w, c.w, C3);
          wv[gi * GR + u] = w;
          T = take ? Tn : T;
          last = take ? (int)(b0 - rg.x) + i + 1 : last;
        }
      }
      bool any = false;
#pragma unroll
      for (int i = 0; i < 16; ++i) any |= wv[i] != 0.f;
      if (__ballot(any) == 0ull) continue;
      bf16x8 bw[2][3];   // [pixel block][hi, mid, lo]
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(wv[j]), __float_as_uint(wv[8 + j]), false,
                                                        false);
        __bf16 h, m, l;
        split3(__uint_as_float(r[0]), h, m, l);
        bw[0][0][j] = h; bw[0][1][j] = m; bw[0][2][j] = l;
        split3(__uint_as_float(r[1]), h, m, l);
        bw[1][0][j] = h; bw[1][1][j] = m; bw[1][2][j] = l;
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        bf16x8 fa[NPL];
#pragma unroll
        for (int p = 0; p < NPL; ++p) fa[p] = load_a_tr<FROW>(&s_f[p][0][0], 16 * s, 32 * cb, lane);
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
          f32x16 z = acc[pb][cb];
          if constexpr (NPL == 1) {
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][0], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][1], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][2], z, 0, 0, 0);
          } else {
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][0], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][1], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], bw[pb][0], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], bw[pb][2], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], bw[pb][1], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[2], bw[pb][0], z, 0, 0, 0);
          }
          acc[pb][cb] = z;
        }
      }
    }
  }
  // ---- outputs ----
  const int64_t HW = (int64_t)a.W * a.H;
  if (inside) {
    const int64_t p = (int64_t)py * a.W + px;
    a.out_rgb[p] = __builtin_fmaf(T, a.bg[0], C0);
    a.out_rgb[HW + p] = __builtin_fmaf(T, a.bg[1], C1);
    a.out_rgb[2 * HW + p] = __builtin_fmaf(T, a.bg[2], C2);
    if (a.out_depth) a.out_depth[p] = C3;
    a.out_T[p] = T;
    a.out_n[p] = last;
  }
  // feature image: accumulator row = channel, column = pixel
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
    const int lpo = wave * 64 + 32 * pb + (lane & 31);
    const int ox = (tile % a.tiles_x) * a.tile_w + lpo % a.tile_w;
    const int oy = (tile / a.tiles_x) * tile_h + lpo / a.tile_w;
    if (ox < a.W && oy < a.H) {
      const int64_t p = (int64_t)oy * a.W + ox;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int c = 32 * cb + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (c < a.D) a.out_feat[c * HW + p] = acc[pb][cb][v];
        }
    }
  }
  // per-tile walk length (used by the backward to size its partial rows)
  if (last > 0) atomicMax(&s_maxlast, last);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.tile_maxlast[tile] = (uint32_t)s_maxlast;
    if (s_maxlast > 0) atomicAdd(&a.report[kRepRows], (unsigned long long)s_maxlast);
  }
}

// Wave-specialized form (BF16-stored features, D <= 128).  The block has
// 2 NT threads: NT "walker" threads (one pixel each) compute the weights of
// batch k front to back and leave them in LDS as float32 rows (pixel-major),
// while NT "accumulator" threads run the D-channel contraction of batch k-1
// on the matrix cores and stage batch k+1.  Accumulator wave w owns the 64
// pixels of walker wave w and all channel blocks, so every weight is split
// into its three exact bf16 parts once, by the one wave that consumes it.
// Colour and depth (eq. 7) ride along as one more channel block: its rows
// 0-3, 4-7 and 8-11 hold the three exact bf16 parts of (r, g, b, depth) of
// each Gaussian, so the block's three row groups sum to C = sum_i w_i c_i
// with every product exact and float32 accumulation.
// The roles need about half the registers each, so two waves share a SIMD.
// One barrier per batch (the early-termination count); weights and records
// are double-buffered, feature rows triple-buffered.
template <int DP, int NT>
__device__ __forceinline__ void fwd_ws_tile(const MfmaArgs& a, const int tile) {
  constexpr int CB = DP / 32;
  constexpr int NW = NT / 64;
  constexpr int FROW = DP + 32;
  constexpr int WROW = kNB + 4;                // float32 weight row of a pixel (bank spread)
  __shared__ float2 s_xy[2][kNB];
  __shared__ float4 s_co[2][kNB];
  __shared__ float s_tg[2][kNB];
  __shared__ uint2 s_box[2][kNB];             // packed (origin, extent)
  // feature rows: channels 0..DP-1, then the colour block (12 used columns)
  __shared__ __attribute__((aligned(16))) __bf16 s_f[3][kNB][FROW];
  __shared__ __attribute__((aligned(16))) float s_w[2][NT][WROW];
  __shared__ float s_T[NT];                    // final transmittance of each pixel
  __shared__ int s_any[2][NW][2];              // the chunk has a nonzero weight in the k step
  __shared__ int s_maxlast;

  const bool walker = (int)threadIdx.x < NT;
  const int q = walker ? (int)threadIdx.x : (int)threadIdx.x - NT;
  const int lane = q & 63;
  const int wave = q >> 6;
  const int tile_h = NT / a.tile_w;
  const int px = (tile % a.tiles_x) * a.tile_w + q % a.tile_w;
  const int py = (tile / a.tiles_x) * tile_h + q / a.tile_w;
  const bool inside = walker & (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const u16x2 pp = {(unsigned short)px, (unsigned short)py};
  const uint2 rg = uniform_u2(a.ranges[tile]);
  const int nbatch = (int)((rg.y - rg.x + kNB - 1) / kNB);
  if (threadIdx.x == 0) s_maxlast = 0;

  // ---- accumulators: software-pipelined staging ----
  constexpr int FQ = DP / 4;
  constexpr int FI = (kNB * FQ + NT - 1) / NT;
  uint32_t id_n[FI + 1];
  FeatGroup<uint16_t> fv[FI];
  float2 p_xy = make_float2(0.f, 0.f);
  float4 p_co = make_float4(0.f, 0.f, 0.f, 0.f), p_rgb = p_co;
  short4 p_box = make_short4(1, 1, 0, 0);
  auto load_ids = [&](int k) {
    const uint32_t b0 = rg.x + (uint32_t)k * kNB;
#pragma unroll
    for (int j = 0; j < FI; ++j) {
      const int i = (q + j * NT) / FQ;
      id_n[j] = (j * NT + q < kNB * FQ && k < nbatch && b0 + i < rg.y) ? a.gauss[b0 + i] : 0xFFFFFFFFu;
    }
    id_n[FI] = (q < kNB && k < nbatch && b0 + q < rg.y) ? a.gauss[b0 + q] : 0xFFFFFFFFu;
  };
  auto load_data = [&]() {
#pragma unroll
    for (int j = 0; j < FI; ++j) {
      const int c = ((q + j * NT) % FQ) * 4;
      fv[j].clear();
      if (id_n[j] != 0xFFFFFFFFu && c < a.D) fv[j].load(a.feat, (int64_t)id_n[j] * a.D, c, a.D, a.vec);
    }
    if (id_n[FI] != 0xFFFFFFFFu) {
      const uint32_t g = id_n[FI];
      p_xy = a.xy[g];
      p_co = a.conic_o[g];
      p_rgb = a.rgb[g];
      p_box = a.box[g];
    }
  };
  auto stage = [&](int k) {
    const int b2 = k & 1, b3 = k % 3;
    const int nb = (int)min((uint32_t)kNB, rg.y - (rg.x + (uint32_t)k * kNB));
    if (q < kNB) {
      // conic as (a, 2 b, c, opacity); padding entries get opacity 0
      s_xy[b2][q] = p_xy;
      const float4 cs = scale_conic(p_co);
      s_co[b2][q] = make_float4(cs.x, cs.y, cs.z, q < nb ? p_co.w : 0.f);
      s_tg[b2][q] = blend_cut(q < nb ? p_co.w : 0.f);
      s_box[b2][q] = pack_box(p_box);
      // colour block: exact three-part split of (r, g, b, depth)
      uint32_t h0, m0, l0, h1, m1, l1;
      split3_pair(p_rgb.x, p_rgb.y, h0, m0, l0);
      split3_pair(p_rgb.z, p_rgb.w, h1, m1, l1);
      __bf16* row = &s_f[b3][q][DP];
      *reinterpret_cast<uint2*>(row) = make_uint2(h0, h1);
      *reinterpret_cast<uint2*>(row + 4) = make_uint2(m0, m1);
      *reinterpret_cast<uint2*>(row + 8) = make_uint2(l0, l1);
    }
#pragma unroll
    for (int j = 0; j < FI; ++j) {
      const int e = q + j * NT;
      if (e < kNB * FQ) {
        const int i = e / FQ;
        const int c = (e % FQ) * 4;
        // the stored bf16 bits go to LDS unchanged (channel c in the low half)
        *reinterpret_cast<uint2*>(&s_f[b3][i][c]) = i < nb ? fv[j].v : make_uint2(0u, 0u);
      }
    }
  };

  float colv[2][4];   // accumulators: colour and depth of pixels lane (< 32) of each 32-pixel block
  if (walker) {
    // ================= walkers =================
    // T < 0 marks a finished pixel (|T| is its final transmittance), and a
    // skipped pair carries alpha 0: a finished pixel or a skipped pair then
    // leaves T, the colour and the weights unchanged with no per-pair mask
    // logic, so the front-to-back chain is a few dependent VALU operations.
    float T = inside ? 1.0f : -1.0f;
    int last = 0;
    for (int kk = 0;; ++kk) {
      const int k = __builtin_amdgcn_readfirstlane(kk);   // scalar: keeps the barrier loop uniform
      const int alive = __syncthreads_count(T > 0.f);
      const bool more = k < nbatch && alive > 0;
      if (!more) break;
      const int b2 = k & 1;
      const int pos0 = k * kNB;
      const bool wave_live = __ballot(T > 0.f) != 0ull;
#pragma unroll
      for (int s = 0; s < kNB / 16; ++s) {
        float wv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) wv[i] = 0.f;
        int lrel = 0;                                  // 1 + last pair of the 16 with a weight
        if (wave_live) {
          // alpha of the 16 pairs, independent of each other (padding
          // entries of the batch carry opacity 0 and are skipped here)
          float al[16], om[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int i = 16 * s + u;
            const float2 m = s_xy[b2][i];
            const float4 co = s_co[b2][i];            // scaled conic, opacity
            const float dx = fpx - m.x, dy = fpy - m.y;
            const float qs = scaled_q(co, dx, dy);
            const bool inb = in_box(pp, s_box[b2][i]);
            const float alpha = fminf(kAlphaMax, co.w * __builtin_amdgcn_exp2f(qs));
            al[u] = (inb & (qs >= s_tg[b2][i])) ? alpha : 0.f;
            om[u] = 1.0f - al[u];
          }
          // front-to-back transmittance chain
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            // T (1 - alpha) as every forward kernel forms it, so that the stop
            // decisions, final_T and n_contrib are the same in all of them
            const float Tn = T * om[u];
            const bool stop = Tn < kTStop;             // also true once T < 0
            const float w = stop ? 0.f : al[u] * T;
            T = stop ? -fabsf(T) : Tn;
            wv[u] = w;
            lrel = w != 0.f ? u + 1 : lrel;
          }
          if (lrel > 0) last = pos0 + 16 * s + lrel;
        }
        const bool wany = __ballot(lrel > 0) != 0ull;
        if (lane == 0) s_any[b2][wave][s] = wany ? 1 : 0;
        if (wany) {
#pragma unroll
          for (int i = 0; i < 16; i += 4)
            *reinterpret_cast<float4*>(&s_w[b2][q][16 * s + i]) = make_float4(wv[i], wv[i + 1], wv[i + 2], wv[i + 3]);
        }
      }
    }
    T = fabsf(T);
    s_T[q] = T;
    if (inside) {
      const int64_t p = (int64_t)py * a.W + px;
      a.out_T[p] = T;
      a.out_n[p] = last;
    }
    if (last > 0) atomicMax(&s_maxlast, last);
  } else {
    // ================= accumulators =================
    // acc[c][pb]: channels 32 c.. x pixels 64 wave + 32 pb.. (c = CB: colour)
    f32x16 acc[CB + 1][2];
#pragma unroll
    for (int c = 0; c <= CB; ++c) acc[c][0] = acc[c][1] = f32x16{};
    // unused columns of the colour block: zero once (the staging writes 12)
    for (int e = q; e < 3 * kNB * 5; e += NT)
      *reinterpret_cast<uint2*>(&s_f[e / (5 * kNB)][(e / 5) % kNB][DP + 12 + 4 * (e % 5)]) = make_uint2(0u, 0u);
    load_ids(0);
    load_data();
    load_ids(1);
    stage(0);
    load_data();
    load_ids(2);
    for (int kk = 0;; ++kk) {
      // the batch counter is read back as a scalar so that the compiler keeps
      // the loop (and its barrier) uniform
      const int k = __builtin_amdgcn_readfirstlane(kk);
      const int alive = __syncthreads_count(0);
      const bool more = k < nbatch && alive > 0;
      if (k >= 1) {
        // contraction of batch k-1: Z (channels x pixels) += F^T W
        const int b2 = (k - 1) & 1, b3 = (k - 1) % 3;
#pragma unroll
        for (int s = 0; s < kNB / 16; ++s) {
          // the flag is wave-uniform: a scalar branch keeps the barrier loop uniform
          if (!__builtin_amdgcn_readfirstlane(s_any[b2][wave][s])) continue;
          bf16x8 fa[CB + 1];
#pragma unroll
          for (int c = 0; c <= CB; ++c) fa[c] = load_a_tr<FROW>(&s_f[b3][0][0], 16 * s, 32 * c, lane);
#pragma unroll
          for (int pb = 0; pb < 2; ++pb) {
            const float* wr = &s_w[b2][64 * wave + 32 * pb + (lane & 31)][16 * s + 8 * (lane >> 5)];
            const float4 w0 = *reinterpret_cast<const float4*>(wr);
            const float4 w1 = *reinterpret_cast<const float4*>(wr + 4);
            const float wf[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
            u32x4 bw[3];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              uint32_t h, m, l;
              split3_pair(wf[2 * j], wf[2 * j + 1], h, m, l);
              bw[0][j] = h;
              bw[1][j] = m;
              bw[2][j] = l;
            }
#pragma unroll
            for (int c = 0; c <= CB; ++c) {
              f32x16 z = acc[c][pb];
#pragma unroll
              for (int t = 0; t < 3; ++t)
                z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[c], __builtin_bit_cast(bf16x8, bw[t]), z, 0, 0, 0);
              acc[c][pb] = z;
            }
          }
        }
      }
      if (!more) break;
      if (k + 1 < nbatch) {
        stage(k + 1);
        load_data();
        load_ids(k + 3);
      }
    }
    // feature image: accumulator row = channel, column = pixel
    const int64_t HW = (int64_t)a.W * a.H;
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      const int lpo = 64 * wave + 32 * pb + (lane & 31);
      const int ox = (tile % a.tiles_x) * a.tile_w + lpo % a.tile_w;
      const int oy = (tile / a.tiles_x) * tile_h + lpo / a.tile_w;
      if (ox < a.W && oy < a.H) {
        const int64_t p = (int64_t)oy * a.W + ox;
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int ch = 32 * c + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            if (ch < a.D) a.out_feat[ch * HW + p] = acc[c][pb][v];
          }
      }
    }
    // colour block: rows 0-3 (c_hi parts) sit in v 0-3 of lanes 0-31, rows
    // 4-7 (c_mid) in v 0-3 of lanes 32-63, rows 8-11 (c_lo) in v 4-7 of lanes 0-31
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const float mid = __shfl_xor(acc[CB][pb][n], 32, 64);
        colv[pb][n] = acc[CB][pb][n] + (mid + acc[CB][pb][4 + n]);
      }
  }
  // per-tile walk length (used by the backward to size its partial rows);
  // the walkers' final transmittance is in s_T
  __syncthreads();
  if (threadIdx.x == 0) {
    a.tile_maxlast[tile] = (uint32_t)s_maxlast;
    if (s_maxlast > 0) atomicAdd(&a.report[kRepRows], (unsigned long long)s_maxlast);
  }
  if (!walker) {
    // colour image (the background behind the final transmittance)
    const int64_t HW = (int64_t)a.W * a.H;
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      const float* col = colv[pb];
      const int lpo = 64 * wave + 32 * pb + (lane & 31);
      const int ox = (tile % a.tiles_x) * a.tile_w + lpo % a.tile_w;
      const int oy = (tile / a.tiles_x) * tile_h + lpo / a.tile_w;
      if (lane < 32 && ox < a.W && oy < a.H) {
        const int64_t p = (int64_t)oy * a.W + ox;
        const float Tf = s_T[lpo];
        a.out_rgb[p] = __builtin_fmaf(Tf, a.bg[0], col[0]);
        a.out_rgb[HW + p] = __builtin_fmaf(Tf, a.bg[1], col[1]);
        a.out_rgb[2 * HW + p] = __builtin_fmaf(Tf, a.bg[2], col[2]);
        if (a.out_depth) a.out_depth[p] = col[3];
      }
    }
  }
}

template <int DP, int NT>
__global__ __launch_bounds__(2 * NT) void composite_fwd_ws_kernel(MfmaArgs a) {
  fwd_ws_tile<DP, NT>(a, fwd_tile(a));
}

// Persistent form over many frames: each workgroup takes (frame, tile) items
// from a queue sorted longest first until the queue is empty.
template <int DP, int NT>
__global__ __launch_bounds__(2 * NT) void composite_fwd_ws_persistent(const MfmaArgs* __restrict__ args,
                                                                      TileQueue tq) {
  __shared__ uint32_t s_item;
  const uint32_t n_items = __builtin_amdgcn_readfirstlane(*tq.count);
  // items are fetched at the end of the loop (a divergent fetch at its head
  // has been lowered into a nested loop with a per-lane exit); the second
  // barrier keeps thread 0 from overwriting s_item before everyone read it
  if (threadIdx.x == 0) s_item = atomicAdd(tq.head, 1u);
  __syncthreads();
  uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
  __syncthreads();
  while (it < n_items) {
    const uint2 item = tq.items[it];
    const MfmaArgs a = args[item.x];   // a private copy of the frame record (see the backward)
    fwd_ws_tile<DP, NT>(a, (int)item.y);
    if (threadIdx.x == 0) s_item = atomicAdd(tq.head, 1u);
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
  }
}

template <int DP, typename FT>
hipError_t launch_nt(int nt, const MfmaArgs& a, int tiles, bool ws, hipStream_t s) {
  // wave-specialized kernel for BF16 features up to 128 channels
  if constexpr (std::is_same<FT, uint16_t>::value && DP <= 128) {
    if (ws) {
      switch (nt) {
        case 64: hipLaunchKernelGGL((composite_fwd_ws_kernel<DP, 64>), dim3(tiles), dim3(128), 0, s, a); break;
        case 128: hipLaunchKernelGGL((composite_fwd_ws_kernel<DP, 128>), dim3(tiles), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((composite_fwd_ws_kernel<DP, 256>), dim3(tiles), dim3(512), 0, s, a); break;
      }
      return hipGetLastError();
    }
  }
  switch (nt) {
    case 64: hipLaunchKernelGGL((composite_fwd_mfma_kernel<DP, FT, 64>), dim3(tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL((composite_fwd_mfma_kernel<DP, FT, 128>), dim3(tiles), dim3(128), 0, s, a); break;
    default: hipLaunchKernelGGL((composite_fwd_mfma_kernel<DP, FT, 256>), dim3(tiles), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

template <typename FT>
hipError_t dispatch(int D, int nt, const MfmaArgs& a, int tiles, bool ws, hipStream_t s) {
  if (D <= 32) return launch_nt<32, FT>(nt, a, tiles, ws, s);
  if (D <= 64) return launch_nt<64, FT>(nt, a, tiles, ws, s);
  if (D <= 128) return launch_nt<128, FT>(nt, a, tiles, ws, s);
  return launch_nt<256, FT>(nt, a, tiles, ws, s);
}

}  // namespace

static MfmaArgs make_args(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                          const fe_images* out) {
  MfmaArgs a{};
  a.ranges = v.ranges;
  a.gauss = v.gauss;
  a.xy = v.xy;
  a.conic_o = v.conic_o;
  a.rgb = v.rgb;
  a.box = v.box;
  a.feat = g->feat;
  a.out_rgb = out->rgb;
  a.out_feat = out->feat;
  a.out_T = out->final_T;
  a.out_n = out->n_contrib;
  a.out_depth = out->depth;
  a.tile_maxlast = v.tile_maxlast;
  a.order = v.n > 0 ? v.tile_order : nullptr;   // the binning writes it whenever there are Gaussians
  a.report = v.report;
  for (int k = 0; k < 3; ++k) a.bg[k] = cfg->bg_rgb[k];
  a.W = cam->width;
  a.H = cam->height;
  a.tile_w = cfg->tile_w;
  a.tiles_x = v.tiles_x;
  a.D = cfg->feat_dim;
  const size_t esz = cfg->feat_dtype == FE_BF16 ? 2 : 4;
  a.vec = cfg->feat_dim % 4 == 0 && reinterpret_cast<uintptr_t>(g->feat) % (4 * esz) == 0;
  return a;
}

hipError_t launch_composite_fwd_mfma(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                     const StateView& v, const fe_images* out, hipStream_t s) {
  if (v.tiles == 0) return hipSuccess;
  const MfmaArgs a = make_args(cfg, cam, g, v, out);
  const int nt = cfg->tile_w * cfg->tile_h;
  const bool ws = forward_wave_specialized(cfg);
  return cfg->feat_dtype == FE_BF16 ? dispatch<uint16_t>(cfg->feat_dim, nt, a, v.tiles, ws, s)
                                    : dispatch<float>(cfg->feat_dim, nt, a, v.tiles, ws, s);
}

// Wave-specialized forward (2 NT threads per tile) for BF16 features up to
// 128 channels, unless threads_per_tile asks for one thread per pixel.
bool forward_wave_specialized(const fe_config* cfg) {
  return cfg->feat_dtype == FE_BF16 && cfg->feat_dim <= 128 && cfg->threads_per_tile != cfg->tile_w * cfg->tile_h;
}

// ---- persistent multi-frame form (wave-specialized kernels only) ----
bool composite_persistent_supported(const fe_config* cfg) {
  return cfg->variant != FE_VARIANT_VALU && forward_wave_specialized(cfg);
}

size_t composite_fwd_record_bytes() { return sizeof(MfmaArgs); }

void composite_fwd_record(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                          const fe_images* out, void* dst) {
  const MfmaArgs a = make_args(cfg, cam, g, v, out);
  std::memcpy(dst, &a, sizeof(a));
}

template <int DP, int NT>
static int fwd_grid() {
  int per_cu = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, composite_fwd_ws_persistent<DP, NT>, 2 * NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

template <int DP>
static int fwd_grid_nt(int nt) {
  return nt == 64 ? fwd_grid<DP, 64>() : nt == 128 ? fwd_grid<DP, 128>() : fwd_grid<DP, 256>();
}

int composite_fwd_persistent_grid(const fe_config* cfg) {
  const int nt = cfg->tile_w * cfg->tile_h, D = cfg->feat_dim;
  return D <= 32 ? fwd_grid_nt<32>(nt) : D <= 64 ? fwd_grid_nt<64>(nt) : fwd_grid_nt<128>(nt);
}

template <int DP>
static hipError_t fwd_persistent_nt(int nt, const MfmaArgs* r, const TileQueue& q, int grid, hipStream_t s) {
  switch (nt) {
    case 64: hipLaunchKernelGGL((composite_fwd_ws_persistent<DP, 64>), dim3(grid), dim3(128), 0, s, r, q); break;
    case 128: hipLaunchKernelGGL((composite_fwd_ws_persistent<DP, 128>), dim3(grid), dim3(256), 0, s, r, q); break;
    default: hipLaunchKernelGGL((composite_fwd_ws_persistent<DP, 256>), dim3(grid), dim3(512), 0, s, r, q); break;
  }
  return hipGetLastError();
}

hipError_t launch_composite_fwd_persistent(const fe_config* cfg, const void* records, const TileQueue& q,
                                           int grid, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  const int nt = cfg->tile_w * cfg->tile_h, D = cfg->feat_dim;
  const MfmaArgs* r = static_cast<const MfmaArgs*>(records);
  return D <= 32 ? fwd_persistent_nt<32>(nt, r, q, grid, s)
                 : D <= 64 ? fwd_persistent_nt<64>(nt, r, q, grid, s) : fwd_persistent_nt<128>(nt, r, q, grid, s);
}

}  // namespace fe
