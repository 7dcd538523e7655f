// Backward of the per-tile blending with both D-channel contractions on the
// matrix cores, and the per-Gaussian reduction of the tiles' partial
// gradients.
//
// For a tile and a batch of NB Gaussians (walked back to front), with the
// upstream feature gradient G [pixels x D] of the tile:
//   S  = F G^T        s_i(p) = g(p) . f_i           (needed before the walk)
//   walk per pixel    T_i = T_{i+1} / (1 - alpha_i), w_i = alpha_i T_i,
//                     dL/dalpha_i = T_i s_i - (sum_{j>i} w_j s_j + T_f s_bg) / (1 - alpha_i)
//   dF = W^T G        dL/df_i = sum_p w_i(p) g(p)
// Both contractions run as v_mfma_f32_32x32x16_bf16 with every float32
// operand split into bf16 parts (G and W into hi + lo, float32 features into
// hi + mid): the products kept are those of combined order <= 1, so each
// result carries about 16 significant bits before the float32 accumulation.
//
// Partial results are not added into the outputs with device-wide atomics
// (the eight XCDs keep no common cache, so those run at memory speed).  Each
// (tile, list position) walked writes one row [dL/df (D), dL/d(u, v, A, B, C,
// opacity, r, g, b, depth)] into a compact buffer; rows of a tile start at an
// exclusive scan of the tiles' walk lengths.  A second kernel sums, per
// Gaussian, the rows of the tiles it was walked in, found through the
// emit-position -> sorted-position map written by the tile sort.
#include "fe_common.h"

#include <cstring>
#include <type_traits>

#pragma clang fp contract(off)

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kNB = 32;

struct BwdArgs {
  const uint2* ranges;
  const uint32_t* gauss;
  const float2* xy;
  const float4* conic_o;
  const float4* rgb;
  const short4* box;
  const void* feat;
  const float* final_T;
  const int32_t* n_contrib;
  const float* d_rgb;
  const float* d_feat;
  const float* d_depth;      // [H][W] or null (no depth gradient)
  const uint32_t* tile_maxlast;
  const uint32_t* row_base;
  const uint32_t* order;        // [tiles] launch order of the per-frame kernels (longest walks first)
  float* rows;
  int64_t row_cap;
  uint32_t* rowidx;          // [cap] 1 + row of each walked pair, by emit position (0: not walked)
  const uint32_t* epos;      // [cap] emit position of each sorted pair
  unsigned long long* report;
  float bg[3];
  int32_t W, H, tile_w, tiles_x, D, RS;
  bool vec;                  // feature rows allow aligned 4-channel vector loads
};

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// sum of the 16 lanes of each DPP row, complete in lanes 15, 31, 47 and 63
__device__ __forceinline__ float row_sum16(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
  return v;
}

template <int DP, typename FT, int NT, bool kLeaveEmpty>
__device__ __forceinline__ void bwd_mfma_tile(const BwdArgs& a, const int tile) {
  constexpr bool F32 = std::is_same<FT, float>::value;
  constexpr int NPF = F32 ? 2 : 1;     // feature planes in GEMM1 (hi, mid)
  constexpr int CB = DP / 32;
  constexpr int KS1 = DP / 16;
  constexpr int NW = NT / 64;
  constexpr int FROW = DP + 8;         // padded LDS rows (bank spread)
  constexpr int WROW = 64 + 8;
  constexpr int DFROW = DP + 8;        // rows 4 apart land 32 banks apart
  constexpr int GROW = NT + 1;
  // GEMM2 work is split into CB units per wave, a unit being one 32-channel
  // block over one wave's 64 pixels (a pixel chunk).  With CB >= NW a wave
  // owns whole channel blocks (all chunks) and stores its sums directly;
  // otherwise KSPL waves share a block and leave partial sums in LDS.
  constexpr int KSPL = NW > CB ? NW / CB : 1;
  // The upstream-gradient slice is needed only before the first batch; the
  // weight transposes and the partial dF sums only after it: they share one
  // LDS region.
  constexpr size_t kGBytes = sizeof(float) * 32 * GROW;
  constexpr size_t kWBytes = sizeof(__bf16) * NW * 2 * kNB * WROW;
  constexpr size_t kDFBytes = KSPL > 1 ? sizeof(float) * KSPL * kNB * DFROW : 0;
  constexpr size_t kShared = kGBytes > kWBytes + kDFBytes ? kGBytes : kWBytes + kDFBytes;
  __shared__ float2 s_xy[kNB];
  __shared__ float4 s_co[kNB];
  __shared__ float s_tg[kNB];
  __shared__ float4 s_rgb[kNB];
  __shared__ int4 s_box[kNB];
  __shared__ __attribute__((aligned(16))) __bf16 s_f[NPF][kNB][FROW];
  __shared__ float s_red[12][kNB];
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[kShared];
  float (*s_g)[GROW] = reinterpret_cast<float (*)[GROW]>(s_raw);
  __bf16 (*s_w)[2][kNB][WROW] = reinterpret_cast<__bf16 (*)[2][kNB][WROW]>(s_raw);
  float (*s_df)[kNB][DFROW] = reinterpret_cast<float (*)[kNB][DFROW]>(s_raw + kWBytes);   // [KSPL]
  __shared__ int s_live[NW];
  __shared__ float s_gr[4][NT];                              // upstream colour and depth gradient of the tile
  // MFMA B operands of the colour sums, per wave and 32-pixel k step: lane l
  // holds colour l % 16 (zero from 3 on) at pixels 8 (l / 16) + 0..7, hi / lo
  __shared__ bf16x8 s_grb[NW][2][2][64];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // GEMM2 unit u of this wave: channel block and pixel chunk
  auto unit_cb = [&](int u) { return CB >= NW ? wave + NW * (u / NW) : wave % CB; };
  auto unit_chunk = [&](int u) { return CB >= NW ? u % NW : (wave / CB) * CB + u; };
  const int tile_h = NT / a.tile_w;
  const int tx0 = (tile % a.tiles_x) * a.tile_w;
  const int ty0 = (tile / a.tiles_x) * tile_h;
  const int px = tx0 + (int)threadIdx.x % a.tile_w;
  const int py = ty0 + (int)threadIdx.x / a.tile_w;
  const bool inside = (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const int64_t HW = (int64_t)a.W * a.H;
  // The upstream feature gradient of this thread's pixel is loaded first, GS
  // 32-channel slices at once (all of them for D <= 128), so that its latency
  // overlaps the tile's list lookups and the first batch's loads.
  constexpr int GS = CB < (F32 ? 2 : 4) ? CB : (F32 ? 2 : 4);
  float gv[GS][32];
  auto load_g = [&](int cb, float* dst) {
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int ch = 32 * cb + c;
      dst[c] = (inside && ch < a.D) ? a.d_feat[ch * HW + (int64_t)py * a.W + px] : 0.f;
    }
  };
#pragma unroll
  for (int cb = 0; cb < GS; ++cb) load_g(cb, gv[cb]);
  const uint2 rg = uniform_u2(a.ranges[tile]);
  const int walk_all = __builtin_amdgcn_readfirstlane((int)min(a.tile_maxlast[tile], rg.y - rg.x));
  const int64_t row0 = uniform_i64(a.row_base[tile]);
  const bool overflow = __builtin_amdgcn_readfirstlane((int)(row0 + walk_all > a.row_cap));
  if (overflow && threadIdx.x == 0) a.report[kRepBwdStatus] = (unsigned long long)FE_ERR_ROW_OVERFLOW;
  // nothing of an overflowing tile can be stored: it is walked as empty.  The
  // per-tile kernel leaves empty tiles at once; inside the persistent loop the
  // tile keeps a single exit (empty tiles are not queued there).
  const int walk = __builtin_amdgcn_readfirstlane(overflow ? 0 : walk_all);
  if constexpr (kLeaveEmpty) {
    if (walk == 0) return;
  }

  // Batches are walked back to front: batch k covers list positions
  // [r1 - kNB, r1) clipped at 0, r1 = walk - k kNB.  Staging is
  // software-pipelined: the Gaussian ids of batch k+2 and the records /
  // feature rows of batch k+1 are loaded into registers while batch k is
  // processed.
  constexpr int FQ = DP / 4;                               // 4-channel groups per row
  constexpr int FI = (kNB * FQ + NT - 1) / NT;             // feature groups per thread
  uint32_t id_n;                                          // Gaussian (tid % kNB) of the next batch
  uint32_t ep_n = 0, ep_data = 0, ep_cur = 0;             // its emit position (row index slot), pipelined
  FeatGroup<FT> fv[FI];
  float2 p_xy = make_float2(0.f, 0.f);
  float4 p_co = make_float4(0.f, 0.f, 0.f, 0.f), p_rgb = p_co;
  short4 p_box = make_short4(1, 1, 0, 0);
  // Staging thread t works on Gaussian t % kNB of a batch (feature groups
  // t / kNB + k NT / kNB), so it needs one id.
  const int si = (int)threadIdx.x % kNB;
  auto load_ids = [&](int r1) {
    const int r0 = r1 > kNB ? r1 - kNB : 0;
    const bool ok = r0 + si < r1;
    id_n = ok ? a.gauss[rg.x + r0 + si] : 0xFFFFFFFFu;
    ep_n = (ok && (int)threadIdx.x < kNB) ? a.epos[rg.x + r0 + si] : 0u;
  };
  auto load_data = [&]() {
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int e = threadIdx.x + k * NT;
      const int c = (e / kNB) * 4;
      fv[k].clear();
      if (e < kNB * FQ && id_n != 0xFFFFFFFFu && c < a.D) fv[k].load(a.feat, (int64_t)id_n * a.D, c, a.D, a.vec);
    }
    ep_data = ep_n;
    if ((int)threadIdx.x < kNB && id_n != 0xFFFFFFFFu) {
      const uint32_t g = id_n;
      p_xy = a.xy[g];
      p_co = a.conic_o[g];
      p_rgb = a.rgb[g];
      p_box = a.box[g];
    }
  };
  load_ids(walk);

  // ---- per-pixel state ----
  float gr0 = 0.f, gr1 = 0.f, gr2 = 0.f, gr3 = 0.f;   // upstream colour and depth gradient
  float T = 1.0f;
  int last = 0;
  if (inside) {
    const int64_t p = (int64_t)py * a.W + px;
    gr0 = a.d_rgb[p];
    gr1 = a.d_rgb[HW + p];
    gr2 = a.d_rgb[2 * HW + p];
    gr3 = a.d_depth ? a.d_depth[p] : 0.f;
    T = a.final_T[p];
    last = a.n_contrib[p];
  }

  // ---- upstream feature gradient of the wave's 64 pixels, in both operand layouts,
  //      staged through LDS one 32-channel slice at a time ----
  bf16x8 g1[2][KS1][2];   // GEMM1 B: [pixel block][k step][hi, lo]; lane: pixel l%32, channels 8(l/32)+j
  bf16x8 g2[CB][4][2];    // GEMM2 B: [unit][k step][hi, lo]; lane: channel l%32, pixels 8(l/32)+j of the chunk
  s_gr[0][threadIdx.x] = gr0;
  s_gr[1][threadIdx.x] = gr1;
  s_gr[2][threadIdx.x] = gr2;
  s_gr[3][threadIdx.x] = gr3;
  load_data();
  load_ids(walk - kNB);
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    if (cb > 0) __syncthreads();
#pragma unroll
    for (int c = 0; c < 32; ++c) s_g[c][threadIdx.x] = gv[cb % GS][c];
    if (cb + GS < CB) load_g(cb + GS, gv[cb % GS]);
    __syncthreads();
#pragma unroll
    for (int pb = 0; pb < 2; ++pb)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 h, l;
          split2(s_g[16 * s2 + 8 * (lane >> 5) + j][64 * wave + 32 * pb + (lane & 31)], h, l);
          g1[pb][2 * cb + s2][0][j] = h;
          g1[pb][2 * cb + s2][1][j] = l;
        }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      if (unit_cb(u) != cb) continue;
      const int q0 = 64 * unit_chunk(u) + 8 * (lane >> 5);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 h, l;
          split2(s_g[lane & 31][q0 + 16 * s + j], h, l);
          g2[u][s][0][j] = h;
          g2[u][s][1][j] = l;
        }
    }
  }
  float acc = T * ((gr0 * a.bg[0] + gr1 * a.bg[1]) + gr2 * a.bg[2]);
  int wave_last = last;
  for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));

  {
    const int n = lane & 15;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = n < 4 ? s_gr[n < 4 ? n : 0][64 * wave + 32 * ks + 8 * (lane >> 4) + j] : 0.f;
        __bf16 xh, xl;
        split2(x, xh, xl);
        h[j] = xh;
        l[j] = xl;
      }
      s_grb[wave][ks][0][lane] = h;
      s_grb[wave][ks][1][lane] = l;
    }
  }
  __syncthreads();   // the gradient slices are consumed; the region now holds W and dF

  for (int r0 = walk;; r0 -= kNB) {
    const int r1 = __builtin_amdgcn_readfirstlane(r0);   // scalar: keeps the barrier loop uniform
    if (r1 <= 0) break;
    const int pos0 = r1 > kNB ? r1 - kNB : 0;
    const int nb = r1 - pos0;
    __syncthreads();
    // ---- stage the batch from registers; clear the per-Gaussian sums ----
    ep_cur = ep_data;
    for (int e = threadIdx.x; e < 12 * kNB; e += NT) (&s_red[0][0])[e] = 0.f;
    if ((int)threadIdx.x < kNB) {
      s_xy[threadIdx.x] = p_xy;
      s_co[threadIdx.x] = p_co;
      s_tg[threadIdx.x] = blend_cut(p_co.w);
      s_rgb[threadIdx.x] = p_rgb;
      s_box[threadIdx.x] = make_int4(p_box.x, p_box.y, p_box.z, p_box.w);
    }
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < kNB * FQ) {
        const int i = e % kNB;
        const int c = (e / kNB) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = i < nb ? fv[k].get(j) : 0.f;
          if constexpr (F32) {
            __bf16 h, m;
            split2(v, h, m);
            s_f[0][i][c + j] = h;
            s_f[1][i][c + j] = m;
          } else {
            s_f[0][i][c + j] = (__bf16)v;   // exact: the value is a bf16
          }
        }
      }
    }
    // ---- issue the next batches' loads ----
    load_data();
    load_ids(r1 - 2 * kNB);
    __syncthreads();
    const bool live = wave_last > pos0;
    if (lane == 0) s_live[wave] = live ? 1 : 0;
    if (live) {
      // ---- GEMM1: S^T (Gaussians x pixels) = F (Gaussians x D) . G^T (D x pixels) ----
      f32x16 s1[2] = {f32x16{}, f32x16{}};
#pragma unroll
      for (int s = 0; s < KS1; ++s) {
        const int kc = 16 * s + 8 * (lane >> 5);
        bf16x8 fa[NPF];
#pragma unroll
        for (int p = 0; p < NPF; ++p) fa[p] = *reinterpret_cast<const bf16x8*>(&s_f[p][lane & 31][kc]);
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
          s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], g1[pb][s][0], s1[pb], 0, 0, 0);
          s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], g1[pb][s][1], s1[pb], 0, 0, 0);
          if constexpr (F32) s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], g1[pb][s][0], s1[pb], 0, 0, 0);
        }
      }
      // this lane's pixel gets s_i for all 32 Gaussians
      float S[kNB];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(s1[0][v]), __float_as_uint(s1[1][v]),
                                                        false, false);
        S[8 * (v >> 2) + (v & 3)] = __uint_as_float(r[0]);
        S[8 * (v >> 2) + 4 + (v & 3)] = __uint_as_float(r[1]);
      }
      // ---- back-to-front walk of this lane's pixel, in groups of 8 ----
      // Branch-free so that the independent per-pair work of a group
      // interleaves; only the transmittance / suffix recurrences are serial.
      constexpr int GR = 8;
#pragma unroll
      for (int gi = kNB / GR - 1; gi >= 0; --gi) {
        float al[GR], Gv[GR], dxv[GR], dyv[GR];
        bool ct[GR], unc[GR];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int i = gi * GR + u;
          const float2 m = s_xy[i];
          const float4 co = s_co[i];
          const int4 b = s_box[i];
          const float dx = fpx - m.x, dy = fpy - m.y;
          const float qs = scaled_q(scale_conic(co), dx, dy);
          const bool inb = (px >= b.x) & (px <= b.z) & (py >= b.y) & (py <= b.w);
          const float G = __builtin_amdgcn_exp2f(qs);
          const float opG = co.w * G;
          const float alpha = fminf(kAlphaMax, opG);
          ct[u] = (i < nb) & (pos0 + i < last) & inb & (qs >= s_tg[i]);
          unc[u] = opG <= kAlphaMax;   // alpha not clamped: it depends on opacity and q
          al[u] = alpha;
          Gv[u] = G;
          dxv[u] = dx;
          dyv[u] = dy;
        }
        // X = G dL/dalpha for blended, unclamped pairs: every projected-space
        // gradient of the pair is X times a factor of the Gaussian (opacity,
        // conic) and of (dx, dy), applied after the pixel sums
        float wg[GR], xg[GR];
#pragma unroll
        for (int u = GR - 1; u >= 0; --u) {
          const int i = gi * GR + u;
          const float4 c = s_rgb[i];
          const float sv = S[i] + (((gr0 * c.x + gr1 * c.y) + gr2 * c.z) + gr3 * c.w);
          const float inv_om = __builtin_amdgcn_rcpf(1.0f - al[u]);
          const float Tn = T * inv_om;
          const float w = al[u] * Tn;
          const float da = Tn * sv - acc * inv_om;
          T = ct[u] ? Tn : T;
          acc = ct[u] ? __builtin_fmaf(w, sv, acc) : acc;
          wg[u] = ct[u] ? w : 0.f;
          xg[u] = (ct[u] & unc[u]) ? Gv[u] * da : 0.f;
        }
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          // W^T of the wave into LDS (Gaussian-major, pixels contiguous)
          __bf16 h, l;
          split2(wg[u], h, l);
          s_w[wave][0][gi * GR + u][lane] = h;
          s_w[wave][1][gi * GR + u][lane] = l;
        }
        // Sums over the wave's 64 pixels of [X dx, X dy, X dx^2, X dx dy,
        // X dy^2, X] for two Gaussians at a time (12 values): halve with
        // the 32-lane swap (lanes >= 32 keep the second Gaussian), then the
        // 16-lane swap (odd rows keep values 3..5), then a 16-lane row sum;
        // lane 15 of row r holds Gaussian u0 + r / 2, values 3 (r % 2) + 0..2.
        // A pair that no pixel of the wave blends adds nothing.
        float red[GR / 2][3];
        bool anyp[GR / 2];
#pragma unroll
        for (int up = 0; up < GR / 2; ++up) {
          const int u0 = 2 * up;
          anyp[up] = __ballot(ct[u0] | ct[u0 + 1]) != 0ull;
          red[up][0] = red[up][1] = red[up][2] = 0.f;
          if (!anyp[up]) continue;
          float vals[12];
#pragma unroll
          for (int hf = 0; hf < 2; ++hf) {
            const int u = u0 + hf;
            const float X = xg[u];
            const float Xdx = X * dxv[u], Xdy = X * dyv[u];
            float* v = vals + 6 * hf;
            v[0] = Xdx;
            v[1] = Xdy;
            v[2] = Xdx * dxv[u];
            v[3] = Xdx * dyv[u];
            v[4] = Xdy * dyv[u];
            v[5] = X;
          }
          float h6[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(vals[k]), __float_as_uint(vals[k + 6]),
                                                            false, false);
            h6[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(h6[k]), __float_as_uint(h6[k + 3]),
                                                            false, false);
            red[up][k] = row_sum16(__uint_as_float(r[0]) + __uint_as_float(r[1]));
          }
        }
        if ((lane & 15) == 15) {
          const int base = 3 * ((lane >> 4) & 1);
#pragma unroll
          for (int up = 0; up < GR / 2; ++up)
            if (anyp[up])
#pragma unroll
              for (int k = 0; k < 3; ++k) atomicAdd(&s_red[base + k][gi * GR + 2 * up + (lane >> 5)], red[up][k]);
        }
      }
      // ---- colour sums dL/dc_i = sum_p w_i(p) g_rgb(p) of the wave's pixels on the
      //      matrix cores: 16x16x32 MFMAs, A = W^T (16 Gaussians x 32 pixels) from
      //      LDS, B = the tile's upstream colour gradient (columns 0..2) ----
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        f32x4 cs = f32x4{};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const int kp = 32 * ks + 8 * (lane >> 4);
          const bf16x8 wh = *reinterpret_cast<const bf16x8*>(&s_w[wave][0][16 * mb + (lane & 15)][kp]);
          const bf16x8 wl = *reinterpret_cast<const bf16x8*>(&s_w[wave][1][16 * mb + (lane & 15)][kp]);
          const bf16x8 gh = s_grb[wave][ks][0][lane];
          const bf16x8 gl = s_grb[wave][ks][1][lane];
          cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, gh, cs, 0, 0, 0);
          cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, gl, cs, 0, 0, 0);
          cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, gh, cs, 0, 0, 0);
        }
        if ((lane & 15) < 4) {
#pragma unroll
          for (int v = 0; v < 4; ++v) atomicAdd(&s_red[6 + (lane & 15)][16 * mb + 4 * (lane >> 4) + v], cs[v]);
        }
      }
    }
    __syncthreads();
    // ---- GEMM2: dF (Gaussians x D) = W^T (Gaussians x pixels) . G (pixels x D),
    //      one unit per (channel block, pixel chunk); two accumulators so
    //      that two MFMA chains interleave ----
    {
      f32x16 d[2] = {f32x16{}, f32x16{}};
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int chunk = unit_chunk(u);
        if (s_live[chunk]) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int kp = 16 * s + 8 * (lane >> 5);
            const bf16x8 wh = *reinterpret_cast<const bf16x8*>(&s_w[chunk][0][lane & 31][kp]);
            const bf16x8 wl = *reinterpret_cast<const bf16x8*>(&s_w[chunk][1][lane & 31][kp]);
            d[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, g2[u][s][0], d[0], 0, 0, 0);
            d[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, g2[u][s][1], d[1], 0, 0, 0);
            d[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, g2[u][s][0], d[0], 0, 0, 0);
          }
        }
        // a channel block is complete after its last unit of this wave
        const bool block_end = CB >= NW ? (u % NW == NW - 1) : (u == CB - 1);
        if (block_end) {
          const int cb = unit_cb(u);
          const int c = 32 * cb + (lane & 31);
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const float x = d[0][v] + d[1][v];
            if constexpr (KSPL == 1) {
              if (i < nb && c < a.D) a.rows[(row0 + pos0 + i) * a.RS + c] = x;
            } else {
              s_df[wave / CB][i][c] = x;
            }
          }
          d[0] = d[1] = f32x16{};
        }
      }
    }
    if constexpr (KSPL > 1) __syncthreads();   // partial sums of all waves are in LDS
    // ---- rest of the rows of this batch: [dL/df (D) | u v A B C o r g b depth | pad],
    //      one float4 per thread and step.  The walk left the pixel sums S, Sx,
    //      Sy, Sxx, Sxy, Syy of X, X dx, X dy, X dx^2, X dx dy, X dy^2; with the
    //      Gaussian's conic (a, b, c) and opacity o the projected-space
    //      gradients are o (a Sx + b Sy), o (b Sx + c Sy), -o Sxx / 2, -o Sxy,
    //      -o Syy / 2 and S ----
    {
      const int cstart = KSPL > 1 ? 0 : (a.D & ~3);   // columns before cstart were stored by GEMM2
      const int nq = (a.RS - cstart) >> 2;
      for (int t = threadIdx.x; t < nb * nq; t += NT) {
        const int i = t / nq;
        const int c0 = cstart + 4 * (t - i * nq);
        const float4 co = s_co[i];
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = c0 + j;
          float x = 0.f;
          if (c < a.D) {
            if constexpr (KSPL > 1) {
#pragma unroll
              for (int k = 0; k < KSPL; ++k) x += s_df[k][i][c];
            }
          } else {
            switch (c - a.D) {
              case 0: x = co.w * (co.x * s_red[0][i] + co.y * s_red[1][i]); break;
              case 1: x = co.w * (co.y * s_red[0][i] + co.z * s_red[1][i]); break;
              case 2: x = -0.5f * co.w * s_red[2][i]; break;
              case 3: x = -co.w * s_red[3][i]; break;
              case 4: x = -0.5f * co.w * s_red[4][i]; break;
              case 5: x = s_red[5][i]; break;
              case 6: x = s_red[6][i]; break;
              case 7: x = s_red[7][i]; break;
              case 8: x = s_red[8][i]; break;
              case 9: x = s_red[9][i]; break;
              default: break;
            }
          }
          v[j] = x;
        }
        float* dst = &a.rows[(row0 + pos0 + i) * a.RS + c0];
        if (KSPL > 1 || c0 >= a.D) {
          *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
          // group straddling the end of the D columns stored by GEMM2
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (c0 + j >= a.D) dst[j] = v[j];
        }
      }
    }
    if ((int)threadIdx.x < nb) a.rowidx[ep_cur] = (uint32_t)(row0 + pos0 + threadIdx.x + 1);
  }
}

#ifndef WS_GR
#define WS_GR 4
#endif
// Wave-specialized form of the same computation (D <= 128 and at least as
// many 32-channel blocks as 64-pixel chunks).  The block has 2 NT threads:
// NT "walker" threads (one pixel each) run GEMM1, the back-to-front walk and
// the per-Gaussian pixel sums of batch k; NT "contractor" threads run GEMM2
// and write the rows of batch k-1, then stage the records and feature rows of
// batch k+1.  Each role keeps only its own operand layout of the upstream
// feature gradient in registers (128 VGPRs at D = 128), so two waves share
// each SIMD and the latency of one role hides behind the other's issue.  One
// barrier per batch: the weights and liveness are double-buffered, the batch
// records double- (conic/opacity and the sums triple-) buffered.
template <int DP, typename FT, int NT, bool kLeaveEmpty>
__device__ __forceinline__ void bwd_ws_tile(const BwdArgs& a, const int tile) {
  constexpr bool F32 = std::is_same<FT, float>::value;
  constexpr int NPF = F32 ? 2 : 1;
  constexpr int CB = DP / 32;
  constexpr int KS1 = DP / 16;
  constexpr int NW = NT / 64;
  static_assert(CB >= NW, "each contractor wave owns whole channel blocks");
  constexpr int FROW = DP + 8;
  constexpr int WROW = 64 + 8;
  constexpr int GROW = NT + 1;
  constexpr size_t kGBytes = sizeof(float) * 32 * GROW;
  constexpr size_t kWBytes = sizeof(__bf16) * 2 * NW * 2 * kNB * WROW;
  constexpr size_t kShared = kGBytes > kWBytes ? kGBytes : kWBytes;
  __shared__ float2 s_xy[3][kNB];
  __shared__ float4 s_co[3][kNB];
  __shared__ float4 s_cs[3][kNB];             // scaled conic for the walkers
  __shared__ float s_tg[3][kNB];              // blend cut on qs
  __shared__ float4 s_rgb[2][kNB];
  __shared__ uint2 s_box[2][kNB];             // packed (origin, extent)
  __shared__ __attribute__((aligned(16))) __bf16 s_f[2][NPF][kNB][FROW];
  // per walker wave: pixel moments (about the tile centre) and colour sums of
  // each Gaussian of a batch, and the X values of a 16-Gaussian half
  __shared__ float s_mom[2][NW][6][kNB];
  __shared__ float s_col[2][NW][4][kNB];
  // rows padded to 68 floats: the moment pass reads 16 rows at one column,
  // 16 bytes per lane, which then fall in 16 distinct bank groups
  __shared__ float s_xm[NW][16][68];
  __shared__ int s_live[2][NW];
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[kShared];
  float (*s_g)[GROW] = reinterpret_cast<float (*)[GROW]>(s_raw);
  __bf16 (*s_w)[NW][2][kNB][WROW] = reinterpret_cast<__bf16 (*)[NW][2][kNB][WROW]>(s_raw);   // [2]
  __shared__ __attribute__((aligned(16))) float s_gr[4][NT];
  __shared__ bf16x8 s_grb[NW][2][2][64];

  const bool walker = (int)threadIdx.x < NT;
  const int q = walker ? (int)threadIdx.x : (int)threadIdx.x - NT;   // thread index within the role
  const int lane = q & 63;
  const int wave = q >> 6;                                            // wave index within the role
  auto unit_cb = [&](int u) { return wave + NW * (u / NW); };
  auto unit_chunk = [&](int u) { return u % NW; };
  const int tile_h = NT / a.tile_w;
  const int tx0 = (tile % a.tiles_x) * a.tile_w;
  const int ty0 = (tile / a.tiles_x) * tile_h;
  const int px = tx0 + q % a.tile_w;
  const int py = ty0 + q / a.tile_w;
  const bool inside = (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const u16x2 pp = {(unsigned short)px, (unsigned short)py};
  const int64_t HW = (int64_t)a.W * a.H;
  // walkers: the upstream feature gradient of their pixel, all slices issued first
  constexpr int GS = CB < 2 ? CB : 2;
  float gv[GS][32];
  auto load_g = [&](int cb, float* dst) {
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int ch = 32 * cb + c;
      dst[c] = (walker && inside && ch < a.D) ? a.d_feat[ch * HW + (int64_t)py * a.W + px] : 0.f;
    }
  };
  if (walker) {
#pragma unroll
    for (int cb = 0; cb < GS; ++cb) load_g(cb, gv[cb]);
  }
  const uint2 rg = uniform_u2(a.ranges[tile]);
  const int walk_all = __builtin_amdgcn_readfirstlane((int)min(a.tile_maxlast[tile], rg.y - rg.x));
  const int64_t row0 = uniform_i64(a.row_base[tile]);
  const bool overflow = __builtin_amdgcn_readfirstlane((int)(row0 + walk_all > a.row_cap));
  if (overflow && threadIdx.x == 0) a.report[kRepBwdStatus] = (unsigned long long)FE_ERR_ROW_OVERFLOW;
  // nothing of an overflowing tile can be stored: it is walked as empty.  The
  // per-tile kernel leaves empty tiles at once; inside the persistent loop the
  // tile keeps a single exit (empty tiles are not queued there).
  const int walk = __builtin_amdgcn_readfirstlane(overflow ? 0 : walk_all);
  if constexpr (kLeaveEmpty) {
    if (walk == 0) return;
  }
  const int nbatch = __builtin_amdgcn_readfirstlane((walk + kNB - 1) / kNB);
  // batch k covers list positions [pos0(k), pos0(k) + nb(k)), walked back to front
  auto bpos0 = [&](int k) { const int r1 = walk - k * kNB; return r1 > kNB ? r1 - kNB : 0; };
  auto bnb = [&](int k) { return walk - k * kNB - bpos0(k); };

  // ---- contractors: software-pipelined staging (ids of batch k+2, records
  //      and feature rows of batch k+1 in registers while batch k is staged) ----
  constexpr int FQ = DP / 4;
  constexpr int FI = (kNB * FQ + NT - 1) / NT;
  uint32_t id_n = 0xFFFFFFFFu;
  uint32_t ep_n = 0, ep_data = 0, ep_s = 0, ep_w = 0;      // emit position of Gaussian q % kNB, pipelined
  FeatGroup<FT> fv[FI];
  float2 p_xy = make_float2(0.f, 0.f);
  float4 p_co = make_float4(0.f, 0.f, 0.f, 0.f), p_rgb = p_co;
  short4 p_box = make_short4(1, 1, 0, 0);
  const int si = q % kNB;
  auto load_ids = [&](int k) {
    const int r0 = bpos0(k), r1 = r0 + bnb(k);
    const bool ok = k < nbatch && r0 + si < r1;
    id_n = ok ? a.gauss[rg.x + r0 + si] : 0xFFFFFFFFu;
    ep_n = (ok && q < kNB) ? a.epos[rg.x + r0 + si] : 0u;
  };
  auto load_data = [&]() {
#pragma unroll
    for (int k = 0; k < FI; ++k) {
      const int e = q + k * NT;
      const int c = (e / kNB) * 4;
      fv[k].clear();
      if (e < kNB * FQ && id_n != 0xFFFFFFFFu && c < a.D) fv[k].load(a.feat, (int64_t)id_n * a.D, c, a.D, a.vec);
    }
    ep_data = ep_n;
    if (q < kNB && id_n != 0xFFFFFFFFu) {
      p_xy = a.xy[id_n];
      p_co = a.conic_o[id_n];
      p_rgb = a.rgb[id_n];
      p_box = a.box[id_n];
    }
  };
  auto stage = [&](int k) {
    const int b2 = k & 1, b3 = k % 3, nb = bnb(k);
    ep_s = ep_data;
    if (q < kNB) {
      s_xy[b3][q] = p_xy;
      s_co[b3][q] = p_co;
      s_cs[b3][q] = scale_conic(p_co);
      s_tg[b3][q] = blend_cut(p_co.w);
      s_rgb[b2][q] = p_rgb;
      s_box[b2][q] = pack_box(p_box);
    }
#pragma unroll
    for (int k2 = 0; k2 < FI; ++k2) {
      const int e = q + k2 * NT;
      if (e < kNB * FQ) {
        const int i = e % kNB;
        const int c = (e / kNB) * 4;
        if constexpr (F32) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float v = i < nb ? fv[k2].get(j) : 0.f;
            __bf16 h, m;
            split2(v, h, m);
            s_f[b2][0][i][c + j] = h;
            s_f[b2][1][i][c + j] = m;
          }
        } else {
          // the stored bf16 bits go to LDS unchanged, four channels per store
          *reinterpret_cast<uint2*>(&s_f[b2][0][i][c]) = i < nb ? fv[k2].v : make_uint2(0u, 0u);
        }
      }
    }
  };
  if (!walker) {
    load_ids(0);
    load_data();
    load_ids(1);
  }

  // ---- walkers: per-pixel state ----
  float gr0 = 0.f, gr1 = 0.f, gr2 = 0.f, gr3 = 0.f;   // upstream colour and depth gradient
  float T = 1.0f;
  int last = 0;
  if (walker && inside) {
    const int64_t p = (int64_t)py * a.W + px;
    gr0 = a.d_rgb[p];
    gr1 = a.d_rgb[HW + p];
    gr2 = a.d_rgb[2 * HW + p];
    gr3 = a.d_depth ? a.d_depth[p] : 0.f;
    T = a.final_T[p];
    last = a.n_contrib[p];
  }
  if (walker) {
    s_gr[0][q] = gr0;
    s_gr[1][q] = gr1;
    s_gr[2][q] = gr2;
    s_gr[3][q] = gr3;
  }

  // ---- upstream feature gradient into the two operand layouts, one 32-channel
  //      slice at a time through LDS: walkers keep the GEMM1 layout of their
  //      pixels, contractors the GEMM2 layout of their channel blocks ----
  // One register array holds the walker's GEMM1 operand or the contractor's
  // GEMM2 operand (both DP/4 fragments), so the two roles share registers.
  bf16x8 gop[DP / 4];
  auto g1 = [&](int pb, int s, int h) -> bf16x8& { return gop[(pb * KS1 + s) * 2 + h]; };   // pixel block, k step, hi/lo
  auto g2 = [&](int u, int s, int h) -> bf16x8& { return gop[(u * 4 + s) * 2 + h]; };       // unit, k step, hi/lo
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    if (cb > 0) __syncthreads();
    if (walker) {
#pragma unroll
      for (int c = 0; c < 32; ++c) s_g[c][q] = gv[cb % GS][c];
      if (cb + GS < CB) load_g(cb + GS, gv[cb % GS]);
    }
    __syncthreads();
    if (walker) {
#pragma unroll
      for (int pb = 0; pb < 2; ++pb)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            __bf16 h, l;
            split2(s_g[16 * s2 + 8 * (lane >> 5) + j][64 * wave + 32 * pb + (lane & 31)], h, l);
            g1(pb, 2 * cb + s2, 0)[j] = h;
            g1(pb, 2 * cb + s2, 1)[j] = l;
          }
    } else {
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        if (unit_cb(u) != cb) continue;
        const int q0 = 64 * unit_chunk(u) + 8 * (lane >> 5);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            __bf16 h, l;
            split2(s_g[lane & 31][q0 + 16 * s + j], h, l);
            g2(u, s, 0)[j] = h;
            g2(u, s, 1)[j] = l;
          }
      }
    }
  }
  float acc = T * ((gr0 * a.bg[0] + gr1 * a.bg[1]) + gr2 * a.bg[2]);
  int wave_last = last;
  for (int o = 32; o > 0; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));
  if (walker) {
    const int n = lane & 15;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = n < 4 ? s_gr[n < 4 ? n : 0][64 * wave + 32 * ks + 8 * (lane >> 4) + j] : 0.f;
        __bf16 xh, xl;
        split2(x, xh, xl);
        h[j] = xh;
        l[j] = xl;
      }
      s_grb[wave][ks][0][lane] = h;
      s_grb[wave][ks][1][lane] = l;
    }
  } else {
    stage(0);
    load_data();
    load_ids(2);
  }
  __syncthreads();   // gradient slices consumed (the region now holds W), batch 0 staged
  // The colour/depth gradient of each walker pixel as two-part bf16 (hi at
  // .xy, lo at .zw) in the space of s_gr, which no one reads any more: one
  // more k block of the GEMM1 pixel operand (see the colour step there).
  uint4* const s_gc = reinterpret_cast<uint4*>(&s_gr[0][0]);
  if (walker) {
    const f32x2 g01 = {gr0, gr1}, g23 = {gr2, gr3};
    const bf16x2 h01 = __builtin_convertvector(g01, bf16x2), h23 = __builtin_convertvector(g23, bf16x2);
    const bf16x2 l01 = __builtin_convertvector(g01 - __builtin_convertvector(h01, f32x2), bf16x2);
    const bf16x2 l23 = __builtin_convertvector(g23 - __builtin_convertvector(h23, f32x2), bf16x2);
    s_gc[q] = make_uint4(__builtin_bit_cast(uint32_t, h01), __builtin_bit_cast(uint32_t, h23),
                         __builtin_bit_cast(uint32_t, l01), __builtin_bit_cast(uint32_t, l23));
    // each wave reads the entries of its own 64 pixels only
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // The two roles run separate loops with the same number of barriers, so
  // that the registers of one role are not live in the other's loop.
  if (walker) {
    for (int i0 = 0;; ++i0) {
      const int it = __builtin_amdgcn_readfirstlane(i0);   // scalar: keeps the barrier loop uniform
      if (it > nbatch) break;
      if (it < nbatch) {
        // ================= walkers: batch it =================
        const int b2 = it & 1, b3 = it % 3;
        const int pos0 = bpos0(it), nb = bnb(it);
        const bool live = wave_last > pos0;
        if (lane == 0) s_live[b2][wave] = live ? 1 : 0;
        if (live) {
          // GEMM1: S^T (Gaussians x pixels) = F (Gaussians x D) . G^T (D x pixels)
          f32x16 s1[2] = {f32x16{}, f32x16{}};
#pragma unroll
          for (int s = 0; s < KS1; ++s) {
            const int kc = 16 * s + 8 * (lane >> 5);
            bf16x8 fa[NPF];
#pragma unroll
            for (int p = 0; p < NPF; ++p) fa[p] = *reinterpret_cast<const bf16x8*>(&s_f[b2][p][lane & 31][kc]);
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
              s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], g1(pb, s, 0), s1[pb], 0, 0, 0);
              s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0], g1(pb, s, 1), s1[pb], 0, 0, 0);
              if constexpr (F32) s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[1], g1(pb, s, 0), s1[pb], 0, 0, 0);
            }
          }
          // colour step: one more k block adds the colour and depth term
          // c_i . (dL/dC, dL/dD) of every pair to S.  Gaussian row i holds
          // (c_hi, c_lo) at k 0-7 and (c_hi, 0) at k 8-15, the pixel column
          // (g_hi, g_hi) and (g_lo, 0), so the block sums c_hi g_hi + c_lo g_hi
          // + c_hi g_lo, the two-part product without its smallest term.
          {
            const bool khi = lane >= 32;
            const float4 c = s_rgb[b2][lane & 31];
            const f32x2 c01 = {c.x, c.y}, c23 = {c.z, c.w};
            const bf16x2 h01 = __builtin_convertvector(c01, bf16x2), h23 = __builtin_convertvector(c23, bf16x2);
            const bf16x2 l01 = __builtin_convertvector(c01 - __builtin_convertvector(h01, f32x2), bf16x2);
            const bf16x2 l23 = __builtin_convertvector(c23 - __builtin_convertvector(h23, f32x2), bf16x2);
            const uint4 av = make_uint4(__builtin_bit_cast(uint32_t, h01), __builtin_bit_cast(uint32_t, h23),
                                        khi ? 0u : __builtin_bit_cast(uint32_t, l01),
                                        khi ? 0u : __builtin_bit_cast(uint32_t, l23));
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
              const uint4 g = s_gc[64 * wave + 32 * pb + (lane & 31)];
              const uint4 bv = khi ? make_uint4(g.z, g.w, 0u, 0u) : make_uint4(g.x, g.y, g.x, g.y);
              s1[pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                               __builtin_bit_cast(bf16x8, bv), s1[pb], 0, 0, 0);
            }
          }
          // pairs at list positions >= min(last, pos0 + nb) are not walked for this pixel
          const int lim = min(last, pos0 + nb) - pos0;
          constexpr int GR = WS_GR;
          // alpha, 1 / (1 - alpha) and G of the GR pairs of group gi, independent
          // of each other; a pair that is not walked gets alpha 0 (and G 0),
          // which leaves the chain below unchanged without per-pair selects
          auto alpha_group = [&](int gi, float (&al)[GR], float (&inv)[GR], float (&gx)[GR]) {
#pragma unroll
            for (int u = 0; u < GR; ++u) {
              const int i = gi * GR + u;
              const float2 m = s_xy[b3][i];
              const float4 co = s_cs[b3][i];
              const float dx = fpx - m.x, dy = fpy - m.y;
              const float qs = scaled_q(co, dx, dy);
              const bool inb = in_box(pp, s_box[b2][i]);
              const float G = __builtin_amdgcn_exp2f(qs);
              const float opG = co.w * G;
              const float alpha = fminf(kAlphaMax, opG);
              const bool ct = (i < lim) & inb & (qs >= s_tg[b3][i]);
              al[u] = ct ? alpha : 0.f;
              inv[u] = __builtin_amdgcn_rcpf(1.0f - al[u]);
              gx[u] = (ct & (opG <= kAlphaMax)) ? G : 0.f;
            }
          };
          // the first group walked (the batch's last GR pairs) is evaluated while
          // the matrix cores finish GEMM1: it does not need S
          constexpr int kFirst = 2 * (16 / GR) - 1;
          float al0[GR], inv0[GR], gx0[GR];
          alpha_group(kFirst, al0, inv0, gx0);
          float S[kNB];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(s1[0][v]), __float_as_uint(s1[1][v]),
                                                            false, false);
            S[8 * (v >> 2) + (v & 3)] = __uint_as_float(r[0]);
            S[8 * (v >> 2) + 4 + (v & 3)] = __uint_as_float(r[1]);
          }
#pragma unroll
          for (int h = 1; h >= 0; --h) {
#pragma unroll
            for (int gq = 16 / GR - 1; gq >= 0; --gq) {
              const int gi = (16 / GR) * h + gq;
              float al[GR], inv[GR], gx[GR];
              if (gi == kFirst) {
#pragma unroll
                for (int u = 0; u < GR; ++u) {
                  al[u] = al0[u];
                  inv[u] = inv0[u];
                  gx[u] = gx0[u];
                }
              } else {
                alpha_group(gi, al, inv, gx);
              }
              // back-to-front recovery of T and the running colour/feature sum
              float wg[GR];
#pragma unroll
              for (int u = GR - 1; u >= 0; --u) {
                const float sv = S[gi * GR + u];   // dL/d(c_i, f_i) . (c_i, f_i) at this pixel
                const float Tn = T * inv[u];
                const float w = al[u] * Tn;
                const float da = inv[u] * __builtin_fmaf(T, sv, -acc);   // (T sv - acc) / (1 - alpha)
                T = Tn;
                acc = __builtin_fmaf(w, sv, acc);
                wg[u] = w;
                s_xm[wave][gq * GR + u][lane] = gx[u] * da;   // X = G dL/dalpha at this pixel
              }
              // two-part bf16 split of the weights, two pairs per conversion
#pragma unroll
              for (int u = 0; u < GR; u += 2) {
                const f32x2 w2 = {wg[u], wg[u + 1]};
                const bf16x2 h2 = __builtin_convertvector(w2, bf16x2);
                const bf16x2 l2 = __builtin_convertvector(w2 - __builtin_convertvector(h2, f32x2), bf16x2);
                s_w[b2][wave][0][gi * GR + u][lane] = h2[0];
                s_w[b2][wave][0][gi * GR + u + 1][lane] = h2[1];
                s_w[b2][wave][1][gi * GR + u][lane] = l2[0];
                s_w[b2][wave][1][gi * GR + u + 1][lane] = l2[1];
              }
            }
            // six pixel moments of X per Gaussian of the half: lane l sums 16
            // pixels (quarter l / 16 of the wave) of Gaussian l % 16 from LDS
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int qr = lane >> 4;
            const float* xr = &s_xm[wave][lane & 15][16 * qr];
            float xv[16];
#pragma unroll
            for (int j4 = 0; j4 < 4; ++j4) {
              const float4 v4 = *reinterpret_cast<const float4*>(xr + 4 * j4);
              xv[4 * j4] = v4.x;
              xv[4 * j4 + 1] = v4.y;
              xv[4 * j4 + 2] = v4.z;
              xv[4 * j4 + 3] = v4.w;
            }
            // runs of 8 pixels: sums of X, j X, j^2 X (j = 0..7 along the run)
            float r0[2], r1[2], r2[2];
#pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
              r0[rr] = r1[rr] = r2[rr] = 0.f;
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                const float x = xv[8 * rr + j];
                r0[rr] += x;
                r1[rr] = __builtin_fmaf((float)j, x, r1[rr]);
                r2[rr] = __builtin_fmaf((float)(j * j), x, r2[rr]);
              }
            }
            // pixel coordinates relative to the tile centre: the quarter starts at
            // tile pixel p0; with tiles at least 16 wide it is part of one row,
            // 8-wide tiles put its two runs on two rows
            const int p0 = 64 * wave + 16 * qr;
            const float hx = 0.5f - 0.5f * (float)a.tile_w, hy = 0.5f - 0.5f * (float)tile_h;
            float mom[6];   // X, X lx, X ly, X lx^2, X lx ly, X ly^2
            if (a.tile_w >= 16) {
              const float x0 = (float)(p0 % a.tile_w) + hx, y0 = (float)(p0 / a.tile_w) + hy;
              const float s0 = r0[0] + r0[1];
              const float s1 = r1[0] + __builtin_fmaf(8.0f, r0[1], r1[1]);
              const float s2 = r2[0] + __builtin_fmaf(16.0f, r1[1], __builtin_fmaf(64.0f, r0[1], r2[1]));
              const float m10 = __builtin_fmaf(x0, s0, s1);
              mom[0] = s0;
              mom[1] = m10;
              mom[2] = y0 * s0;
              mom[3] = __builtin_fmaf(x0, __builtin_fmaf(x0, s0, 2.0f * s1), s2);
              mom[4] = y0 * m10;
              mom[5] = y0 * y0 * s0;
            } else {
              const float x0 = hx, ya = (float)(p0 / a.tile_w) + hy, yb = ya + 1.0f;
              const float ma = __builtin_fmaf(x0, r0[0], r1[0]), mb = __builtin_fmaf(x0, r0[1], r1[1]);
              mom[0] = r0[0] + r0[1];
              mom[1] = ma + mb;
              mom[2] = __builtin_fmaf(ya, r0[0], yb * r0[1]);
              mom[3] = __builtin_fmaf(x0, __builtin_fmaf(x0, mom[0], 2.0f * (r1[0] + r1[1])), r2[0] + r2[1]);
              mom[4] = __builtin_fmaf(ya, ma, yb * mb);
              mom[5] = __builtin_fmaf(ya * ya, r0[0], yb * yb * r0[1]);
            }
            // sums over the wave's four 16-lane quarters with lane swaps: the
            // 32-lane swap of (moment k, moment k + 3) leaves the half sums of
            // k in lanes 0-31 and of k + 3 in lanes 32-63; the 16-lane swap of
            // two such registers finishes four moments, one per 16-lane row
            float R[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(mom[k]), __float_as_uint(mom[k + 3]),
                                                              false, false);
              R[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
            }
            const auto p01 = __builtin_amdgcn_permlane16_swap(__float_as_uint(R[0]), __float_as_uint(R[1]), false, false);
            const auto p22 = __builtin_amdgcn_permlane16_swap(__float_as_uint(R[2]), __float_as_uint(R[2]), false, false);
            const float mA = __uint_as_float(p01[0]) + __uint_as_float(p01[1]);   // rows: moments 0, 1, 3, 4
            const float mB = __uint_as_float(p22[0]) + __uint_as_float(p22[1]);   // rows 0-1: moment 2; 2-3: 5
            const int row = lane >> 4;
            s_mom[b2][wave][row < 2 ? row : row + 1][16 * h + (lane & 15)] = mA;
            if ((lane & 16) == 0) s_mom[b2][wave][row == 0 ? 2 : 5][16 * h + (lane & 15)] = mB;
            // s_xm is rewritten by the next half only after every lane has read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
          // colour sums of the wave's pixels on the matrix cores
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
          for (int mb = 0; mb < 2; ++mb) {
            f32x4 cs = f32x4{};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
              const int kp = 32 * ks + 8 * (lane >> 4);
              const bf16x8 wh = *reinterpret_cast<const bf16x8*>(&s_w[b2][wave][0][16 * mb + (lane & 15)][kp]);
              const bf16x8 wl = *reinterpret_cast<const bf16x8*>(&s_w[b2][wave][1][16 * mb + (lane & 15)][kp]);
              const bf16x8 gh = s_grb[wave][ks][0][lane];
              const bf16x8 gl = s_grb[wave][ks][1][lane];
              cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, gh, cs, 0, 0, 0);
              cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, gl, cs, 0, 0, 0);
              cs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, gh, cs, 0, 0, 0);
            }
            if ((lane & 15) < 4) {
#pragma unroll
              for (int v = 0; v < 4; ++v) s_col[b2][wave][lane & 15][16 * mb + 4 * (lane >> 4) + v] = cs[v];
            }
          }
        }
      }
      __syncthreads();
    }
  } else {
    for (int i0 = 0;; ++i0) {
      const int it = __builtin_amdgcn_readfirstlane(i0);   // scalar: keeps the barrier loop uniform
      if (it > nbatch) break;
      // ================= contractors: GEMM2 and rows of batch it-1, staging of batch it+1 =================
      if (it >= 1) {
        const int k = it - 1;
        const int b2 = k & 1, b3 = k % 3;
        const int pos0 = bpos0(k), nb = bnb(k);
        // one accumulator (a dependent MFMA chain) keeps registers for the
        // upstream-gradient operand, which holds 128 VGPRs at D = 128
        f32x16 d = f32x16{};
#pragma unroll
        for (int u = 0; u < CB; ++u) {
          const int chunk = unit_chunk(u);
          if (s_live[b2][chunk]) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int kp = 16 * s + 8 * (lane >> 5);
              const bf16x8 wh = *reinterpret_cast<const bf16x8*>(&s_w[b2][chunk][0][lane & 31][kp]);
              const bf16x8 wl = *reinterpret_cast<const bf16x8*>(&s_w[b2][chunk][1][lane & 31][kp]);
              d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, g2(u, s, 0), d, 0, 0, 0);
              d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wh, g2(u, s, 1), d, 0, 0, 0);
              d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, g2(u, s, 0), d, 0, 0, 0);
            }
          }
          if (u % NW == NW - 1) {   // the channel block is complete
            const int c = 32 * unit_cb(u) + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
              if (i < nb && c < a.D) a.rows[(row0 + pos0 + i) * a.RS + c] = d[v];
            }
            d = f32x16{};
          }
        }
        // rest of the rows (one lane per Gaussian of the batch): the walker waves'
        // pixel moments and colour sums are added up, moved from the tile centre
        // to the Gaussian's centre and turned into projected-space gradients with
        // its conic and opacity; the row is closed with zeros up to its stride
        if (q < nb) {
          const int i = q;
          float P[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, Cc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int w = 0; w < NW; ++w) {
            if (!s_live[b2][w]) continue;
#pragma unroll
            for (int k2 = 0; k2 < 6; ++k2) P[k2] += s_mom[b2][w][k2][i];
#pragma unroll
            for (int c = 0; c < 4; ++c) Cc[c] += s_col[b2][w][c][i];
          }
          const float2 m = s_xy[b3][i];
          const float4 co = s_co[b3][i];
          // Gaussian centre relative to the tile centre; dx = lx - ux per pixel
          const float ux = m.x - ((float)tx0 + 0.5f * (float)a.tile_w);
          const float uy = m.y - ((float)ty0 + 0.5f * (float)tile_h);
          const float S0 = __builtin_fmaf(-ux, P[0], P[1]);                          // sum X dx
          const float S1 = __builtin_fmaf(-uy, P[0], P[2]);                          // sum X dy
          const float S2 = __builtin_fmaf(-ux, __builtin_fmaf(-ux, P[0], 2.0f * P[1]), P[3]);   // X dx^2
          const float S3 = __builtin_fmaf(-ux, __builtin_fmaf(-uy, P[0], P[2]), __builtin_fmaf(-uy, P[1], P[4]));
          const float S4 = __builtin_fmaf(-uy, __builtin_fmaf(-uy, P[0], 2.0f * P[2]), P[5]);   // X dy^2
          float v9[10];
          v9[0] = co.w * (co.x * S0 + co.y * S1);
          v9[1] = co.w * (co.y * S0 + co.z * S1);
          v9[2] = -0.5f * co.w * S2;
          v9[3] = -co.w * S3;
          v9[4] = -0.5f * co.w * S4;
          v9[5] = P[0];
          v9[6] = Cc[0];
          v9[7] = Cc[1];
          v9[8] = Cc[2];
          v9[9] = Cc[3];
          float* row = &a.rows[(row0 + pos0 + i) * a.RS];
          if ((a.D & 3) == 0) {
            // the sums start on a 16-byte boundary: three vector stores, then
            // zeros to the end of the row's last 128-byte line
            float4* r4 = reinterpret_cast<float4*>(row + a.D);
            r4[0] = make_float4(v9[0], v9[1], v9[2], v9[3]);
            r4[1] = make_float4(v9[4], v9[5], v9[6], v9[7]);
            r4[2] = make_float4(v9[8], v9[9], 0.f, 0.f);
            for (int c = a.D + 12; c < a.RS; c += 4) *reinterpret_cast<float4*>(row + c) = make_float4(0.f, 0.f, 0.f, 0.f);
          } else {
            auto pick = [&](int t) {
              float x = 0.f;
#pragma unroll
              for (int k2 = 0; k2 < 10; ++k2) x = t == k2 ? v9[k2] : x;
              return x;
            };
            int c = a.D;
            for (; (c & 3) != 0 && c < a.RS; ++c) row[c] = pick(c - a.D);
            for (; c < a.RS; c += 4)
              *reinterpret_cast<float4*>(row + c) =
                  make_float4(pick(c - a.D), pick(c + 1 - a.D), pick(c + 2 - a.D), pick(c + 3 - a.D));
          }
        }
        if (q < nb) a.rowidx[ep_w] = (uint32_t)(row0 + pos0 + q + 1);
      }
      ep_w = ep_s;
      if (it + 1 < nbatch) {
        stage(it + 1);
        load_data();
        load_ids(it + 3);
      }
      __syncthreads();
    }
  }
}

// Tiles in the backward preparation's order (longest walks first), dealt to
// the XCDs in runs as everywhere else.
__device__ __forceinline__ int bwd_tile(const BwdArgs& a) {
  return (int)__builtin_amdgcn_readfirstlane(a.order[xcd_tile((int)blockIdx.x, (int)gridDim.x)]);
}

template <int DP, typename FT, int NT>
__global__ __launch_bounds__(NT) void composite_bwd_mfma_kernel(BwdArgs a) {
  bwd_mfma_tile<DP, FT, NT, true>(a, bwd_tile(a));
}

template <int DP, typename FT, int NT>
__global__ __launch_bounds__(2 * NT) void composite_bwd_ws_kernel(BwdArgs a) {
  bwd_ws_tile<DP, FT, NT, true>(a, bwd_tile(a));
}

// The wave-specialized form applies where contractor waves own whole channel
// blocks; elsewhere one wave per 64 pixels runs both roles.
template <int DP, int NT>
constexpr bool bwd_ws_available() { return DP <= 128 && DP / 32 >= NT / 64; }

// Persistent form over many frames: each workgroup takes (frame, tile) items
// from a queue sorted by walk length, longest first, until it is empty.
template <int DP, typename FT, int NT, bool WS>
__global__ __launch_bounds__((WS ? 2 * NT : NT)) void composite_bwd_persistent(
    const BwdArgs* __restrict__ args, TileQueue tq) {
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
    // the frame record is copied out of global memory, so that the tile's
    // stores cannot be taken to alias it (its fields stay in registers)
    const BwdArgs a = args[item.x];
    if constexpr (WS) bwd_ws_tile<DP, FT, NT, false>(a, (int)item.y);
    else bwd_mfma_tile<DP, FT, NT, false>(a, (int)item.y);
    if (threadIdx.x == 0) s_item = atomicAdd(tq.head, 1u);
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
  }
}

// ---- per-Gaussian sum of the rows of the tiles it was walked in ----
struct ReduceArgs {
  int64_t n;
  int32_t D, RS;
  const uint32_t* count;
  const uint32_t* eoff;
  const uint32_t* rowidx;       // [cap] 1 + row by emit position, 0 when the pair was not walked
  const float* rows;
  const unsigned long long* report;
  float* grad2d;                // [n][12]
  float* grad_feat;             // [n][D]
  int accumulate;
  int vec_out;                  // grad_feat rows allow aligned float4 stores
};

// LPG lanes per Gaussian (a power of two dividing 64); lane k owns the
// 4-channel groups k, k + LPG, ... of the row.  A Gaussian's pairs are
// contiguous in emit order, so its row indices are one coalesced read; up to
// four rows are loaded before they are summed, so that several row reads are
// in flight per lane.
template <int LPG, int GPL>
__device__ __forceinline__ void reduce_one(const ReduceArgs& a, int64_t g, uint32_t cnt, uint32_t e0, uint32_t ri0) {
  const int sub = threadIdx.x & (LPG - 1);
  const int gbase = (int)(threadIdx.x & 63) & ~(LPG - 1);      // first lane of the group in the wave
  const bool live = g < a.n;
  float4 acc[GPL];
#pragma unroll
  for (int k = 0; k < GPL; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  float acc9 = 0.f;
  uint32_t cmax = cnt;
  for (int o = 32; o >= LPG; o >>= 1) cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, o, 64));
  const int D4 = a.D >> 2;                  // whole 4-channel groups
  for (uint32_t base = 0; base < cmax; base += LPG) {
    const uint32_t ri = base == 0 ? ri0 : (base + sub < cnt ? a.rowidx[e0 + base + sub] : 0u);
    const unsigned long long m = __ballot(ri != 0u);
    unsigned long long mine = LPG == 64 ? m : (m >> gbase) & ((1ull << (LPG & 63)) - 1ull);
    int most = __popcll(mine);
    for (int o = 32; o >= LPG; o >>= 1) most = max(most, __shfl_xor(most, o, 64));
    for (int k = 0; k < most; k += 4) {
      uint32_t r[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int b = mine ? __ffsll(mine) - 1 : 0;
        r[t] = (uint32_t)__shfl((int)ri, gbase + b, 64);
        r[t] = mine ? r[t] : 0u;
        mine &= mine - 1;
      }
      float4 v[4][GPL];
      float t9[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float* src = a.rows + (int64_t)(r[t] ? r[t] - 1 : 0) * a.RS;
#pragma unroll
        for (int q = 0; q < GPL; ++q) {
          const int grp = sub + q * LPG;
          v[t][q] = (r[t] && grp < D4) ? *reinterpret_cast<const float4*>(src + 4 * grp) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        // channels past the last whole group, and the 10 projected-space sums
        const int c = 4 * D4 + sub;
        t9[t] = (r[t] && c < a.D + 10) ? src[c] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int q = 0; q < GPL; ++q) {
          acc[q].x += v[t][q].x;
          acc[q].y += v[t][q].y;
          acc[q].z += v[t][q].z;
          acc[q].w += v[t][q].w;
        }
        acc9 += t9[t];
      }
    }
  }
  if (!live) return;
  float* fo = a.grad_feat + g * a.D;
#pragma unroll
  for (int q = 0; q < GPL; ++q) {
    const int grp = sub + q * LPG;
    if (grp < D4) {
      float4 x = acc[q];
      if (a.vec_out) {
        float4* o4 = reinterpret_cast<float4*>(fo + 4 * grp);
        if (a.accumulate) {
          const float4 y = *o4;
          x = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
        }
        *o4 = x;
      } else {
        const float xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) fo[4 * grp + j] = a.accumulate ? fo[4 * grp + j] + xs[j] : xs[j];
      }
    }
  }
  // lane sub holds column 4 D4 + sub: a leftover channel or one of the 10 sums
  const int c = 4 * D4 + sub;
  if (c < a.D) fo[c] = a.accumulate ? fo[c] + acc9 : acc9;
  // the 10 sums sit in lanes (D - 4 D4) .. (D - 4 D4 + 9)
  const int k9 = c - a.D;
  if (k9 >= 0 && k9 < 10) a.grad2d[g * 12 + k9] = acc9;
  if (sub < 2) a.grad2d[g * 12 + 10 + sub] = 0.f;
}

// Each group of LPG lanes sums the rows of NG consecutive Gaussians; their
// counts, first emit positions and first row indices are loaded together, so
// a group waits on one chain of dependent loads for all NG instead of NG
// chains.
template <int LPG, int GPL, int NG>
__global__ __launch_bounds__(256) void reduce_rows_kernel(ReduceArgs a) {
  const int sub = threadIdx.x & (LPG - 1);
  const int64_t g0 = (((int64_t)blockIdx.x * 256 + threadIdx.x) / LPG) * NG;
  const bool ok = a.report[kRepStatus] == 0ull && a.report[kRepBwdStatus] == 0ull;
  uint32_t cnt[NG], e0[NG], ri0[NG];
#pragma unroll
  for (int k = 0; k < NG; ++k) {
    const int64_t g = g0 + k;
    const bool live = g < a.n;
    cnt[k] = (live && ok) ? a.count[g] : 0u;
    e0[k] = live ? a.eoff[g] : 0u;        // read whether or not used: it does not wait on the count
  }
#pragma unroll
  for (int k = 0; k < NG; ++k) ri0[k] = (uint32_t)sub < cnt[k] ? a.rowidx[e0[k] + sub] : 0u;
#pragma unroll
  for (int k = 0; k < NG; ++k) reduce_one<LPG, GPL>(a, g0 + k, cnt[k], e0[k], ri0[k]);
}

template <int DP, typename FT, int NT>
static void launch_bwd_tiles(const BwdArgs& a, int tiles, bool ws, hipStream_t s) {
  if constexpr (bwd_ws_available<DP, NT>()) {
    if (ws) {
      hipLaunchKernelGGL((composite_bwd_ws_kernel<DP, FT, NT>), dim3(tiles), dim3(2 * NT), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((composite_bwd_mfma_kernel<DP, FT, NT>), dim3(tiles), dim3(NT), 0, s, a);
}

template <int DP, typename FT>
hipError_t launch_bwd_nt(int nt, const BwdArgs& a, int tiles, bool ws, hipStream_t s) {
  switch (nt) {
    case 64: launch_bwd_tiles<DP, FT, 64>(a, tiles, ws, s); break;
    case 128: launch_bwd_tiles<DP, FT, 128>(a, tiles, ws, s); break;
    default: launch_bwd_tiles<DP, FT, 256>(a, tiles, ws, s); break;
  }
  return hipGetLastError();
}

// Feature width of the instantiation a backward launch uses: the next of 32,
// 64, 128, 256 at or above D.  The wave-specialized form needs a 32-channel
// block per contractor wave (NT / 64 of them), so narrower features take the
// instantiation with that many blocks; their extra channels are zero (staged
// as zeros, never stored).
int bwd_width(int D, int nt, bool ws) {
  int dp = D <= 32 ? 32 : D <= 64 ? 64 : D <= 128 ? 128 : 256;
  if (ws && dp < 32 * (nt / 64)) dp = 32 * (nt / 64);
  return dp;
}

template <typename FT>
hipError_t dispatch_bwd(int D, int nt, const BwdArgs& a, int tiles, bool ws, hipStream_t s) {
  switch (bwd_width(D, nt, ws)) {
    case 32: return launch_bwd_nt<32, FT>(nt, a, tiles, ws, s);
    case 64: return launch_bwd_nt<64, FT>(nt, a, tiles, ws, s);
    case 128: return launch_bwd_nt<128, FT>(nt, a, tiles, ws, s);
    default: return launch_bwd_nt<256, FT>(nt, a, tiles, ws, s);
  }
}

}  // namespace

// Wave-specialized backward (2 NT threads per tile) for D <= 128 (narrower
// features use a wider instantiation, see bwd_width) where threads_per_tile
// asks for it or leaves the choice to the library.
bool backward_wave_specialized(const fe_config* cfg) {
  const int nt = cfg->tile_w * cfg->tile_h;
  return cfg->feat_dim <= 128 && nt <= 256 && cfg->threads_per_tile != nt;
}

// Rows are padded to whole 128-byte lines: each 32-channel block of dF and
// the closing block of the row (the nine projected-space sums and zeros) is
// then one full, aligned line written by one store instruction, instead of
// partial lines written at different times by different waves.
int backward_row_stride(int D) { return (D + 10 + 31) & ~31; }

static BwdArgs make_bwd_args(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                              const fe_images* fwd, const float* d_rgb, const float* d_feat, const float* d_depth,
                              const uint32_t* row_base, float* rows, int64_t row_cap, uint32_t* rowidx) {
  BwdArgs a{};
  a.ranges = v.ranges;
  a.gauss = v.gauss;
  a.xy = v.xy;
  a.conic_o = v.conic_o;
  a.rgb = v.rgb;
  a.box = v.box;
  a.feat = g->feat;
  a.final_T = fwd->final_T;
  a.n_contrib = fwd->n_contrib;
  a.d_rgb = d_rgb;
  a.d_feat = d_feat;
  a.d_depth = d_depth;
  a.tile_maxlast = v.tile_maxlast;
  a.row_base = row_base;
  a.order = row_base + v.tiles + 1;   // written by the backward preparation
  a.rows = rows;
  a.row_cap = row_cap;
  a.rowidx = rowidx;
  a.epos = v.epos;
  a.report = v.report;
  for (int k = 0; k < 3; ++k) a.bg[k] = cfg->bg_rgb[k];
  a.W = cam->width;
  a.H = cam->height;
  a.tile_w = cfg->tile_w;
  a.tiles_x = v.tiles_x;
  a.D = cfg->feat_dim;
  a.RS = backward_row_stride(cfg->feat_dim);
  const size_t esz = cfg->feat_dtype == FE_BF16 ? 2 : 4;
  a.vec = cfg->feat_dim % 4 == 0 && reinterpret_cast<uintptr_t>(g->feat) % (4 * esz) == 0;
  return a;
}

hipError_t launch_composite_bwd_mfma(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                     const StateView& v, const fe_images* fwd, const float* d_rgb,
                                     const float* d_feat, const float* d_depth, const uint32_t* row_base, float* rows,
                                     int64_t row_cap, uint32_t* rowidx, hipStream_t s) {
  if (v.tiles == 0) return hipSuccess;
  const BwdArgs a = make_bwd_args(cfg, cam, g, v, fwd, d_rgb, d_feat, d_depth, row_base, rows, row_cap, rowidx);
  const int nt = cfg->tile_w * cfg->tile_h;
  const bool ws = backward_wave_specialized(cfg);
  return cfg->feat_dtype == FE_BF16 ? dispatch_bwd<uint16_t>(cfg->feat_dim, nt, a, v.tiles, ws, s)
                                    : dispatch_bwd<float>(cfg->feat_dim, nt, a, v.tiles, ws, s);
}

// ---- persistent multi-frame form (BF16 features, D <= 128) ----
size_t composite_bwd_record_bytes() { return sizeof(BwdArgs); }

void composite_bwd_record(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v,
                          const fe_images* fwd, const float* d_rgb, const float* d_feat, const float* d_depth,
                          const uint32_t* row_base, float* rows, int64_t row_cap, uint32_t* rowidx, void* dst) {
  const BwdArgs a = make_bwd_args(cfg, cam, g, v, fwd, d_rgb, d_feat, d_depth, row_base, rows, row_cap, rowidx);
  std::memcpy(dst, &a, sizeof(a));
}

template <int DP, int NT, bool WS>
static int bwd_grid() {
  int per_cu = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, composite_bwd_persistent<DP, uint16_t, NT, WS>,
                                                   WS ? 2 * NT : NT, 0) != hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

template <int DP, int NT>
static int bwd_grid_ws(bool ws) {
  if constexpr (bwd_ws_available<DP, NT>()) {
    if (ws) return bwd_grid<DP, NT, true>();
  }
  return bwd_grid<DP, NT, false>();
}

template <int DP>
static int bwd_grid_nt(int nt, bool ws) {
  return nt == 64 ? bwd_grid_ws<DP, 64>(ws) : nt == 128 ? bwd_grid_ws<DP, 128>(ws) : bwd_grid_ws<DP, 256>(ws);
}

int composite_bwd_persistent_grid(const fe_config* cfg) {
  const int nt = cfg->tile_w * cfg->tile_h;
  const bool ws = backward_wave_specialized(cfg);
  const int dp = bwd_width(cfg->feat_dim, nt, ws);
  return dp <= 32 ? bwd_grid_nt<32>(nt, ws) : dp <= 64 ? bwd_grid_nt<64>(nt, ws) : bwd_grid_nt<128>(nt, ws);
}

template <int DP, int NT>
static void bwd_persistent_launch(const BwdArgs* r, const TileQueue& q, int grid, bool ws, hipStream_t s) {
  if constexpr (bwd_ws_available<DP, NT>()) {
    if (ws) {
      hipLaunchKernelGGL((composite_bwd_persistent<DP, uint16_t, NT, true>), dim3(grid), dim3(2 * NT), 0, s, r, q);
      return;
    }
  }
  hipLaunchKernelGGL((composite_bwd_persistent<DP, uint16_t, NT, false>), dim3(grid), dim3(NT), 0, s, r, q);
}

template <int DP>
static hipError_t bwd_persistent_nt(int nt, const BwdArgs* r, const TileQueue& q, int grid, bool ws,
                                    hipStream_t s) {
  switch (nt) {
    case 64: bwd_persistent_launch<DP, 64>(r, q, grid, ws, s); break;
    case 128: bwd_persistent_launch<DP, 128>(r, q, grid, ws, s); break;
    default: bwd_persistent_launch<DP, 256>(r, q, grid, ws, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_composite_bwd_persistent(const fe_config* cfg, const void* records, const TileQueue& q,
                                           int grid, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  const int nt = cfg->tile_w * cfg->tile_h;
  const bool ws = backward_wave_specialized(cfg);
  const BwdArgs* r = static_cast<const BwdArgs*>(records);
  const int dp = bwd_width(cfg->feat_dim, nt, ws);
  return dp <= 32 ? bwd_persistent_nt<32>(nt, r, q, grid, ws, s)
                  : dp <= 64 ? bwd_persistent_nt<64>(nt, r, q, grid, ws, s)
                             : bwd_persistent_nt<128>(nt, r, q, grid, ws, s);
}

hipError_t launch_reduce_rows(const fe_config* cfg, const StateView& v, const uint32_t* rowidx,
                              const float* rows, float* grad2d, float* grad_feat, hipStream_t s) {
  if (v.n == 0) return hipSuccess;
  ReduceArgs a{};
  a.n = v.n;
  a.D = cfg->feat_dim;
  a.RS = backward_row_stride(cfg->feat_dim);
  a.count = v.count;
  a.eoff = v.eoff;
  a.rowidx = rowidx;
  a.rows = rows;
  a.report = v.report;
  a.grad2d = grad2d;
  a.grad_feat = grad_feat;
  a.accumulate = (cfg->flags & FE_FLAG_NO_ZERO_GRADS) ? 1 : 0;
  a.vec_out = cfg->feat_dim % 4 == 0 && reinterpret_cast<uintptr_t>(grad_feat) % 16 == 0;
  const int D = cfg->feat_dim;
  // lanes per Gaussian: enough 4-channel groups per lane for the row, and at
  // least 16 lanes so that the leftover channels and the 10 sums have a lane
  constexpr int NG = 4;   // Gaussians per lane group
  if (D <= 64) {
    const unsigned blocks = (unsigned)((v.n + 16 * NG - 1) / (16 * NG));
    hipLaunchKernelGGL((reduce_rows_kernel<16, 1, NG>), dim3(blocks), dim3(256), 0, s, a);
  } else if (D <= 128) {
    const unsigned blocks = (unsigned)((v.n + 8 * NG - 1) / (8 * NG));
    hipLaunchKernelGGL((reduce_rows_kernel<32, 1, NG>), dim3(blocks), dim3(256), 0, s, a);
  } else {
    const unsigned blocks = (unsigned)((v.n + 4 * NG - 1) / (4 * NG));
    hipLaunchKernelGGL((reduce_rows_kernel<64, 1, NG>), dim3(blocks), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace fe
