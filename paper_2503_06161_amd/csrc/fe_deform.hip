// FST deformation module (Sec. 3.2, eqs. 4-6; appendix "FST Deformation
// Module"): canonical Gaussians + time -> G_t, the rasterizer's input.
//
// One workgroup of 4 waves takes 64 Gaussians through the whole module:
//   1. HexPlane: every (Gaussian, level) is one item; C/4 lanes share an
//      item, each holding 4 channels, so every tap of a plane is one
//      contiguous C-channel read shared by those lanes.  Coordinates and
//      interpolation weights in float64, samples and the plane product in
//      float32.  The features go to LDS, one row per Gaussian.
//   2. The affine layers (F_out, the four branches, the semantic updater) on
//      16x16x32 bf16 MFMAs: wave w owns Gaussians 16w..16w+15 in every
//      layer, so activations pass from layer to layer through that wave's
//      own LDS rows with no workgroup barrier.  A = activations (split into
//      bf16 hi + lo as they are read), B = weights (split once per call by
//      the prep kernel into the workspace, zero rows padding the outputs to a
//      multiple of 16); products hi*hi + hi*lo + lo*hi, float32 accumulation.
//   3. G_t written from the head outputs and the semantic update.
#include "fe_common.h"

#include <math.h>

#pragma clang fp contract(off)

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW = 64;            // F_out width
constexpr int kRows = 64;         // Gaussians per workgroup
constexpr int kThreads = 256;     // 4 waves x 16 Gaussians
constexpr int kLayers = 22;       // F_out 8, branches 4 x 3, semantic 2
constexpr int kPlanes = 24;       // 4 levels x 6 pairs
constexpr int kBranchDim[4] = {3, 4, 3, 1};
constexpr int kDOff[4] = {0, 3, 7, 10};   // columns of the head outputs
constexpr int kLdA = kW + 4;              // padded LDS rows
constexpr int kLdD = 12;

__host__ __device__ constexpr int pair_a(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__host__ __device__ constexpr int pair_b(int p) { return p == 0 ? 1 : (p == 1 ? 2 : (p == 3 ? 2 : 3)); }

struct LayerDesc {
  int in, out, out_pad;
  int64_t w_off, b_off;   // floats into the weight array
  int64_t p_off;          // elements into each split part
};
struct PlaneDesc {
  int64_t off;            // floats into the plane array
  int ra, rb;             // columns (coordinate a), rows (coordinate b)
};

struct DeformArgs {
  LayerDesc layer[kLayers];
  PlaneDesc plane[kPlanes];
  const float* planes;
  const float* weights;
  const __bf16* whi;
  const __bf16* wlo;
  double lo[3], hi[3];
  double ut;              // time coordinate in [-1, 1]
  int64_t n;
  int N;
  int out_bf16;
  const float* means;
  const float* quats;
  const float* log_scales;
  const float* logit_opacity;
  const float* feat;
  float* out_means;
  float* out_quats;
  float* out_scales;
  float* out_opacity;
  void* out_feat;
};

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Weights of every layer into bf16 hi / lo parts in the order the MFMA B
// operand is read: 512-element blocks of 16 outputs x 32 inputs, block
// (output tile tb, input step kb) at (tb * in / 32 + kb) * 512, lane l of a
// block holding outputs 16 tb + l % 16, inputs 32 kb + 8 (l / 16) .. + 7 as
// 8 consecutive elements (rows past `out` are zero).
__global__ __launch_bounds__(256) void deform_prep_kernel(DeformArgs a, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  int l = 0;
  while (l + 1 < kLayers && i >= a.layer[l + 1].p_off) ++l;
  const LayerDesc L = a.layer[l];
  const int64_t e = i - L.p_off;
  const int blk = (int)(e / 512), w = (int)(e % 512), ln = w / 8, j = w % 8;
  const int tb = blk / (L.in / 32), kb = blk % (L.in / 32);
  const int n = 16 * tb + (ln & 15), k = 32 * kb + 8 * (ln >> 4) + j;
  const float v = n < L.out ? a.weights[L.w_off + (int64_t)n * L.in + k] : 0.f;
  __bf16 hi, lo;
  split2(v, hi, lo);
  const_cast<__bf16*>(a.whi)[i] = hi;
  const_cast<__bf16*>(a.wlo)[i] = lo;
}

// acc[nt] (16 x 16 tiles of columns n0 + 16 nt ..) += act(X rows of this
// wave) W[:, k0 .. k0 + K)^T: K of the layer's inputs, starting at input k0.
template <int K, int NT, bool RELU>
__device__ __forceinline__ void dense(const float* X, int ldx, const DeformArgs& a, const LayerDesc& L, int n0,
                                      int k0, f32x4 (&acc)[NT], int lane, int wave) {
  const int r = 16 * wave + (lane & 15);
  const int kq = 8 * (lane >> 4);
  const __bf16* bh0 = a.whi + L.p_off + 8 * lane;
  const __bf16* bl0 = a.wlo + L.p_off + 8 * lane;
  const int bstride = (L.in / 32) * 512;          // one output tile
  const int boff = (n0 / 16) * bstride + (k0 / 32) * 512;
#pragma unroll
  for (int ks = 0; ks < K / 32; ++ks) {
    const float* xp = X + r * ldx + 32 * ks + kq;
    const float4 x0 = *reinterpret_cast<const float4*>(xp);
    const float4 x1 = *reinterpret_cast<const float4*>(xp + 4);
    float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    bf16x8 ah, al;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 hi, lo;
      split2(RELU ? fmaxf(xs[j], 0.f) : xs[j], hi, lo);
      ah[j] = hi;
      al[j] = lo;
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int e = boff + nt * bstride + ks * 512;
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(bh0 + e);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(bl0 + e);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[nt], 0, 0, 0);
    }
  }
}

// acc[nt] = the bias of the lane's output column (the products are added to it).
template <int NT>
__device__ __forceinline__ void init_bias(f32x4 (&acc)[NT], const DeformArgs& a, const LayerDesc& L, int n0,
                                          int lane) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = n0 + 16 * nt + (lane & 15);
    const float b = n < L.out ? a.weights[L.b_off + n] : 0.f;
    acc[nt] = f32x4{b, b, b, b};
  }
}

// Y[rows of this wave][n0 + ...] = acc, for the layer's real outputs.
template <int NT>
__device__ __forceinline__ void store_rows(float* Y, int ldy, const LayerDesc& L, int n0, const f32x4 (&acc)[NT],
                                           int lane, int wave) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = n0 + 16 * nt + (lane & 15);
    if (n < L.out) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Y[(16 * wave + 4 * (lane >> 4) + v) * ldy + (n - n0)] = acc[nt][v];
    }
  }
}

template <int K, int NT, bool RELU>
__device__ __forceinline__ void layer(const float* X, int ldx, float* Y, int ldy, const DeformArgs& a, int l,
                                      int lane, int wave) {
  const LayerDesc L = a.layer[l];
  f32x4 acc[NT];
  init_bias<NT>(acc, a, L, 0, lane);
  dense<K, NT, RELU>(X, ldx, a, L, 0, 0, acc, lane, wave);
  store_rows<NT>(Y, ldy, L, 0, acc, lane, wave);
  wave_sync();
}

// acc[nt] += (A operands held in registers, K = 32 KS) W[:, 0 .. K)^T.
template <int KS, int NT>
__device__ __forceinline__ void dense_regs(const bf16x8 (&ah)[KS], const bf16x8 (&al)[KS], const DeformArgs& a,
                                           const LayerDesc& L, f32x4 (&acc)[NT], int lane) {
  const __bf16* bh0 = a.whi + L.p_off + 8 * lane;
  const __bf16* bl0 = a.wlo + L.p_off + 8 * lane;
  const int bstride = (L.in / 32) * 512;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int e = nt * bstride + ks * 512;
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(bh0 + e);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(bl0 + e);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bh, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bl, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], bh, acc[nt], 0, 0, 0);
    }
}

// A operands (hi / lo, optionally after ReLU) of this wave's 16 rows of X,
// K = 32 KS inputs.
template <int KS, bool RELU>
__device__ __forceinline__ void load_a(const float* X, int ldx, bf16x8 (&ah)[KS], bf16x8 (&al)[KS], int lane,
                                       int wave) {
  const float* xp = X + (16 * wave + (lane & 15)) * ldx + 8 * (lane >> 4);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const float4 x0 = *reinterpret_cast<const float4*>(xp + 32 * ks);
    const float4 x1 = *reinterpret_cast<const float4*>(xp + 32 * ks + 4);
    const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 hi, lo;
      split2(RELU ? fmaxf(xs[j], 0.f) : xs[j], hi, lo);
      ah[ks][j] = hi;
      al[ks][j] = lo;
    }
  }
}

// The MLP keeps one LDS buffer, the HexPlane features' [64][4C + 4]: wave w
// owns rows 16w..16w+15, and every layer reads its input rows (all of them,
// into registers) before it writes its output rows in place.
template <int C>
__global__ __launch_bounds__(kThreads) void deform_kernel(DeformArgs a) {
  constexpr int LDX = 4 * C + 4;
  constexpr int KS0 = 4 * C / 32;            // k steps of the first layer
  __shared__ double s_u[kRows][4];
  __shared__ __attribute__((aligned(16))) float s_x[kRows * LDX];
  __shared__ float s_d[kRows * kLdD];        // head outputs

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t g0 = (int64_t)blockIdx.x * kRows;

  // normalised coordinates (past the last Gaussian: the last one's)
  if (threadIdx.x < kRows) {
    const int64_t g = g0 + threadIdx.x < a.n ? g0 + threadIdx.x : a.n - 1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double m = (double)a.means[g * 3 + k];
      const double u = 2.0 * (m - a.lo[k]) / (a.hi[k] - a.lo[k]) - 1.0;
      s_u[threadIdx.x][k] = fmin(fmax(u, -1.0), 1.0);
    }
    s_u[threadIdx.x][3] = a.ut;
  }
  __syncthreads();

  // 1. HexPlane: item = (Gaussian, level), C/4 lanes per item
  {
    constexpr int CG = C / 4;
    constexpr int IPW = 64 / CG;                 // items per wave and pass
    constexpr int PASSES = kRows * 4 / (IPW * (kThreads / 64));
    const int chunk = lane % CG;
#pragma unroll 1
    for (int pass = 0; pass < PASSES; ++pass) {
      const int it = (pass * (kThreads / 64) + wave) * IPW + lane / CG;
      const int gi = it >> 2, lvl = it & 3;
      float4 prod = make_float4(1.f, 1.f, 1.f, 1.f);
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const PlaneDesc pd = a.plane[lvl * 6 + p];
        const double x = (s_u[gi][pair_a(p)] + 1.0) / 2.0 * (double)(pd.ra - 1);
        const double y = (s_u[gi][pair_b(p)] + 1.0) / 2.0 * (double)(pd.rb - 1);
        int x0 = (int)floor(x), y0 = (int)floor(y);
        x0 = x0 < 0 ? 0 : (x0 > pd.ra - 2 ? pd.ra - 2 : x0);
        y0 = y0 < 0 ? 0 : (y0 > pd.rb - 2 ? pd.rb - 2 : y0);
        const double wx = x - (double)x0, wy = y - (double)y0;
        const float w00 = (float)((1.0 - wx) * (1.0 - wy)), w01 = (float)(wx * (1.0 - wy));
        const float w10 = (float)((1.0 - wx) * wy), w11 = (float)(wx * wy);
        const float* base = a.planes + pd.off + ((int64_t)y0 * pd.ra + x0) * C + 4 * chunk;
        const float4 v00 = *reinterpret_cast<const float4*>(base);
        const float4 v01 = *reinterpret_cast<const float4*>(base + C);
        const float4 v10 = *reinterpret_cast<const float4*>(base + (int64_t)pd.ra * C);
        const float4 v11 = *reinterpret_cast<const float4*>(base + (int64_t)pd.ra * C + C);
        float4 s;
        s.x = ((w00 * v00.x + w01 * v01.x) + w10 * v10.x) + w11 * v11.x;
        s.y = ((w00 * v00.y + w01 * v01.y) + w10 * v10.y) + w11 * v11.y;
        s.z = ((w00 * v00.z + w01 * v01.z) + w10 * v10.z) + w11 * v11.z;
        s.w = ((w00 * v00.w + w01 * v01.w) + w10 * v10.w) + w11 * v11.w;
        prod.x *= s.x;
        prod.y *= s.y;
        prod.z *= s.z;
        prod.w *= s.w;
        if (p == 2) __builtin_amdgcn_sched_barrier(0);   // at most three planes' taps in flight
      }
      *reinterpret_cast<float4*>(&s_x[gi * LDX + lvl * C + 4 * chunk]) = prod;
    }
  }
  __syncthreads();

  // 2. the affine layers, in place in s_x
  {
    bf16x8 ah[KS0], al[KS0];
    load_a<KS0, false>(s_x, LDX, ah, al, lane, wave);
    const LayerDesc L0 = a.layer[0];
    f32x4 acc[4];
    init_bias<4>(acc, a, L0, 0, lane);
    dense_regs<KS0, 4>(ah, al, a, L0, acc, lane);
    store_rows<4>(s_x, LDX, L0, 0, acc, lane, wave);
    wave_sync();
  }
#pragma unroll 1
  for (int l = 1; l < 8; ++l) {
    bf16x8 ah[2], al[2];
    load_a<2, true>(s_x, LDX, ah, al, lane, wave);
    const LayerDesc L = a.layer[l];
    f32x4 acc[4];
    init_bias<4>(acc, a, L, 0, lane);
    dense_regs<2, 4>(ah, al, a, L, acc, lane);
    store_rows<4>(s_x, LDX, L, 0, acc, lane, wave);
    wave_sync();
  }
  // h = F_out(f); the A operands of relu(h) stay in registers for the four
  // branches.  E1 acts on u_all = [h_mu | h_rot | h_scale | h_opacity]: it is
  // accumulated branch by branch from each h_g (E1's input columns 32g..), so
  // u_all is never stored.
  bf16x8 hh[2], hl[2];
  load_a<2, true>(s_x, LDX, hh, hl, lane, wave);
  float* tmp = s_x;
  // the canonical features this lane adds its updates to (first 128 columns),
  // loaded now so that their latency hides behind the branches
  constexpr int kZPre = 2;   // 64-column chunks
  float zpre[kZPre][4][4];
#pragma unroll
  for (int c = 0; c < kZPre; ++c)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = 64 * c + 16 * nt + (lane & 15);
        const int64_t g = g0 + 16 * wave + 4 * (lane >> 4) + v;
        zpre[c][nt][v] = (n < a.N && g < a.n) ? a.feat[g * a.N + n] : 0.f;
      }
  f32x4 e1[4];
  init_bias<4>(e1, a, a.layer[20], 0, lane);
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const int l = 8 + 3 * g;
    {
      f32x4 acc[4];
      init_bias<4>(acc, a, a.layer[l], 0, lane);
      dense_regs<2, 4>(hh, hl, a, a.layer[l], acc, lane);
      store_rows<4>(s_x, LDX, a.layer[l], 0, acc, lane, wave);
      wave_sync();
    }
    layer<kW, 2, true>(s_x, LDX, s_x, LDX, a, l + 1, lane, wave);          // h_g, in place
    layer<kW / 2, 1, true>(s_x, LDX, s_d + kDOff[g], kLdD, a, l + 2, lane, wave);
    dense<kW / 2, 4, false>(s_x, LDX, a, a.layer[20], 0, (kW / 2) * g, e1, lane, wave);
    wave_sync();   // h_g is overwritten by the next branch
  }
  store_rows<4>(s_x, LDX, a.layer[20], 0, e1, lane, wave);
  wave_sync();

  // 3. semantic update, written as z + dz, 64 columns at a time
  {
    const LayerDesc L = a.layer[21];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int n0 = 64 * c;
      if (n0 >= a.N) break;
      f32x4 acc[4];
      init_bias<4>(acc, a, L, n0, lane);
      dense<kW, 4, true>(tmp, LDX, a, L, n0, 0, acc, lane, wave);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int n = n0 + 16 * nt + (lane & 15);
        if (n < a.N) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t g = g0 + 16 * wave + 4 * (lane >> 4) + v;
            if (g < a.n) {
              const float z0 = c < kZPre ? zpre[c < kZPre ? c : 0][nt][v] : a.feat[g * a.N + n];
              const float z = z0 + acc[nt][v];
              if (a.out_bf16)
                static_cast<__bf16*>(a.out_feat)[g * a.N + n] = (__bf16)z;
              else
                static_cast<float*>(a.out_feat)[g * a.N + n] = z;
            }
          }
        }
      }
    }
  }
  // geometric updates: lane r < 16 of wave w writes Gaussian 16w + r
  if (lane < 16) {
    const int r = 16 * wave + lane;
    const int64_t g = g0 + r;
    if (g < a.n) {
      const float* d = s_d + r * kLdD;
#pragma unroll
      for (int k = 0; k < 3; ++k) a.out_means[g * 3 + k] = a.means[g * 3 + k] + d[kDOff[0] + k];
#pragma unroll
      for (int k = 0; k < 4; ++k) a.out_quats[g * 4 + k] = a.quats[g * 4 + k] + d[kDOff[1] + k];
#pragma unroll
      for (int k = 0; k < 3; ++k) a.out_scales[g * 3 + k] = expf(a.log_scales[g * 3 + k] + d[kDOff[2] + k]);
      a.out_opacity[g] = 1.f / (1.f + expf(-(a.logit_opacity[g] + d[kDOff[3]])));
    }
  }
}

struct DeformLayout {
  LayerDesc layer[kLayers];
  PlaneDesc plane[kPlanes];
  int64_t weight_floats, plane_floats, split_elems;
};

bool net_supported(const fe_deform_net* net) {
  if (!net) return false;
  if (net->channels != 32 && net->channels != 64) return false;
  if (net->width != kW) return false;
  if (net->feat_dim < 16 || net->feat_dim > 256 || net->feat_dim % 16 != 0) return false;
  for (int k = 0; k < 4; ++k) {
    if (net->base_res[k] < 2 || net->base_res[k] > 4096) return false;
    if (net->level_mult[k] < 1 || net->level_mult[k] > 64) return false;
  }
  return true;
}

DeformLayout make_layout(const fe_deform_net* net) {
  DeformLayout L{};
  const int W = net->width, C = net->channels, N = net->feat_dim;
  int io[kLayers][2];
  io[0][0] = 4 * C;
  io[0][1] = W;
  for (int l = 1; l < 8; ++l) io[l][0] = io[l][1] = W;
  for (int g = 0; g < 4; ++g) {
    io[8 + 3 * g][0] = W;
    io[8 + 3 * g][1] = W;
    io[9 + 3 * g][0] = W;
    io[9 + 3 * g][1] = W / 2;
    io[10 + 3 * g][0] = W / 2;
    io[10 + 3 * g][1] = kBranchDim[g];
  }
  io[20][0] = 2 * W;
  io[20][1] = W;
  io[21][0] = W;
  io[21][1] = N;
  int64_t w = 0, p = 0;
  for (int l = 0; l < kLayers; ++l) {
    LayerDesc& d = L.layer[l];
    d.in = io[l][0];
    d.out = io[l][1];
    d.out_pad = (d.out + 15) / 16 * 16;
    if (l == 21) d.out_pad = (d.out + 63) / 64 * 64;   // read in 64-column chunks
    d.w_off = w;
    d.b_off = w + (int64_t)d.out * d.in;
    w = d.b_off + d.out;
    d.p_off = p;
    p += (int64_t)d.out_pad * d.in;
  }
  L.weight_floats = w;
  L.split_elems = p;
  int64_t o = 0;
  for (int lv = 0; lv < 4; ++lv)
    for (int q = 0; q < 6; ++q) {
      const int a = pair_a(q), b = pair_b(q);
      const int ra = a < 3 ? net->base_res[a] * net->level_mult[lv] : net->base_res[a];
      const int rb = b < 3 ? net->base_res[b] * net->level_mult[lv] : net->base_res[b];
      PlaneDesc& d = L.plane[lv * 6 + q];
      d.off = o;
      d.ra = ra;
      d.rb = rb;
      o += (int64_t)ra * rb * C;
    }
  L.plane_floats = o;
  return L;
}

fe_status hip_to_status(hipError_t e) { return e == hipSuccess ? FE_OK : FE_ERR_HIP; }

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" {

size_t fe_deform_plane_floats(const fe_deform_net* net) {
  return net_supported(net) ? (size_t)make_layout(net).plane_floats : 0;
}

size_t fe_deform_weight_floats(const fe_deform_net* net) {
  return net_supported(net) ? (size_t)make_layout(net).weight_floats : 0;
}

size_t fe_deform_workspace_bytes(const fe_deform_net* net) {
  if (!net_supported(net)) return 0;
  const int64_t e = make_layout(net).split_elems;
  return 2 * (((size_t)e * sizeof(__bf16) + 255) & ~(size_t)255);
}

fe_status fe_deform_forward(const fe_deform_net* net, const fe_deform_io* io, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!net || !io) return FE_ERR_INVALID_ARG;
  if (!net_supported(net)) return FE_ERR_UNSUPPORTED;
  if (io->n < 0 || io->n > ((int64_t)1 << 40)) return FE_ERR_INVALID_ARG;
  if (io->out_feat_dtype != FE_F32 && io->out_feat_dtype != FE_BF16) return FE_ERR_INVALID_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(net->hi[k] > net->lo[k])) return FE_ERR_INVALID_ARG;
  if (!(io->t == io->t)) return FE_ERR_INVALID_ARG;
  if (!net->planes || !net->weights || !workspace) return FE_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0 || reinterpret_cast<uintptr_t>(net->planes) % 16 != 0)
    return FE_ERR_INVALID_ARG;
  if (workspace_bytes < fe_deform_workspace_bytes(net)) return FE_ERR_WORKSPACE_TOO_SMALL;
  if (io->n == 0) return FE_OK;
  if (!io->means || !io->quats || !io->log_scales || !io->logit_opacity || !io->feat || !io->out_means ||
      !io->out_quats || !io->out_scales || !io->out_opacity || !io->out_feat)
    return FE_ERR_INVALID_ARG;
  const DeformLayout L = make_layout(net);
  DeformArgs a{};
  for (int l = 0; l < kLayers; ++l) a.layer[l] = L.layer[l];
  for (int q = 0; q < kPlanes; ++q) a.plane[q] = L.plane[q];
  a.planes = net->planes;
  a.weights = net->weights;
  const size_t part = (((size_t)L.split_elems * sizeof(__bf16) + 255) & ~(size_t)255);
  a.whi = static_cast<const __bf16*>(workspace);
  a.wlo = reinterpret_cast<const __bf16*>(static_cast<const char*>(workspace) + part);
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = (double)net->lo[k];
    a.hi[k] = (double)net->hi[k];
  }
  const double ut = 2.0 * (double)io->t - 1.0;
  a.ut = ut < -1.0 ? -1.0 : (ut > 1.0 ? 1.0 : ut);
  a.n = io->n;
  a.N = net->feat_dim;
  a.out_bf16 = io->out_feat_dtype == FE_BF16;
  a.means = io->means;
  a.quats = io->quats;
  a.log_scales = io->log_scales;
  a.logit_opacity = io->logit_opacity;
  a.feat = io->feat;
  a.out_means = io->out_means;
  a.out_quats = io->out_quats;
  a.out_scales = io->out_scales;
  a.out_opacity = io->out_opacity;
  a.out_feat = io->out_feat;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(deform_prep_kernel, dim3((unsigned)((L.split_elems + 255) / 256)), dim3(256), 0, s, a,
                     L.split_elems);
  const unsigned grid = (unsigned)((io->n + kRows - 1) / kRows);
  if (net->channels == 32)
    hipLaunchKernelGGL(deform_kernel<32>, dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(deform_kernel<64>, dim3(grid), dim3(kThreads), 0, s, a);
  return hip_to_status(hipGetLastError());
}

}  // extern "C"
