// Per-tile front-to-back blending of colour and D feature channels
// (eqs. 7 and 8 share the weights alpha_i prod_{j<i}(1 - alpha_j)), and its
// backward.
//
// One workgroup per tile, one pixel per lane.  The tile's depth-ordered list
// is walked in batches staged in LDS (pixel position, conic, opacity, colour,
// pixel box, and the batch's feature rows widened to float32).  A wave whose
// lanes have all stopped skips the rest of a batch, and the workgroup leaves
// the list once every lane has stopped (barrier count at batch boundaries).
//
// The alpha of a (pixel, Gaussian) pair is evaluated by the same inline
// function in both directions, so the backward re-derives exactly the
// forward's skip decisions; n_contrib bounds its walk and the forward's final
// transmittance seeds the back-to-front recovery T_i = T_{i+1} / (1 - alpha_i).
#include "fe_common.h"

#pragma clang fp contract(off)

namespace fe {
namespace {

struct CompArgs {
  const uint2* ranges;
  const uint32_t* gauss;     // sorted Gaussian index per key
  const float2* xy;
  const float4* conic_o;
  const float4* rgb;
  const short4* box;
  const void* feat;          // [n][D] float or bf16
  float* out_rgb;            // [3][H][W]
  float* out_feat;           // [D][H][W]
  float* out_T;              // [H][W]
  int32_t* out_n;            // [H][W]
  float* out_depth;          // [H][W] or null
  // backward
  const float* d_rgb;
  const float* d_feat;
  const float* d_depth;      // [H][W] or null
  float* grad2d;             // [n][12]
  float* grad_feat;          // [n][D]
  uint32_t* tile_maxlast;    // [tiles]
  unsigned long long* report;
  float bg[3];
  int32_t W, H, tile_w, tiles_x;
  int32_t D;                 // real feature count
};

// Alpha of one (pixel, Gaussian) pair; returns false when the pair is
// skipped (outside the box, q > 9, alpha < 1/255).
__device__ __forceinline__ bool pair_alpha(float fpx, float fpy, int px, int py, float2 m, float4 co, float tg,
                                           int4 b, float& dx, float& dy, float& G, float& alpha) {
  dx = fpx - m.x;
  dy = fpy - m.y;
  // the same expression as the matrix-core kernels, so every variant gives
  // bit-identical images
  const float qs = scaled_q(scale_conic(co), dx, dy);
  const bool inb = (px >= b.x) & (px <= b.z) & (py >= b.y) & (py <= b.w);
  if (!(inb && qs >= tg)) return false;
  G = __builtin_amdgcn_exp2f(qs);
  alpha = fminf(kAlphaMax, co.w * G);
  return true;
}

template <typename FT>
__device__ __forceinline__ float feat_at(const void* p, int64_t i) {
  return load_as_float<FT>(p, i);
}

template <int D, typename FT, int NT, int NB>
__device__ __forceinline__ void stage_batch(const CompArgs& a, uint32_t b0, int nb, float2* s_xy, float4* s_co, float* s_tg,
                                            float4* s_rgb, int4* s_box, uint32_t* s_gid, float* s_f) {
  for (int t = threadIdx.x; t < nb; t += NT) {
    const uint32_t g = a.gauss[b0 + t];
    s_gid[t] = g;
    s_xy[t] = a.xy[g];
    const float4 co = a.conic_o[g];
    s_co[t] = co;
    s_tg[t] = blend_cut(co.w);
    s_rgb[t] = a.rgb[g];
    const short4 b = a.box[g];
    s_box[t] = make_int4(b.x, b.y, b.z, b.w);
  }
  constexpr int G4 = D / 4 > 0 ? D / 4 : 1;
  for (int e = threadIdx.x; e < nb * G4; e += NT) {
    const int j = e / G4;
    const int c = (e % G4) * 4;
    const int64_t g = a.gauss[b0 + j];
    float4 v;
    v.x = c + 0 < a.D ? feat_at<FT>(a.feat, g * a.D + c + 0) : 0.f;
    v.y = c + 1 < a.D ? feat_at<FT>(a.feat, g * a.D + c + 1) : 0.f;
    v.z = c + 2 < a.D ? feat_at<FT>(a.feat, g * a.D + c + 2) : 0.f;
    v.w = c + 3 < a.D ? feat_at<FT>(a.feat, g * a.D + c + 3) : 0.f;
    *reinterpret_cast<float4*>(s_f + j * D + c) = v;
  }
}

template <int D>
constexpr int batch_size() { return D >= 256 ? 32 : 64; }

template <int D, typename FT, int NT>
__global__ __launch_bounds__(NT) void composite_fwd_kernel(CompArgs a) {
  constexpr int NB = batch_size<D>();
  __shared__ float2 s_xy[NB];
  __shared__ float4 s_co[NB];
  __shared__ float s_tg[NB];
  __shared__ float4 s_rgb[NB];
  __shared__ int4 s_box[NB];
  __shared__ uint32_t s_gid[NB];
  __shared__ __attribute__((aligned(16))) float s_f[NB * D];
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tile_h = NT / a.tile_w;
  const int px = (tile % a.tiles_x) * a.tile_w + (int)threadIdx.x % a.tile_w;
  const int py = (tile / a.tiles_x) * tile_h + (int)threadIdx.x / a.tile_w;
  const bool inside = (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const uint2 rg = a.ranges[tile];
  float T = 1.0f;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, C3 = 0.f;   // colour, depth
  float Z[D];
#pragma unroll
  for (int k = 0; k < D; ++k) Z[k] = 0.f;
  int last = 0;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += NB) {
    const int nb = (int)min((uint32_t)NB, rg.y - b0);
    if (__syncthreads_count(!done) == 0) break;
    stage_batch<D, FT, NT, NB>(a, b0, nb, s_xy, s_co, s_tg, s_rgb, s_box, s_gid, s_f);
    __syncthreads();
    if (!done) {
      for (int j = 0; j < nb; ++j) {
        float dx, dy, G, alpha;
        if (!pair_alpha(fpx, fpy, px, py, s_xy[j], s_co[j], s_tg[j], s_box[j], dx, dy, G, alpha)) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < kTStop) {
          done = true;
          break;
        }
        const float w = alpha * T;
        const float4 c = s_rgb[j];
        C0 = __builtin_fmaf(w, c.x, C0);
        C1 = __builtin_fmaf(w, c.y, C1);
        C2 = __builtin_fmaf(w, c.z, C2);
        C3 = __builtin_fmaf(w, c.w, C3);
        const float4* f4 = reinterpret_cast<const float4*>(s_f + j * D);
#pragma unroll
        for (int k4 = 0; k4 < D / 4; ++k4) {
          const float4 f = f4[k4];
          Z[4 * k4 + 0] = __builtin_fmaf(w, f.x, Z[4 * k4 + 0]);
          Z[4 * k4 + 1] = __builtin_fmaf(w, f.y, Z[4 * k4 + 1]);
          Z[4 * k4 + 2] = __builtin_fmaf(w, f.z, Z[4 * k4 + 2]);
          Z[4 * k4 + 3] = __builtin_fmaf(w, f.w, Z[4 * k4 + 3]);
        }
        T = Tn;
        last = (int)(b0 - rg.x) + j + 1;
      }
    }
  }
  if (inside) {
    const int64_t HW = (int64_t)a.W * a.H;
    const int64_t p = (int64_t)py * a.W + px;
    a.out_rgb[p] = __builtin_fmaf(T, a.bg[0], C0);
    a.out_rgb[HW + p] = __builtin_fmaf(T, a.bg[1], C1);
    a.out_rgb[2 * HW + p] = __builtin_fmaf(T, a.bg[2], C2);
    if (a.out_depth) a.out_depth[p] = C3;
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k < a.D) a.out_feat[k * HW + p] = Z[k];
    a.out_T[p] = T;
    a.out_n[p] = last;
  }
  // per-tile walk length (sizes the matrix-core backward's partial rows)
  __shared__ int s_maxlast;
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  if (last > 0) atomicMax(&s_maxlast, last);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.tile_maxlast[tile] = (uint32_t)s_maxlast;
    if (s_maxlast > 0) atomicAdd(&a.report[kRepRows], (unsigned long long)s_maxlast);
  }
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int D, typename FT, int NT>
__global__ __launch_bounds__(NT) void composite_bwd_kernel(CompArgs a) {
  constexpr int NB = batch_size<D>();
  __shared__ float2 s_xy[NB];
  __shared__ float4 s_co[NB];
  __shared__ float s_tg[NB];
  __shared__ float4 s_rgb[NB];
  __shared__ int4 s_box[NB];
  __shared__ uint32_t s_gid[NB];
  __shared__ __attribute__((aligned(16))) float s_f[NB * D];
  __shared__ int s_maxlast;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tile_h = NT / a.tile_w;
  const int px = (tile % a.tiles_x) * a.tile_w + (int)threadIdx.x % a.tile_w;
  const int py = (tile / a.tiles_x) * tile_h + (int)threadIdx.x / a.tile_w;
  const bool inside = (px < a.W) & (py < a.H);
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const uint2 rg = a.ranges[tile];
  const int64_t HW = (int64_t)a.W * a.H;
  const int64_t p = (int64_t)py * a.W + px;
  float gr[4] = {0.f, 0.f, 0.f, 0.f};   // colour, depth
  float gf[D];
#pragma unroll
  for (int k = 0; k < D; ++k) gf[k] = 0.f;
  float T = 1.0f;
  int last = 0;
  if (inside) {
    gr[0] = a.d_rgb[p];
    gr[1] = a.d_rgb[HW + p];
    gr[2] = a.d_rgb[2 * HW + p];
    gr[3] = a.d_depth ? a.d_depth[p] : 0.f;
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k < a.D) gf[k] = a.d_feat[k * HW + p];
    T = a.out_T[p];
    last = a.out_n[p];
  }
  // running sum over the Gaussians behind: sum_{j>i} w_j s_j + T_final s_bg
  float acc = T * ((gr[0] * a.bg[0] + gr[1] * a.bg[1]) + gr[2] * a.bg[2]);
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  if (last > 0) atomicMax(&s_maxlast, last);
  __syncthreads();
  const uint32_t end = min(rg.y, rg.x + (uint32_t)s_maxlast);
  const int lane = threadIdx.x & 63;
  for (uint32_t b1 = end; b1 > rg.x;) {
    const uint32_t b0 = b1 - rg.x > (uint32_t)NB ? b1 - NB : rg.x;
    const int nb = (int)(b1 - b0);
    __syncthreads();
    stage_batch<D, FT, NT, NB>(a, b0, nb, s_xy, s_co, s_tg, s_rgb, s_box, s_gid, s_f);
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const int pos = (int)(b0 - rg.x) + j;
      float dx = 0.f, dy = 0.f, G = 0.f, alpha = 0.f;
      bool contrib = false;
      if (inside && pos < last) contrib = pair_alpha(fpx, fpy, px, py, s_xy[j], s_co[j], s_tg[j], s_box[j], dx, dy, G, alpha);
      if (__ballot(contrib) == 0ull) continue;
      float v[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      float w = 0.f;
      if (contrib) {
        const float om = 1.0f - alpha;
        T = T / om;
        w = alpha * T;
        const float4 c = s_rgb[j];
        float s = ((gr[0] * c.x + gr[1] * c.y) + gr[2] * c.z) + gr[3] * c.w;
        const float4* f4 = reinterpret_cast<const float4*>(s_f + j * D);
#pragma unroll
        for (int k4 = 0; k4 < D / 4; ++k4) {
          const float4 f = f4[k4];
          s = __builtin_fmaf(gf[4 * k4 + 0], f.x, s);
          s = __builtin_fmaf(gf[4 * k4 + 1], f.y, s);
          s = __builtin_fmaf(gf[4 * k4 + 2], f.z, s);
          s = __builtin_fmaf(gf[4 * k4 + 3], f.w, s);
        }
        const float dalpha = T * s - acc / om;
        acc = __builtin_fmaf(w, s, acc);
        v[6] = w * gr[0];
        v[7] = w * gr[1];
        v[8] = w * gr[2];
        v[9] = w * gr[3];
        const float4 co = s_co[j];
        const float opG = co.w * G;
        if (opG <= kAlphaMax) {
          v[5] = G * dalpha;
          const float dq = -0.5f * opG * dalpha;
          v[2] = dq * dx * dx;
          v[3] = dq * 2.0f * dx * dy;
          v[4] = dq * dy * dy;
          v[0] = -2.0f * dq * (co.x * dx + co.y * dy);
          v[1] = -2.0f * dq * (co.y * dx + co.z * dy);
        }
      }
      const uint32_t g = s_gid[j];
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        const float r = wave_sum(v[k]);
        if (lane == 0 && r != 0.f) atomicAdd(a.grad2d + (int64_t)g * 12 + k, r);
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if (k < a.D) {
          const float r = wave_sum(w * gf[k]);
          if (lane == 0 && r != 0.f) atomicAdd(a.grad_feat + (int64_t)g * a.D + k, r);
        }
      }
    }
    b1 = b0;
  }
}

template <int D, typename FT>
hipError_t launch_fwd_nt(int nt, const CompArgs& a, int tiles, hipStream_t s) {
  switch (nt) {
    case 64: hipLaunchKernelGGL((composite_fwd_kernel<D, FT, 64>), dim3(tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL((composite_fwd_kernel<D, FT, 128>), dim3(tiles), dim3(128), 0, s, a); break;
    default: hipLaunchKernelGGL((composite_fwd_kernel<D, FT, 256>), dim3(tiles), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

template <int D, typename FT>
hipError_t launch_bwd_nt(int nt, const CompArgs& a, int tiles, hipStream_t s) {
  switch (nt) {
    case 64: hipLaunchKernelGGL((composite_bwd_kernel<D, FT, 64>), dim3(tiles), dim3(64), 0, s, a); break;
    case 128: hipLaunchKernelGGL((composite_bwd_kernel<D, FT, 128>), dim3(tiles), dim3(128), 0, s, a); break;
    default: hipLaunchKernelGGL((composite_bwd_kernel<D, FT, 256>), dim3(tiles), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

template <typename FT, bool BWD>
hipError_t dispatch_d(int D, int nt, const CompArgs& a, int tiles, hipStream_t s) {
#define FE_CASE(DP) \
  if (D <= DP) return BWD ? launch_bwd_nt<DP, FT>(nt, a, tiles, s) : launch_fwd_nt<DP, FT>(nt, a, tiles, s);
  FE_CASE(4)
  FE_CASE(8)
  FE_CASE(16)
  FE_CASE(32)
  FE_CASE(64)
  FE_CASE(128)
  FE_CASE(256)
#undef FE_CASE
  return hipErrorInvalidValue;
}

CompArgs make_args(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const StateView& v) {
  CompArgs a{};
  a.ranges = v.ranges;
  a.gauss = v.gauss;
  a.xy = v.xy;
  a.conic_o = v.conic_o;
  a.rgb = v.rgb;
  a.box = v.box;
  a.feat = g->feat;
  a.tile_maxlast = v.tile_maxlast;
  a.report = v.report;
  for (int k = 0; k < 3; ++k) a.bg[k] = cfg->bg_rgb[k];
  a.W = cam->width;
  a.H = cam->height;
  a.tile_w = cfg->tile_w;
  a.tiles_x = v.tiles_x;
  a.D = cfg->feat_dim;
  return a;
}

}  // namespace

hipError_t launch_composite_fwd(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                const StateView& v, const fe_images* out, hipStream_t s) {
  CompArgs a = make_args(cfg, cam, g, v);
  a.out_rgb = out->rgb;
  a.out_feat = out->feat;
  a.out_T = out->final_T;
  a.out_n = out->n_contrib;
  a.out_depth = out->depth;
  const int nt = cfg->tile_w * cfg->tile_h;
  return cfg->feat_dtype == FE_BF16 ? dispatch_d<uint16_t, false>(cfg->feat_dim, nt, a, v.tiles, s)
                                    : dispatch_d<float, false>(cfg->feat_dim, nt, a, v.tiles, s);
}

hipError_t launch_composite_bwd(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                const StateView& v, const fe_images* fwd, const float* d_rgb,
                                const float* d_feat, const float* d_depth, float* grad2d, float* grad_feat,
                                hipStream_t s) {
  CompArgs a = make_args(cfg, cam, g, v);
  a.out_T = fwd->final_T;
  a.out_n = fwd->n_contrib;
  a.d_rgb = d_rgb;
  a.d_feat = d_feat;
  a.d_depth = d_depth;
  a.grad2d = grad2d;
  a.grad_feat = grad_feat;
  const int nt = cfg->tile_w * cfg->tile_h;
  return cfg->feat_dtype == FE_BF16 ? dispatch_d<uint16_t, true>(cfg->feat_dim, nt, a, v.tiles, s)
                                    : dispatch_d<float, true>(cfg->feat_dim, nt, a, v.tiles, s);
}

}  // namespace fe
