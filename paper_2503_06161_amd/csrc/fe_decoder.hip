// Semantic decoder and feature loss, fused (Sec. 3.3, eq. 10), on the matrix
// cores of gfx950.
//
// The rendered feature map z [D][P] (planar, P = H W pixels) goes through
// the pointwise convolution z' = W z + b (W [C][D], C = 256) and is compared
// with the target map t [C][P] by L = (1/P) sum_x |z'(x) - t(x)|_1.  One
// pass over the pixels gives the loss and every gradient: with
// s = sign(z' - t) (sign(0) = 0),
//   dL/dz = W^T s / P,   dL/dW = s z^T / P,   dL/db = sum_x s / P,
// so dL/dz can feed the rasterizer's backward directly.
//
// Two passes over 32-pixel blocks, workgroups of 8 waves:
//   pass 1  decode z'[C x 32] = W z (wave w owns output rows 32w..32w+31:
//           A = its W rows in registers, B = the z block from LDS; 32x32x16
//           MFMAs); residual, loss and sign; the signs of each row are kept
//           as two 32-bit masks per block (2 bits per value); dW [C x D] +=
//           s z^T accumulated in registers over the workgroup's blocks, db as
//           counts of positive minus negative signs;
//   pass 2  dz [D x 32] = W^T s from the masks (16x16x32 MFMAs, A = W^T
//           columns in registers, B = signs expanded into LDS).
// Splitting dz off keeps each pass's resident operands (W rows + dW
// accumulators, W^T columns) within the register file; the masks cost
// 2 bits per output value each way.
// Exactness: float32 operands are split into bf16 parts (x = hi + lo + ...);
// signs are exact bf16.  The decode keeps the products of order <= 1 of
// two-part splits of W and z (about 16 significant bits per product); dz and
// dW multiply exact signs by two-part splits (the same).  Each workgroup
// writes its partial dW, db and loss; a second kernel adds them up.
#include "fe_common.h"

#include <type_traits>

#pragma clang fp contract(off)

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 256;              // decoder output channels
constexpr int kPB = 32;              // pixels per block
constexpr int kDecThreads = 512;     // 8 waves

struct DecArgs {
  const float* feat;      // [D][P]
  const float* weight;    // [C][D]
  const float* bias;      // [C]
  const void* target;     // [C][P] float or bf16 bits
  float* decoded;         // [C][P] or null
  float* d_feat;          // [D][P] or null
  uint2* signs;           // [C][blocks]: (nonzero mask, negative mask) of 32 pixels
  float* partial;         // [grid][C D + C + 1]: dW, db, loss of each workgroup
  int64_t P;
  float inv_p;            // 1 / P
};

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

template <typename TT>
__device__ __forceinline__ const void* target_base(const void* t, int64_t i) {
  return static_cast<const TT*>(t) + i;
}

template <typename TT>
__device__ __forceinline__ float target_at(const void* t, uint32_t i) {
  if constexpr (std::is_same<TT, float>::value)
    return static_cast<const float*>(t)[i];
  else
    return __uint_as_float((uint32_t)static_cast<const uint16_t*>(t)[i] << 16);
}

// Pass 1: decode, residual, loss, signs, dW and db.  Wave w owns output rows
// 32w..32w+31 in every step, so the only data shared between waves is the z
// block.
template <int KIN, typename TT>
__global__ __launch_bounds__(kDecThreads) void decoder_pass1_kernel(DecArgs a) {
  constexpr int KS = KIN / 16;        // k steps of the decode (32x32x16)
  constexpr int NBW = KIN / 32;       // 32-column blocks of dW
  constexpr int ZR = kPB + 8;         // padded rows of the channel-major z tile
  constexpr int ZT = KIN + 8;         // padded rows of the pixel-major z tile
  constexpr int SR = kPB + 8;
  __shared__ __attribute__((aligned(16))) __bf16 s_zc[2][KIN][ZR];   // z[c][px], hi / lo
  __shared__ __attribute__((aligned(16))) __bf16 s_zt[2][kPB][ZT];   // z[px][c], hi / lo
  __shared__ __attribute__((aligned(16))) __bf16 s_sc[kC][SR];       // sign[c][px] (each wave its own rows)
  __shared__ float s_bias[kC];
  __shared__ float s_red[kDecThreads / 64];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int64_t P = a.P;
  const int64_t nblocks = (P + kPB - 1) / kPB;
  for (int c = threadIdx.x; c < kC; c += kDecThreads) s_bias[c] = a.bias[c];

  // W rows of this wave (decode A operand), hi / lo, loaded once
  bf16x8 wa[KS][2];
  {
    const float* wr = a.weight + (int64_t)(32 * wave + (lane & 31)) * KIN + 8 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float4 x0 = *reinterpret_cast<const float4*>(wr + 16 * ks);
      const float4 x1 = *reinterpret_cast<const float4*>(wr + 16 * ks + 4);
      const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 h, l;
        split2(xs[j], h, l);
        wa[ks][0][j] = h;
        wa[ks][1][j] = l;
      }
    }
  }
  f32x16 dw[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) dw[nb] = f32x16{};
  int cnt = 0;            // lane l < 32: (positive - negative) signs of row 32 wave + l
  float loss = 0.f;

  // z block loads: element e = threadIdx.x + 512 i covers channel e / 32, pixel e % 32
  constexpr int ZI = (KIN * kPB + kDecThreads - 1) / kDecThreads;
  float zn[ZI];
  auto load_z = [&](int64_t blk) {
#pragma unroll
    for (int i = 0; i < ZI; ++i) {
      const int e = threadIdx.x + kDecThreads * i;
      const int c = e / kPB, px = e % kPB;
      const int64_t p = blk * kPB + px;
      zn[i] = (e < KIN * kPB && blk < nblocks && p < P) ? a.feat[(int64_t)c * P + p] : 0.f;
    }
  };
  load_z(blockIdx.x);
  __syncthreads();   // s_bias
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t p0 = blk * kPB;
    // z block to LDS (both layouts, hi / lo); the next block's loads go out
#pragma unroll
    for (int i = 0; i < ZI; ++i) {
      const int e = threadIdx.x + kDecThreads * i;
      if (e < KIN * kPB) {
        const int c = e / kPB, px = e % kPB;
        __bf16 h, l;
        split2(zn[i], h, l);
        s_zc[0][c][px] = h;
        s_zc[1][c][px] = l;
        s_zt[0][px][c] = h;
        s_zt[1][px][c] = l;
      }
    }
    load_z(blk + gridDim.x);
    __syncthreads();
    // decode: rows 32 wave.. x the block's 32 pixels
    f32x16 acc = f32x16{};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kc = 16 * ks + 8 * (lane >> 5);
      const bf16x8 zh = *reinterpret_cast<const bf16x8*>(&s_zt[0][lane & 31][kc]);
      const bf16x8 zl = *reinterpret_cast<const bf16x8*>(&s_zt[1][lane & 31][kc]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ks][0], zh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ks][0], zl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ks][1], zh, acc, 0, 0, 0);
    }
    // residual, loss and sign of each (row, pixel); the signs of a row's 32
    // pixels become two 32-bit masks (lane l holds pixel l % 32)
    // Element (row 32 wave + r, pixel p0 + q) sits at base + r P + q: a
    // wave-uniform 64-bit base and a 32-bit offset (pixels < 2^25).  Lanes
    // past the last pixel read that pixel and contribute nothing.
    const int px = lane & 31;
    const bool inside = p0 + px < P;
    const int64_t base = (int64_t)(32 * wave_u) * P + p0;
    const uint32_t off0 =
        (uint32_t)(4 * (lane >> 5)) * (uint32_t)P + (uint32_t)(inside ? px : (int)(P - 1 - p0));
    const void* tb = target_base<TT>(a.target, base);
    float dec[16], tv[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t off = off0 + (uint32_t)(8 * (v >> 2) + (v & 3)) * (uint32_t)P;
      tv[v] = target_at<TT>(tb, off);
      dec[v] = acc[v] + s_bias[32 * wave + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)];
    }
    if (a.decoded && inside) {
#pragma unroll
      for (int v = 0; v < 16; ++v)
        (a.decoded + base)[off0 + (uint32_t)(8 * (v >> 2) + (v & 3)) * (uint32_t)P] = dec[v];
    }
    uint2 mk = make_uint2(0u, 0u);   // lane v < 16: masks of row c(v); lane 16 + v: of row c(v) + 4
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 32 * wave + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      const float r = inside ? dec[v] - tv[v] : 0.f;
      loss += fabsf(r);
      const float s = r > 0.f ? 1.f : (r < 0.f ? -1.f : 0.f);
      s_sc[c][px] = (__bf16)s;
      const unsigned long long nz = __ballot(s != 0.f), ng = __ballot(s < 0.f);
      if (lane == v) mk = make_uint2((uint32_t)nz, (uint32_t)ng);
      if (lane == 16 + v) mk = make_uint2((uint32_t)(nz >> 32), (uint32_t)(ng >> 32));
      // row counts: rows c (lanes 0..31 of the ballot) and c + 4 (lanes 32..63)
      const int pos_lo = __popc((uint32_t)nz & ~(uint32_t)ng), neg_lo = __popc((uint32_t)nz & (uint32_t)ng);
      const int pos_hi = __popc((uint32_t)(nz >> 32) & ~(uint32_t)(ng >> 32));
      const int neg_hi = __popc((uint32_t)(nz >> 32) & (uint32_t)(ng >> 32));
      const int r0 = 8 * (v >> 2) + (v & 3);
      if (lane == r0) cnt += pos_lo - neg_lo;
      if (lane == r0 + 4) cnt += pos_hi - neg_hi;
    }
    if (lane < 32) {
      const int v = lane & 15;
      const int row = 32 * wave + 8 * (v >> 2) + (v & 3) + 4 * (lane >> 4);
      a.signs[(int64_t)row * nblocks + blk] = mk;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW += s z^T over the block's pixels (rows of this wave only)
#pragma unroll
    for (int ks = 0; ks < kPB / 16; ++ks) {
      const int kp = 16 * ks + 8 * (lane >> 5);
      const bf16x8 sa = *reinterpret_cast<const bf16x8*>(&s_sc[32 * wave + (lane & 31)][kp]);
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const bf16x8 zh = *reinterpret_cast<const bf16x8*>(&s_zc[0][32 * nb + (lane & 31)][kp]);
        const bf16x8 zl = *reinterpret_cast<const bf16x8*>(&s_zc[1][32 * nb + (lane & 31)][kp]);
        dw[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa, zh, dw[nb], 0, 0, 0);
        dw[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa, zl, dw[nb], 0, 0, 0);
      }
    }
    __syncthreads();   // the z tiles are rewritten by the next block
  }
  // partial results of this workgroup
  float* out = a.partial + (int64_t)blockIdx.x * (kC * KIN + kC + 1);
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 32 * wave + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
      out[(int64_t)c * KIN + 32 * nb + (lane & 31)] = dw[nb][v] * a.inv_p;
    }
  if (lane < 32) out[kC * KIN + 32 * wave + lane] = (float)cnt * a.inv_p;
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (lane == 0) s_red[wave] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    float l = 0.f;
    for (int w = 0; w < kDecThreads / 64; ++w) l += s_red[w];
    out[kC * KIN + kC] = l * a.inv_p;
  }
}

// Pass 2: dz = W^T s / P from the sign masks (16x16x32; a unit is 16 input
// channels x 16 pixels, and wave w keeps the W^T columns of its units).
template <int KIN>
__global__ __launch_bounds__(kDecThreads) void decoder_pass2_kernel(DecArgs a) {
  constexpr int MB = KIN / 16;
  constexpr int NU = 2 * MB;
  constexpr int UPW = NU > 8 ? NU / 8 : 1;
  constexpr int ST = kC + 8;
  __shared__ __attribute__((aligned(16))) __bf16 s_st[kPB][ST];      // sign[px][c]
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t P = a.P;
  const int64_t nblocks = (P + kPB - 1) / kPB;
  const int u0 = wave % NU;
  const bool has_dz = wave < NU;
  const int mblk = u0 % MB;   // the units of a wave share one row block
  bf16x8 wt[kC / 32][2];
  {
    const int ic = 16 * mblk + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < kC / 32; ++ks)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
        if (has_dz) split2(a.weight[(int64_t)(32 * ks + 8 * (lane >> 4) + j) * KIN + ic], h, l);
        wt[ks][0][j] = h;
        wt[ks][1][j] = l;
      }
  }
  uint2 mk_n = make_uint2(0u, 0u);
  auto load_masks = [&](int64_t blk) {
    mk_n = (threadIdx.x < kC && blk < nblocks) ? a.signs[(int64_t)threadIdx.x * nblocks + blk] : make_uint2(0u, 0u);
  };
  load_masks(blockIdx.x);
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t p0 = blk * kPB;
    // thread c < 256 expands the masks of row c into the sign tile, two
    // pixels per 4-byte store would straddle rows: one bf16 per pixel
    if (threadIdx.x < kC) {
      const uint2 m = mk_n;
#pragma unroll
      for (int q = 0; q < kPB; ++q) {
        const float s = ((m.x >> q) & 1u) ? (((m.y >> q) & 1u) ? -1.f : 1.f) : 0.f;
        s_st[q][threadIdx.x] = (__bf16)s;
      }
    }
    load_masks(blk + gridDim.x);
    __syncthreads();
    if (has_dz) {
#pragma unroll
      for (int k = 0; k < UPW; ++k) {
        const int nblk = (u0 + 8 * k) / MB;
        f32x4 d = f32x4{};
#pragma unroll
        for (int ks = 0; ks < kC / 32; ++ks) {
          const bf16x8 sb = *reinterpret_cast<const bf16x8*>(&s_st[16 * nblk + (lane & 15)][32 * ks + 8 * (lane >> 4)]);
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[ks][0], sb, d, 0, 0, 0);
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt[ks][1], sb, d, 0, 0, 0);
        }
        const int64_t pp = p0 + 16 * nblk + (lane & 15);
        if (pp < P) {
#pragma unroll
          for (int v = 0; v < 4; ++v) a.d_feat[(int64_t)(16 * mblk + 4 * (lane >> 4) + v) * P + pp] = d[v] * a.inv_p;
        }
      }
    }
    __syncthreads();   // the sign tile is rewritten by the next block
  }
}

// Sum of the workgroups' partials: one thread per output value.
__global__ __launch_bounds__(256) void decoder_reduce_kernel(const float* partial, int groups, int n, float* d_weight,
                                                             float* d_bias, float* loss, int nw) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int g = 0; g < groups; ++g) s += partial[(int64_t)g * n + i];
  if (i < nw)
    d_weight[i] = s;
  else if (i < n - 1)
    d_bias[i - nw] = s;
  else
    loss[0] = s;
}

template <int KIN, typename TT>
static int decoder_grid() {
  int per_cu = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decoder_pass1_kernel<KIN, TT>, kDecThreads, 0) !=
      hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
}

template <int KIN, typename TT>
static hipError_t launch_kin(const DecArgs& a0, int grid, float* d_weight, float* d_bias, float* loss,
                             hipStream_t s) {
  DecArgs a = a0;
  hipLaunchKernelGGL((decoder_pass1_kernel<KIN, TT>), dim3(grid), dim3(kDecThreads), 0, s, a);
  if (a.d_feat) hipLaunchKernelGGL((decoder_pass2_kernel<KIN>), dim3(grid), dim3(kDecThreads), 0, s, a);
  const int n = kC * KIN + kC + 1;
  hipLaunchKernelGGL(decoder_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a.partial, grid, n, d_weight,
                     d_bias, loss, kC * KIN);
  return hipGetLastError();
}

}  // namespace

int decoder_grid_size(int in_dim, int target_dtype) {
  const bool bf = target_dtype == FE_BF16;
  switch (in_dim) {
    case 32: return bf ? decoder_grid<32, uint16_t>() : decoder_grid<32, float>();
    case 64: return bf ? decoder_grid<64, uint16_t>() : decoder_grid<64, float>();
    default: return bf ? decoder_grid<128, uint16_t>() : decoder_grid<128, float>();
  }
}

size_t decoder_partial_floats(int in_dim) { return (size_t)kC * in_dim + kC + 1; }

size_t decoder_sign_bytes(int64_t pixels) { return (size_t)kC * (size_t)((pixels + kPB - 1) / kPB) * sizeof(uint2); }

hipError_t launch_decoder_l1(const fe_decoder* d, int grid, float* partial, void* signs, hipStream_t s) {
  DecArgs a{};
  a.signs = static_cast<uint2*>(signs);
  a.feat = d->feat;
  a.weight = d->weight;
  a.bias = d->bias;
  a.target = d->target;
  a.decoded = d->decoded;
  a.d_feat = d->d_feat;
  a.partial = partial;
  a.P = d->pixels;
  a.inv_p = (float)(1.0 / (double)d->pixels);
  const bool bf = d->target_dtype == FE_BF16;
  switch (d->in_dim) {
    case 32:
      return bf ? launch_kin<32, uint16_t>(a, grid, d->d_weight, d->d_bias, d->loss, s)
                : launch_kin<32, float>(a, grid, d->d_weight, d->d_bias, d->loss, s);
    case 64:
      return bf ? launch_kin<64, uint16_t>(a, grid, d->d_weight, d->d_bias, d->loss, s)
                : launch_kin<64, float>(a, grid, d->d_weight, d->d_bias, d->loss, s);
    default:
      return bf ? launch_kin<128, uint16_t>(a, grid, d->d_weight, d->d_bias, d->loss, s)
                : launch_kin<128, float>(a, grid, d->d_weight, d->d_bias, d->loss, s);
  }
}

}  // namespace fe
