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
// Two passes over 32-pixel blocks, all products on 16x16x32 bf16 MFMAs:
//   pass 1  (16 waves; wave w owns output rows 16w..16w+15 in every step)
//           decode z'[C x 32] = W z (A = the wave's W rows in registers,
//           B = the z block from LDS); residual, loss and sign; the signs of
//           each pixel are kept as two 16-bit masks per wave (2 bits per
//           value); dW [C x D] += s z^T and db += s 1 accumulated in
//           registers over the workgroup's blocks;
//   pass 2  (8 waves) dz [D x 32] = W^T s from the masks (A = W^T columns in
//           registers, B = the signs expanded into LDS).
// Splitting dz off keeps each pass's resident operands (W rows + dW
// accumulators, W^T columns) within the register file; the masks cost
// 2 bits per output value each way.
// Exactness: float32 operands are split into bf16 parts (x = hi + lo + ...);
// signs and ones are exact bf16.  The decode keeps the products of order
// <= 1 of two-part splits of W and z (about 16 significant bits per
// product); dz and dW multiply exact signs by two-part splits (the same); db
// sums exact integers.  Each workgroup of pass 1 writes its partial dW, db
// and loss; a third kernel adds them up in a fixed order.
#include "fe_common.h"

#include <atomic>
#include <type_traits>

#pragma clang fp contract(off)

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 256;              // decoder output channels
constexpr int kPB = 32;              // pixels per block
constexpr int kP1Threads = 512;      // pass 1: 8 waves of 32 output rows
constexpr int kDecThreads = 512;     // pass 2: 8 waves
constexpr int kMaxDevices = 64;

struct DecArgs {
  const float* feat;      // [D][P]
  const float* weight;    // [C][D]
  const float* bias;      // [C]
  const void* target;     // [C][P] float or bf16 bits
  float* decoded;         // [C][P] or null
  float* d_feat;          // [D][P] or null
  uint2* signs;           // [blocks][8][32]: per (block, 32-row group, pixel) nonzero and negative masks
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

// Bit b of a pixel's 32-bit sign masks for row group g stands for channel
// 32 g + sign_row(b): the order in which a 32x32 MFMA result holds the rows
// (lane half h, value v: row 8 (v / 4) + 4 h + v % 4), undone in pass 2 by
// reading W^T in that order.
__host__ __device__ constexpr int sign_row(int b) { return 8 * ((b & 15) >> 2) + 4 * (b >> 4) + (b & 3); }

// Pass 1: decode, residual, loss, signs, dW and db.
template <int KIN, typename TT>
__global__ __launch_bounds__(kP1Threads) void decoder_pass1_kernel(DecArgs a) {
  constexpr int KS = KIN / 16;        // k steps of the decode (32x32x16)
  constexpr int NBW = KIN / 32;       // 32-column blocks of dW
  constexpr int ZR = kPB + 8;         // padded rows of the channel-major z tile
  constexpr int ZT = KIN + 8;         // padded rows of the pixel-major z tile
  constexpr int SR = kPB + 8;
  constexpr int NQ = KIN * kPB / 4;   // 2x2 (channel, pixel) quads of a z block
  constexpr int ZQ = (NQ + kP1Threads - 1) / kP1Threads;
  static_assert(NQ % 64 == 0, "whole waves of quads");
  // with 128 input channels the low parts of W live in LDS, which leaves
  // registers for the next block's target values
  constexpr bool kLoLds = KIN > 64;
  constexpr int WL = kLoLds ? KIN + 8 : 8;
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  __shared__ __attribute__((aligned(16))) __bf16 s_zc[2][KIN][ZR];   // z[c][px], hi / lo
  __shared__ __attribute__((aligned(16))) __bf16 s_zt[2][kPB][ZT];   // z[px][c], hi / lo
  __shared__ __attribute__((aligned(16))) __bf16 s_sc[kC][SR];       // sign[c][px] (each wave its own rows)
  __shared__ __attribute__((aligned(16))) __bf16 s_wlo[kLoLds ? kC : 1][WL];  // low parts of W
  __shared__ float s_bias[kC];
  __shared__ float s_red[kP1Threads / 64];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int h = lane >> 5;            // 4-row half of each 8-row group of the result; k half of the operands
  const int px = lane & 31;
  const int64_t P = a.P;
  const uint32_t Pu = (uint32_t)P;
  const int64_t nblocks = (P + kPB - 1) / kPB;
  for (int c = threadIdx.x; c < kC; c += kP1Threads) s_bias[c] = a.bias[c];

  // W rows of this wave (decode A operand: row 32 wave + px, k = 16 ks + 8 h + j), hi / lo
  bf16x8 wa[KS][kLoLds ? 1 : 2];
  {
    const float* wr = a.weight + (int64_t)(32 * wave + px) * KIN + 8 * h;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float4 x0 = *reinterpret_cast<const float4*>(wr + 16 * ks);
      const float4 x1 = *reinterpret_cast<const float4*>(wr + 16 * ks + 4);
      const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      bf16x8 lo8;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 hi, lo;
        split2(xs[j], hi, lo);
        wa[ks][0][j] = hi;
        lo8[j] = lo;
      }
      if constexpr (kLoLds)
        *reinterpret_cast<bf16x8*>(&s_wlo[32 * wave + px][16 * ks + 8 * h]) = lo8;
      else
        wa[ks][kLoLds ? 0 : 1] = lo8;
    }
  }
  bf16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (__bf16)1.f;
  f32x16 dw[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) dw[nb] = f32x16{};
  f32x16 dbv = f32x16{};
  float loss = 0.f;

  // z quads of this thread, q = threadIdx.x + 512 i: channels 2 (q / 16) +
  // {0, 1}, pixels 2 (q % 16) + {0, 1} of the block.  Addresses: a
  // wave-uniform base (8 channel rows per wave and i) plus a 32-bit byte
  // offset (pixels < 2^24); quads exist for whole waves (NQ is a multiple of
  // 64).  Pixels past the last one read that pixel and are zeroed.
  const int zc0 = 2 * (threadIdx.x >> 4), zx = 2 * (threadIdx.x & 15);
  float zn[ZQ][4];
#pragma unroll
  for (int i = 0; i < ZQ; ++i) zn[i][0] = zn[i][1] = zn[i][2] = zn[i][3] = 0.f;
  auto load_z = [&](int64_t blk) {
    if (blk >= nblocks) return;
    const int64_t p0 = blk * kPB;
    const int last = (int)(P - 1 - p0 < kPB ? P - 1 - p0 : kPB - 1);
    const int x0 = zx < last ? zx : last, x1 = zx + 1 < last ? zx + 1 : last;
    const uint32_t r0 = (uint32_t)(zc0 - 8 * wave) * Pu * 4u, r1 = r0 + 4u * Pu;
    // raw values: the pixels past the last one are zeroed when staged, so
    // that nothing waits on these loads before then
#pragma unroll
    for (int i = 0; i < ZQ; ++i) {
      if (threadIdx.x + kP1Threads * i < NQ) {
        const char* base =
            reinterpret_cast<const char*>(a.feat + (int64_t)(8 * wave_u + 2 * (kP1Threads / 16) * i) * P + p0);
        zn[i][0] = *reinterpret_cast<const float*>(base + r0 + 4u * (uint32_t)x0);
        zn[i][1] = *reinterpret_cast<const float*>(base + r0 + 4u * (uint32_t)x1);
        zn[i][2] = *reinterpret_cast<const float*>(base + r1 + 4u * (uint32_t)x0);
        zn[i][3] = *reinterpret_cast<const float*>(base + r1 + 4u * (uint32_t)x1);
      }
    }
  };
  // target of this lane's 16 (row, pixel) entries, one block ahead: rows 32 wave + 8 (v / 4)
  // + 4 h + v % 4, pixel px; lanes past the last pixel read that pixel (and
  // contribute nothing)
  float tv[16];
  auto load_t = [&](int64_t blk) {
    const int64_t p0 = blk * kPB;
    const int x = p0 + px < P ? px : (int)(P - 1 - p0);
    const char* base =
        reinterpret_cast<const char*>(static_cast<const TT*>(a.target) + (int64_t)(32 * wave_u) * P + p0);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint32_t o = ((uint32_t)(8 * (v >> 2) + 4 * h + (v & 3)) * Pu + (uint32_t)x) * (uint32_t)sizeof(TT);
      if constexpr (std::is_same<TT, float>::value)
        tv[v] = *reinterpret_cast<const float*>(base + o);
      else
        tv[v] = __uint_as_float((uint32_t)*reinterpret_cast<const uint16_t*>(base + o) << 16);
    }
  };
  load_z(blockIdx.x);
  load_t(blockIdx.x);
  __syncthreads();   // s_bias, s_wlo
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t p0 = blk * kPB;
    // z block to LDS in both layouts, hi / lo parts; the next block's loads go out
#pragma unroll
    for (int i = 0; i < ZQ; ++i) {
      if (threadIdx.x + kP1Threads * i < NQ) {
        const int c = zc0 + 2 * (kP1Threads / 16) * i;
        __bf16 hi[4], lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool in = p0 + zx + (e & 1) < P;
          split2(in ? zn[i][e] : 0.f, hi[e], lo[e]);
        }
        *reinterpret_cast<bf16x2*>(&s_zc[0][c][zx]) = bf16x2{hi[0], hi[1]};
        *reinterpret_cast<bf16x2*>(&s_zc[0][c + 1][zx]) = bf16x2{hi[2], hi[3]};
        *reinterpret_cast<bf16x2*>(&s_zc[1][c][zx]) = bf16x2{lo[0], lo[1]};
        *reinterpret_cast<bf16x2*>(&s_zc[1][c + 1][zx]) = bf16x2{lo[2], lo[3]};
        *reinterpret_cast<bf16x2*>(&s_zt[0][zx][c]) = bf16x2{hi[0], hi[2]};
        *reinterpret_cast<bf16x2*>(&s_zt[0][zx + 1][c]) = bf16x2{hi[1], hi[3]};
        *reinterpret_cast<bf16x2*>(&s_zt[1][zx][c]) = bf16x2{lo[0], lo[2]};
        *reinterpret_cast<bf16x2*>(&s_zt[1][zx + 1][c]) = bf16x2{lo[1], lo[3]};
      }
    }
    load_z(blk + gridDim.x);
    __syncthreads();
    // decode: rows 32 wave.. x the block's 32 pixels
    f32x16 acc = f32x16{};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kc = 16 * ks + 8 * h;
      const bf16x8 zh = *reinterpret_cast<const bf16x8*>(&s_zt[0][px][kc]);
      const bf16x8 zl = *reinterpret_cast<const bf16x8*>(&s_zt[1][px][kc]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ks][0], zh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ks][0], zl, acc, 0, 0, 0);
      bf16x8 wl;
      if constexpr (kLoLds)
        wl = *reinterpret_cast<const bf16x8*>(&s_wlo[32 * wave + px][kc]);
      else
        wl = wa[ks][kLoLds ? 0 : 1];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wl, zh, acc, 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // residual, loss and sign of each (row, pixel); bit v of nzb / ngb: the
    // sign of (row of v, this pixel) is nonzero / negative
    const bool inside = p0 + px < P;
    uint32_t nzb = 0u, ngb = 0u;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 32 * wave + 8 * (v >> 2) + 4 * h + (v & 3);
      acc[v] += s_bias[c];
      const float r = inside ? acc[v] - tv[v] : 0.f;
      loss += fabsf(r);
      const bool nz = r != 0.f, ng = r < 0.f;
      nzb |= (uint32_t)nz << v;
      ngb |= (uint32_t)ng << v;
      s_sc[c][px] = (__bf16)(nz ? (ng ? -1.f : 1.f) : 0.f);
    }
    if (a.decoded && inside) {
      float* dr = a.decoded + (int64_t)(32 * wave_u) * P + p0;
#pragma unroll
      for (int v = 0; v < 16; ++v) dr[(uint32_t)(8 * (v >> 2) + 4 * h + (v & 3)) * Pu + (uint32_t)px] = acc[v];
    }
    if (blk + gridDim.x < nblocks) load_t(blk + gridDim.x);
    // the pixel's 32-row masks: bits 0..15 from this lane, 16..31 from lane + 32
    const uint32_t onz = (uint32_t)__shfl_xor((int)nzb, 32, 64), ong = (uint32_t)__shfl_xor((int)ngb, 32, 64);
    if (h == 0) a.signs[(blk * 8 + wave) * kPB + px] = make_uint2(nzb | (onz << 16), ngb | (ong << 16));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW += s z^T and db += s 1 over the block's pixels (rows of this wave)
#pragma unroll
    for (int ks = 0; ks < kPB / 16; ++ks) {
      const int kp = 16 * ks + 8 * h;
      const bf16x8 sa = *reinterpret_cast<const bf16x8*>(&s_sc[32 * wave + px][kp]);
      dbv = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa, ones, dbv, 0, 0, 0);
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        const bf16x8 zh = *reinterpret_cast<const bf16x8*>(&s_zc[0][32 * nb + px][kp]);
        const bf16x8 zl = *reinterpret_cast<const bf16x8*>(&s_zc[1][32 * nb + px][kp]);
        dw[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa, zh, dw[nb], 0, 0, 0);
        dw[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(sa, zl, dw[nb], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
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
      const int c = 32 * wave + 8 * (v >> 2) + 4 * h + (v & 3);
      out[(int64_t)c * KIN + 32 * nb + px] = dw[nb][v] * a.inv_p;
    }
  if (px == 0) {
#pragma unroll
    for (int v = 0; v < 16; ++v) out[kC * KIN + 32 * wave + 8 * (v >> 2) + 4 * h + (v & 3)] = dbv[v] * a.inv_p;
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
  if (lane == 0) s_red[wave] = loss;
  __syncthreads();
  if (threadIdx.x == 0) {
    float l = 0.f;
    for (int w = 0; w < kP1Threads / 64; ++w) l += s_red[w];
    out[kC * KIN + kC] = l * a.inv_p;
  }
}

// Pass 2: dz = W^T s / P from the sign masks (16x16x32; a unit is 16 input
// channels x 16 pixels, and wave w keeps the W^T columns of its units).
// Thread t < 256 expands the masks of (row group t / 32, pixel t % 32) into
// bf16 signs in LDS through a 256-entry table (4 nonzero bits + 4 negative
// bits -> four bf16 values).
template <int KIN>
__global__ __launch_bounds__(kDecThreads) void decoder_pass2_kernel(DecArgs a) {
  constexpr int MB = KIN / 16;
  constexpr int NU = 2 * MB;
  constexpr int UPW = NU > 8 ? NU / 8 : 1;
  constexpr int ST = kC + 8;
  __shared__ __attribute__((aligned(16))) __bf16 s_st[kPB][ST];      // sign[px][position]
  __shared__ uint2 s_lut[256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t P = a.P;
  const int64_t nblocks = (P + kPB - 1) / kPB;
  const int u0 = wave % NU;
  const bool has_dz = wave < NU;
  const int mblk = u0 % MB;   // the units of a wave share one row block
  if (threadIdx.x < 256) {
    uint32_t w[2] = {0u, 0u};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t nz = (threadIdx.x >> j) & 1u, ng = (threadIdx.x >> (4 + j)) & 1u;
      const uint32_t bits = nz ? (ng ? 0xBF80u : 0x3F80u) : 0u;
      w[j >> 1] |= bits << (16 * (j & 1));
    }
    s_lut[threadIdx.x] = make_uint2(w[0], w[1]);
  }
  // W^T columns: k position 8 (lane / 16) + j of step ks is channel
  // 32 ks + sign_row(8 (lane / 16) + j)
  bf16x8 wt[kC / 32][2];
  {
    const int ic = 16 * mblk + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < kC / 32; ++ks)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 hi = (__bf16)0.f, lo = (__bf16)0.f;
        if (has_dz) split2(a.weight[(int64_t)(32 * ks + sign_row(8 * (lane >> 4) + j)) * KIN + ic], hi, lo);
        wt[ks][0][j] = hi;
        wt[ks][1][j] = lo;
      }
  }
  const int ex_px = threadIdx.x & 31, ex_g = (threadIdx.x >> 5) & 7;
  const bool expands = threadIdx.x < kC;
  uint2 mk_n = make_uint2(0u, 0u);
  auto load_masks = [&](int64_t blk) {
    if (expands && blk < nblocks) mk_n = a.signs[(blk * 8 + ex_g) * kPB + ex_px];
  };
  load_masks(blockIdx.x);
  __syncthreads();   // s_lut
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t p0 = blk * kPB;
    if (expands) {
      const uint2 m = mk_n;
      uint2 e[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) e[q] = s_lut[((m.x >> (4 * q)) & 15u) | (((m.y >> (4 * q)) & 15u) << 4)];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4*>(&s_st[ex_px][32 * ex_g + 8 * q]) =
            make_uint4(e[2 * q].x, e[2 * q].y, e[2 * q + 1].x, e[2 * q + 1].y);
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

// Sum of the workgroups' partials.  Workgroup b adds up outputs 64 b..64 b+63:
// wave w takes the groups g = w (mod 4), four running sums per lane, and the
// four waves' sums meet in LDS.
__global__ __launch_bounds__(256) void decoder_reduce_kernel(const float* partial, int groups, int n, float* d_weight,
                                                             float* d_bias, float* loss, int nw) {
  __shared__ float s_part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (i < n) {
    int g = wave;
    for (; g + 12 < groups; g += 16) {
      s0 += partial[(int64_t)g * n + i];
      s1 += partial[(int64_t)(g + 4) * n + i];
      s2 += partial[(int64_t)(g + 8) * n + i];
      s3 += partial[(int64_t)(g + 12) * n + i];
    }
    for (; g < groups; g += 4) s0 += partial[(int64_t)g * n + i];
  }
  s_part[wave][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (wave == 0 && i < n) {
    const float s = (s_part[0][lane] + s_part[1][lane]) + (s_part[2][lane] + s_part[3][lane]);
    if (i < nw)
      d_weight[i] = s;
    else if (i < n - 1)
      d_bias[i - nw] = s;
    else
      loss[0] = s;
  }
}

// Resident workgroups of a kernel on the whole device (cached per device).
template <typename K>
static int device_slots(K kernel, int threads, std::atomic<int>* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int per_cu = 0, cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
  v = per_cu * cus;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

template <int KIN, typename TT>
static int decoder_grid() {
  static std::atomic<int> cache[kMaxDevices];
  return device_slots(decoder_pass1_kernel<KIN, TT>, kP1Threads, cache);
}

template <int KIN>
static int decoder_grid2() {
  static std::atomic<int> cache[kMaxDevices];
  return device_slots(decoder_pass2_kernel<KIN>, kDecThreads, cache);
}

template <int KIN, typename TT>
static hipError_t launch_kin(const DecArgs& a0, int grid, float* d_weight, float* d_bias, float* loss,
                             hipStream_t s) {
  DecArgs a = a0;
  hipLaunchKernelGGL((decoder_pass1_kernel<KIN, TT>), dim3(grid), dim3(kP1Threads), 0, s, a);
  if (a.d_feat) {
    const int64_t blocks = (a.P + kPB - 1) / kPB;
    int64_t g2 = decoder_grid2<KIN>();
    if (g2 < 1) return hipErrorInvalidValue;
    if (g2 > blocks) g2 = blocks;
    hipLaunchKernelGGL((decoder_pass2_kernel<KIN>), dim3((unsigned)g2), dim3(kDecThreads), 0, s, a);
  }
  const int n = kC * KIN + kC + 1;
  hipLaunchKernelGGL(decoder_reduce_kernel, dim3((n + 63) / 64), dim3(256), 0, s, a.partial, grid, n, d_weight,
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

size_t decoder_sign_bytes(int64_t pixels) {
  return (size_t)8 * kPB * (size_t)((pixels + kPB - 1) / kPB) * sizeof(uint2);
}

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
