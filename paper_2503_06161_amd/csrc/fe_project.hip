// Per-Gaussian projection, forward and backward, for gfx950.
//
// Forward (one thread per Gaussian, float64 geometry): camera-space centre,
// Sigma = R S S^T R^T from the normalised quaternion (eq. 2), the affine
// approximation J of the perspective map and Sigma' = J W Sigma W^T J^T
// (eq. 9) plus the dilation, the conic Sigma'^-1, the pixel position, the
// 3-sigma pixel box and its tile rectangle, and the view-dependent colour from
// real SH coefficients (Sec. 3.1).  The record is rounded to float32 once.
//
// Every expression that decides a sort key or a box (tz, u, v, Sigma'_xx,
// Sigma'_yy, the box bounds) is evaluated as separate IEEE float64 operations
// in a fixed order with contraction disabled, so the keys are reproducible
// bit for bit by any implementation that evaluates the same expressions.
//
// Backward (one thread per Gaussian, float32): chain rule from the
// screen-space gradients (u, v, conic, opacity, colour) through the conic
// inverse, eq. (9), eq. (2), the quaternion normalisation and the SH basis.
// The skip/stop decisions and the sort order are piecewise constant; the
// colour clamp at 0 and a clamped Jacobian coordinate pass zero.
#include "fe_common.h"

#include <type_traits>

#pragma clang fp contract(off)

namespace fe {
namespace {

// Real SH basis, orthonormal, no Condon-Shortley phase; each constant is
// the closed form K_l^m (times sqrt(2) for m != 0) written out.
constexpr double kC0 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
constexpr double kC1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
constexpr double kC2a = 1.0925484305920792;   // sqrt(15 / pi) / 2
constexpr double kC2b = 0.31539156525252005;  // sqrt(5 / pi) / 4
constexpr double kC2c = 0.5462742152960396;   // sqrt(15 / pi) / 4
constexpr double kC3e = 0.5900435899266435;   // sqrt(35 / (2 pi)) / 4
constexpr double kC3f = 2.890611442640554;    // sqrt(105 / pi) / 2
constexpr double kC3g = 0.4570457994644658;   // sqrt(21 / (2 pi)) / 4
constexpr double kC3h = 0.3731763325901154;   // sqrt(7 / pi) / 4
constexpr double kC3i = 1.445305721320277;    // sqrt(105 / pi) / 4

template <int L, typename T>
__device__ __forceinline__ void sh_basis(T x, T y, T z, T* Y) {
  Y[0] = T(kC0);
  if constexpr (L >= 1) {
    Y[1] = T(kC1) * y;
    Y[2] = T(kC1) * z;
    Y[3] = T(kC1) * x;
  }
  if constexpr (L >= 2) {
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = T(kC2a) * (x * y);
    Y[5] = T(kC2a) * (y * z);
    Y[6] = T(kC2b) * (T(3.0) * zz - T(1.0));
    Y[7] = T(kC2a) * (x * z);
    Y[8] = T(kC2c) * (xx - yy);
    if constexpr (L >= 3) {
      Y[9] = T(kC3e) * y * (T(3.0) * xx - yy);
      Y[10] = T(kC3f) * x * y * z;
      Y[11] = T(kC3g) * y * (T(5.0) * zz - T(1.0));
      Y[12] = T(kC3h) * z * (T(5.0) * zz - T(3.0));
      Y[13] = T(kC3g) * x * (T(5.0) * zz - T(1.0));
      Y[14] = T(kC3i) * z * (xx - yy);
      Y[15] = T(kC3e) * x * (xx - T(3.0) * yy);
    }
  }
}

// Gradient of sum_k c_k Y_k with respect to the direction components,
// accumulated into (gx, gy, gz).
template <int L, typename T>
__device__ __forceinline__ void sh_basis_grad(T x, T y, T z, const T* c, T& gx, T& gy, T& gz) {
  gx = T(0.0);
  gy = T(0.0);
  gz = T(0.0);
  if constexpr (L >= 1) {
    gy += T(kC1) * c[1];
    gz += T(kC1) * c[2];
    gx += T(kC1) * c[3];
  }
  if constexpr (L >= 2) {
    gx += T(kC2a) * y * c[4];
    gy += T(kC2a) * x * c[4];
    gy += T(kC2a) * z * c[5];
    gz += T(kC2a) * y * c[5];
    gz += T(6.0) * T(kC2b) * z * c[6];
    gx += T(kC2a) * z * c[7];
    gz += T(kC2a) * x * c[7];
    gx += T(2.0) * T(kC2c) * x * c[8];
    gy -= T(2.0) * T(kC2c) * y * c[8];
    if constexpr (L >= 3) {
      const T xx = x * x, yy = y * y, zz = z * z;
      gx += T(6.0) * T(kC3e) * x * y * c[9];
      gy += T(kC3e) * (T(3.0) * xx - T(3.0) * yy) * c[9];
      gx += T(kC3f) * y * z * c[10];
      gy += T(kC3f) * x * z * c[10];
      gz += T(kC3f) * x * y * c[10];
      gy += T(kC3g) * (T(5.0) * zz - T(1.0)) * c[11];
      gz += T(10.0) * T(kC3g) * y * z * c[11];
      gz += T(kC3h) * (T(15.0) * zz - T(3.0)) * c[12];
      gx += T(kC3g) * (T(5.0) * zz - T(1.0)) * c[13];
      gz += T(10.0) * T(kC3g) * x * z * c[13];
      gx += T(2.0) * T(kC3i) * x * z * c[14];
      gy -= T(2.0) * T(kC3i) * y * z * c[14];
      gz += T(kC3i) * (xx - yy) * c[14];
      gx += T(kC3e) * (T(3.0) * xx - T(3.0) * yy) * c[15];
      gy -= T(6.0) * T(kC3e) * x * y * c[15];
    }
  }
}

// One Gaussian's SH row [(L+1)^2][3] as floats.  Degree 3 rows (96 B in
// bf16, 192 B in float32) are read with 16-byte loads; smaller rows are not
// 16-byte aligned in general and are read element by element.
template <int L, typename ShT>
__device__ __forceinline__ void load_sh_row(const void* sh, int64_t i, float* out) {
  constexpr int K3 = 3 * (L + 1) * (L + 1);
  if constexpr (L == 3 && std::is_same<ShT, uint16_t>::value) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(sh) + i * K3);
#pragma unroll
    for (int v = 0; v < K3 / 8; ++v) {
      const uint4 q = p[v];
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        out[8 * v + 2 * h] = __uint_as_float(w[h] << 16);
        out[8 * v + 2 * h + 1] = __uint_as_float(w[h] & 0xFFFF0000u);
      }
    }
  } else if constexpr (L == 3) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(sh) + i * K3);
#pragma unroll
    for (int v = 0; v < K3 / 4; ++v) {
      const float4 q = p[v];
      out[4 * v] = q.x;
      out[4 * v + 1] = q.y;
      out[4 * v + 2] = q.z;
      out[4 * v + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < K3; ++k) out[k] = load_as_float<ShT>(sh, i * K3 + k);
  }
}

struct ProjArgs {
  CamConst cc;
  int64_t n;
  int32_t tile_w, tile_h, tiles_x;
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const void* sh;
  StateView v;
};

// Geometry shared by the forward (float64: it decides keys and boxes) and the
// backward (float32: gradients only), in the same expressions.
template <typename T>
struct GeoT {
  T tx, ty, tz;
  T qw, qx, qy, qz, qn;   // normalised quaternion and the input norm
  T R[9];
  T s[3];
  T Sig[6];               // xx xy xz yy yz zz
  T xr, yr;
  bool clampx, clampy;
  T j00, j02, j11, j12;
  T Tm[6];                // 2x3 row-major
  T a, b, c;              // Sigma' (dilated)
  T det;
  T u, v;
};

template <typename T>
__device__ __forceinline__ void geometry(const CamConst& cc, const float* mp, const float* sp,
                                         const float* qp, GeoT<T>& G) {
  const T x = mp[0], y = mp[1], z = mp[2];
  G.tx = ((T(cc.R[0]) * x + T(cc.R[1]) * y) + T(cc.R[2]) * z) + T(cc.t[0]);
  G.ty = ((T(cc.R[3]) * x + T(cc.R[4]) * y) + T(cc.R[5]) * z) + T(cc.t[1]);
  G.tz = ((T(cc.R[6]) * x + T(cc.R[7]) * y) + T(cc.R[8]) * z) + T(cc.t[2]);
  const T w0 = qp[0], x0 = qp[1], y0 = qp[2], z0 = qp[3];
  G.qn = sqrt(((w0 * w0 + x0 * x0) + y0 * y0) + z0 * z0);
  const T w = w0 / G.qn, qx = x0 / G.qn, qy = y0 / G.qn, qz = z0 / G.qn;
  G.qw = w; G.qx = qx; G.qy = qy; G.qz = qz;
  T* R = G.R;
  R[0] = T(1.0) - T(2.0) * (qy * qy + qz * qz);
  R[1] = T(2.0) * (qx * qy - w * qz);
  R[2] = T(2.0) * (qx * qz + w * qy);
  R[3] = T(2.0) * (qx * qy + w * qz);
  R[4] = T(1.0) - T(2.0) * (qx * qx + qz * qz);
  R[5] = T(2.0) * (qy * qz - w * qx);
  R[6] = T(2.0) * (qx * qz - w * qy);
  R[7] = T(2.0) * (qy * qz + w * qx);
  R[8] = T(1.0) - T(2.0) * (qx * qx + qy * qy);
  G.s[0] = sp[0]; G.s[1] = sp[1]; G.s[2] = sp[2];
  T M[9];
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) M[a * 3 + k] = R[a * 3 + k] * G.s[k];
  auto sig = [&](int a, int b) {
    return (M[a * 3 + 0] * M[b * 3 + 0] + M[a * 3 + 1] * M[b * 3 + 1]) + M[a * 3 + 2] * M[b * 3 + 2];
  };
  G.Sig[0] = sig(0, 0); G.Sig[1] = sig(0, 1); G.Sig[2] = sig(0, 2);
  G.Sig[3] = sig(1, 1); G.Sig[4] = sig(1, 2); G.Sig[5] = sig(2, 2);
  G.xr = G.tx / G.tz;
  G.yr = G.ty / G.tz;
  T xc = G.xr, yc = G.yr;
  G.clampx = false;
  G.clampy = false;
  if (T(cc.limx) > T(0.0)) {
    G.clampx = (G.xr < -T(cc.limx)) || (G.xr > T(cc.limx));
    G.clampy = (G.yr < -T(cc.limy)) || (G.yr > T(cc.limy));
    xc = fmin(fmax(G.xr, -T(cc.limx)), T(cc.limx));
    yc = fmin(fmax(G.yr, -T(cc.limy)), T(cc.limy));
  }
  G.j00 = T(cc.fx) / G.tz;
  G.j02 = (-T(cc.fx) * xc) / G.tz;
  G.j11 = T(cc.fy) / G.tz;
  G.j12 = (-T(cc.fy) * yc) / G.tz;
  for (int k = 0; k < 3; ++k) {
    G.Tm[k] = G.j00 * T(cc.R[0 * 3 + k]) + G.j02 * T(cc.R[2 * 3 + k]);
    G.Tm[3 + k] = G.j11 * T(cc.R[1 * 3 + k]) + G.j12 * T(cc.R[2 * 3 + k]);
  }
  const T S[9] = {G.Sig[0], G.Sig[1], G.Sig[2], G.Sig[1], G.Sig[3], G.Sig[4],
                       G.Sig[2], G.Sig[4], G.Sig[5]};
  T U[6];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b)
      U[a * 3 + b] = (G.Tm[a * 3 + 0] * S[0 * 3 + b] + G.Tm[a * 3 + 1] * S[1 * 3 + b]) +
                     G.Tm[a * 3 + 2] * S[2 * 3 + b];
  auto c2 = [&](int a, int b) {
    return (U[a * 3 + 0] * G.Tm[b * 3 + 0] + U[a * 3 + 1] * G.Tm[b * 3 + 1]) + U[a * 3 + 2] * G.Tm[b * 3 + 2];
  };
  G.a = c2(0, 0) + T(cc.dilation);
  G.b = c2(0, 1);
  G.c = c2(1, 1) + T(cc.dilation);
  G.det = G.a * G.c - G.b * G.b;
  G.u = T(cc.fx) * G.xr + T(cc.cx);
  G.v = T(cc.fy) * G.yr + T(cc.cy);
}

using Geo = GeoT<double>;

__device__ __forceinline__ bool all_finite(const float* p, int k) {
  bool ok = true;
  for (int i = 0; i < k; ++i) ok = ok && isfinite(p[i]);
  return ok;
}

template <int L, typename ShT>
__global__ __launch_bounds__(256) void project_fwd_kernel(ProjArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = i < a.n;
  bool nonfinite = false;
  if (in) {
    const CamConst& cc = a.cc;
    const float* mp = a.means + 3 * i;
    const float* sp = a.scales + 3 * i;
    const float* qp = a.quats + 4 * i;
    const float op = a.opacity[i];
    const bool fin = all_finite(mp, 3) && all_finite(sp, 3) && all_finite(qp, 4) && isfinite(op);
    const double q2 = (((double)qp[0] * qp[0] + (double)qp[1] * qp[1]) + (double)qp[2] * qp[2]) +
                      (double)qp[3] * qp[3];
    nonfinite = !(fin && q2 > 0.0);
    uint32_t count = 0;
    uint32_t dkey = 0xFFFFFFFFu;
    float2 xy = make_float2(0.f, 0.f);
    float4 co = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 rgb = make_float4(0.f, 0.f, 0.f, 0.f);
    short4 box = make_short4(1, 1, 0, 0);
    if (!nonfinite) {
      const double tz = ((cc.R[6] * (double)mp[0] + cc.R[7] * (double)mp[1]) + cc.R[8] * (double)mp[2]) + cc.t[2];
      if (tz > cc.near_plane) {
        Geo G;
        geometry(cc, mp, sp, qp, G);
        if (G.det > 0.0 && isfinite(G.det)) {
          const double rx = 3.0 * sqrt(G.a);
          const double ry = 3.0 * sqrt(G.c);
          double i0 = ceil((G.u - rx) - 0.5);
          double i1 = floor((G.u + rx) - 0.5);
          double j0 = ceil((G.v - ry) - 0.5);
          double j1 = floor((G.v + ry) - 0.5);
          i0 = fmax(i0, 0.0);
          j0 = fmax(j0, 0.0);
          i1 = fmin(i1, (double)(cc.width - 1));
          j1 = fmin(j1, (double)(cc.height - 1));
          // conic and the float32 record
          const double A = G.c / G.det, B = -G.b / G.det, C = G.a / G.det;
          xy = make_float2((float)G.u, (float)G.v);
          co = make_float4((float)A, (float)B, (float)C, op);
          // colour from SH along normalise(mu - campos)
          const double dx = (double)mp[0] - cc.campos[0];
          const double dy = (double)mp[1] - cc.campos[1];
          const double dz = (double)mp[2] - cc.campos[2];
          const double dn = sqrt(((dx * dx + dy * dy) + dz * dz));
          double Y[16];
          sh_basis<L>(dx / dn, dy / dn, dz / dn, Y);
          constexpr int K = (L + 1) * (L + 1);
          float shr[3 * K];
          load_sh_row<L, ShT>(a.sh, i, shr);
          double col[3] = {0.5, 0.5, 0.5};
          double acc[3] = {0.0, 0.0, 0.0};
          for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) acc[ch] += (double)shr[k * 3 + ch] * Y[k];
          for (int ch = 0; ch < 3; ++ch) col[ch] = fmax(acc[ch] + 0.5, 0.0);
          // colour and the view-space depth (the depth image's value)
          rgb = make_float4((float)col[0], (float)col[1], (float)col[2], (float)G.tz);
          if (i0 <= i1 && j0 <= j1 && isfinite(G.u) && isfinite(G.v)) {
            const int ii0 = (int)i0, ii1 = (int)i1, jj0 = (int)j0, jj1 = (int)j1;
            box = make_short4((short)ii0, (short)jj0, (short)ii1, (short)jj1);
            const int tx0 = ii0 / a.tile_w, tx1 = ii1 / a.tile_w;
            const int ty0 = jj0 / a.tile_h, ty1 = jj1 / a.tile_h;
            count = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
            dkey = __float_as_uint((float)G.tz);
          }
        }
      }
    }
    a.v.xy[i] = xy;
    a.v.conic_o[i] = co;
    a.v.rgb[i] = rgb;
    a.v.box[i] = box;
    a.v.dkey[i] = dkey;
    a.v.count[i] = count;
  }
  // wave-aggregated count of culled non-finite Gaussians (an atomic only
  // where there are any); the visible count comes from the binning
  const unsigned long long mn = __ballot(nonfinite);
  if (__lane_id() == 0 && mn) atomicAdd(&a.v.report[kRepNonFinite], (unsigned long long)__popcll(mn));
}

struct ProjBwdArgs {
  CamConst cc;
  int64_t n;
  const float* means;
  const float* scales;
  const float* quats;
  const void* sh;
  const float* grad2d;    // [n][12]: u v A B C o r g b depth - -
  const uint32_t* count;
  float* g_means;
  float* g_scales;
  float* g_quats;
  float* g_opacity;
  float* g_sh;
  float* g_means2d;
  int accumulate;
};

template <int L, typename ShT>
__global__ __launch_bounds__(256) void project_bwd_kernel(ProjBwdArgs a) {
  // the chain rule in float32: the gradients need no float64 (the decisions
  // that must match the forward exactly were taken there)
  typedef float T;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = i < a.n;   // every lane stays to the wave's SH-gradient stores
  constexpr int K = (L + 1) * (L + 1);
  T gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = T(0.0);
  // dL/dsh[k][ch] = Y_k * gact[ch] (zero for a culled Gaussian), formed at the store
  T Y[16], gact[3] = {T(0.0), T(0.0), T(0.0)};
  for (int k = 0; k < 16; ++k) Y[k] = T(0.0);
  T gu = T(0.0), gv = T(0.0);
  auto put = [&](float* p, T val) {
    if (a.accumulate) *p += (float)val; else *p = (float)val;
  };
  const bool active = valid && a.count[i] > 0;
  if (active) {
    const CamConst& cc = a.cc;
    const float* mp = a.means + 3 * i;
    const float* g2 = a.grad2d + 12 * i;
    const T gcol[3] = {g2[6], g2[7], g2[8]};
    // colour first (the view direction does not need the geometry), so
    // that its registers are free before the geometry's
    const T dx = (T)mp[0] - T(cc.campos[0]);
    const T dy = (T)mp[1] - T(cc.campos[1]);
    const T dz = (T)mp[2] - T(cc.campos[2]);
    const T dn = sqrt(((dx * dx + dy * dy) + dz * dz));
    const T ux = dx / dn, uy = dy / dn, uz = dz / dn;
    sh_basis<L>(ux, uy, uz, Y);
    float shr[3 * K];
    load_sh_row<L, ShT>(a.sh, i, shr);
    // the clamp at 0 passes the gradient of a channel whose raw value is >= 0
    for (int ch = 0; ch < 3; ++ch) {
      T raw = T(0.0);
      for (int k = 0; k < K; ++k) raw += (T)shr[k * 3 + ch] * Y[k];
      raw += T(0.5);
      gact[ch] = raw >= T(0.0) ? gcol[ch] : T(0.0);
    }
    // direction gradient of sum_ch gact_ch raw_ch: one basis derivative of
    // the channel-combined coefficients
    T cf[16];
    for (int k = 0; k < 16; ++k) cf[k] = T(0.0);
    for (int k = 0; k < K; ++k)
      cf[k] = (gact[0] * (T)shr[k * 3] + gact[1] * (T)shr[k * 3 + 1]) + gact[2] * (T)shr[k * 3 + 2];
    T gdx, gdy, gdz;
    sh_basis_grad<L>(ux, uy, uz, cf, gdx, gdy, gdz);
    const T dd = ux * gdx + uy * gdy + uz * gdz;
    const T idn = T(1.0) / dn;
    gm[0] += (gdx - ux * dd) * idn;
    gm[1] += (gdy - uy * dd) * idn;
    gm[2] += (gdz - uz * dd) * idn;
  }
  if constexpr (L == 3) {
    // The wave's 48-float rows leave through LDS as contiguous float4 stores,
    // half of the wave's Gaussians at a time (one row per lane would make
    // every store instruction touch 64 separate 16-byte pieces)
    static_assert(K * 3 == 48, "degree-3 rows");
    __shared__ float4 s_gsh[4][32 * 13];                 // rows padded to 13 float4
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int64_t w0 = i - lane;                         // the wave's first Gaussian
    const int64_t nv = a.n - w0 < 64 ? a.n - w0 : 64;    // its Gaussians
    auto gsh = [&](int e) { return (float)(Y[e / 3] * gact[e % 3]); };
    float4* base = reinterpret_cast<float4*>(a.g_sh) + w0 * 12;
#pragma unroll
    for (int hg = 0; hg < 2; ++hg) {
      if ((lane >> 5) == hg) {
#pragma unroll
        for (int v = 0; v < 12; ++v)
          s_gsh[wv][(lane & 31) * 13 + v] = make_float4(gsh(4 * v), gsh(4 * v + 1), gsh(4 * v + 2), gsh(4 * v + 3));
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const int e = c * 64 + lane, r = e / 12;
        if (32 * hg + r < nv) {
          float4 o = s_gsh[wv][r * 13 + e % 12];
          float4* q = base + 32 * hg * 12 + e;
          if (a.accumulate) {
            const float4 p = *q;
            o.x += p.x; o.y += p.y; o.z += p.z; o.w += p.w;
          }
          *q = o;
        }
      }
      // the next half rewrites the rows only after every lane has read them
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  } else {
    if (valid)
      for (int k = 0; k < K * 3; ++k) put(a.g_sh + i * K * 3 + k, Y[k / 3] * gact[k % 3]);
  }
  if (!valid) return;
  if (active) {
    const CamConst& cc = a.cc;
    const float* mp = a.means + 3 * i;
    const float* sp = a.scales + 3 * i;
    const float* qp = a.quats + 4 * i;
    const float* g2 = a.grad2d + 12 * i;
    gu = g2[0];
    gv = g2[1];
    const T gA = g2[2], gB = g2[3], gC = g2[4];
    gop = g2[5];
    GeoT<T> G;
    geometry<T>(cc, mp, sp, qp, G);
    // conic -> Sigma':  dL/dSigma' = -M GM M  with M the conic matrix and
    // GM the symmetric gradient (off-diagonal gB / 2)
    const T idet = T(1.0) / G.det;
    const T A = G.c * idet, B = -G.b * idet, C = G.a * idet;
    const T hB = T(0.5) * gB;
    const T P00 = gA * A + hB * B, P01 = gA * B + hB * C;
    const T P10 = hB * A + gC * B, P11 = hB * B + gC * C;
    const T S00 = -(A * P00 + B * P10);
    const T S01 = -(A * P01 + B * P11);
    const T S11 = -(B * P01 + C * P11);
    const T GS[4] = {S00, S01, S01, S11};
    // Sigma' = Tm Sigma Tm^T:  dSigma = Tm^T GS Tm,  dTm = 2 GS Tm Sigma
    const T* Tg = G.Tm;
    const T Sg[9] = {G.Sig[0], G.Sig[1], G.Sig[2], G.Sig[1], G.Sig[3], G.Sig[4],
                          G.Sig[2], G.Sig[4], G.Sig[5]};
    T GT[6];   // GS Tm  (2x3)
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) GT[r * 3 + k] = GS[r * 2 + 0] * Tg[0 * 3 + k] + GS[r * 2 + 1] * Tg[1 * 3 + k];
    T dSig[9];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) dSig[p * 3 + q] = Tg[0 * 3 + p] * GT[0 * 3 + q] + Tg[1 * 3 + p] * GT[1 * 3 + q];
    T dT[6];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k)
        dT[r * 3 + k] = T(2.0) * (GT[r * 3 + 0] * Sg[0 * 3 + k] + GT[r * 3 + 1] * Sg[1 * 3 + k] +
                               GT[r * 3 + 2] * Sg[2 * 3 + k]);
    // Tm = J W:  dJ = dT W^T
    auto dJ = [&](int r, int b) {
      return dT[r * 3 + 0] * T(cc.R[b * 3 + 0]) + dT[r * 3 + 1] * T(cc.R[b * 3 + 1]) + dT[r * 3 + 2] * T(cc.R[b * 3 + 2]);
    };
    const T dj00 = dJ(0, 0), dj02 = dJ(0, 2), dj11 = dJ(1, 1), dj12 = dJ(1, 2);
    const T itz = T(1.0) / G.tz, itz2 = itz * itz, itz3 = itz2 * itz;
    T gtx = T(0.0), gty = T(0.0), gtz = T(0.0);
    gtz += -T(cc.fx) * itz2 * dj00 - T(cc.fy) * itz2 * dj11;
    if (!G.clampx) {
      gtx += -T(cc.fx) * itz2 * dj02;
      gtz += T(2.0) * T(cc.fx) * G.tx * itz3 * dj02;
    } else {
      const T xc = fmin(fmax(G.xr, -T(cc.limx)), T(cc.limx));
      gtz += T(cc.fx) * xc * itz2 * dj02;
    }
    if (!G.clampy) {
      gty += -T(cc.fy) * itz2 * dj12;
      gtz += T(2.0) * T(cc.fy) * G.ty * itz3 * dj12;
    } else {
      const T yc = fmin(fmax(G.yr, -T(cc.limy)), T(cc.limy));
      gtz += T(cc.fy) * yc * itz2 * dj12;
    }
    // pixel position
    gtx += T(cc.fx) * itz * gu;
    gtz += -T(cc.fx) * G.tx * itz2 * gu;
    gty += T(cc.fy) * itz * gv;
    gtz += -T(cc.fy) * G.ty * itz2 * gv;
    // depth image: d(depth)/d(tz) = 1
    gtz += (T)g2[9];
    // t = W mu + t_c
    for (int k = 0; k < 3; ++k) gm[k] += T(cc.R[0 * 3 + k]) * gtx + T(cc.R[1 * 3 + k]) * gty + T(cc.R[2 * 3 + k]) * gtz;
    // Sigma = M M^T, M = R diag(s):  dM = 2 dSigma M
    const T* R = G.R;
    T M[9];
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k) M[p * 3 + k] = R[p * 3 + k] * G.s[k];
    T dR[9];
    for (int p = 0; p < 3; ++p)
      for (int k = 0; k < 3; ++k) {
        const T dM = T(2.0) * (dSig[p * 3 + 0] * M[0 * 3 + k] + dSig[p * 3 + 1] * M[1 * 3 + k] +
                                 dSig[p * 3 + 2] * M[2 * 3 + k]);
        dR[p * 3 + k] = dM * G.s[k];
        gs[k] += dM * R[p * 3 + k];
      }
    // rotation of the normalised quaternion
    const T w = G.qw, x = G.qx, y = G.qy, z = G.qz;
    const T gw = T(2.0) * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    const T gx = T(2.0) * (y * dR[1] + z * dR[2] + y * dR[3] - T(2.0) * x * dR[4] - w * dR[5] + z * dR[6] +
                             w * dR[7] - T(2.0) * x * dR[8]);
    const T gy = T(2.0) * (-T(2.0) * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                             z * dR[7] - T(2.0) * y * dR[8]);
    const T gz = T(2.0) * (-T(2.0) * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - T(2.0) * z * dR[4] +
                             y * dR[5] + x * dR[6] + y * dR[7]);
    const T dot = w * gw + x * gx + y * gy + z * gz;
    const T iqn = T(1.0) / G.qn;
    gq[0] = (gw - w * dot) * iqn;
    gq[1] = (gx - x * dot) * iqn;
    gq[2] = (gy - y * dot) * iqn;
    gq[3] = (gz - z * dot) * iqn;
  }
  for (int k = 0; k < 3; ++k) put(a.g_means + 3 * i + k, gm[k]);
  for (int k = 0; k < 3; ++k) put(a.g_scales + 3 * i + k, gs[k]);
  for (int k = 0; k < 4; ++k) put(a.g_quats + 4 * i + k, gq[k]);
  put(a.g_opacity + i, gop);
  if (a.g_means2d) {
    put(a.g_means2d + 2 * i, gu);
    put(a.g_means2d + 2 * i + 1, gv);
  }
}

template <typename ShT>
hipError_t launch_fwd_typed(int L, const ProjArgs& args, int blocks, hipStream_t s) {
  switch (L) {
    case 0: hipLaunchKernelGGL((project_fwd_kernel<0, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    case 1: hipLaunchKernelGGL((project_fwd_kernel<1, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    case 2: hipLaunchKernelGGL((project_fwd_kernel<2, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    default: hipLaunchKernelGGL((project_fwd_kernel<3, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
  }
  return hipGetLastError();
}

template <typename ShT>
hipError_t launch_bwd_typed(int L, const ProjBwdArgs& args, int blocks, hipStream_t s) {
  switch (L) {
    case 0: hipLaunchKernelGGL((project_bwd_kernel<0, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    case 1: hipLaunchKernelGGL((project_bwd_kernel<1, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    case 2: hipLaunchKernelGGL((project_bwd_kernel<2, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
    default: hipLaunchKernelGGL((project_bwd_kernel<3, ShT>), dim3(blocks), dim3(256), 0, s, args); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_project_fwd(const CamConst& cc, const fe_config* cfg, const fe_gaussians* g,
                              const StateView& v, hipStream_t s) {
  if (g->n == 0) return hipSuccess;
  ProjArgs a;
  a.cc = cc;
  a.n = g->n;
  a.tile_w = cfg->tile_w;
  a.tile_h = cfg->tile_h;
  a.tiles_x = v.tiles_x;
  a.means = g->means;
  a.scales = g->scales;
  a.quats = g->quats;
  a.opacity = g->opacity;
  a.sh = g->sh;
  a.v = v;
  const int blocks = (int)((g->n + 255) / 256);
  return cfg->sh_dtype == FE_BF16 ? launch_fwd_typed<uint16_t>(cfg->sh_degree, a, blocks, s)
                                  : launch_fwd_typed<float>(cfg->sh_degree, a, blocks, s);
}

hipError_t launch_project_bwd(const CamConst& cc, const fe_config* cfg, const fe_gaussians* g,
                              const StateView& v, const float* grad2d, const fe_grads* out,
                              hipStream_t s) {
  if (g->n == 0) return hipSuccess;
  ProjBwdArgs a;
  a.cc = cc;
  a.n = g->n;
  a.means = g->means;
  a.scales = g->scales;
  a.quats = g->quats;
  a.sh = g->sh;
  a.grad2d = grad2d;
  a.count = v.count;
  a.g_means = out->means;
  a.g_scales = out->scales;
  a.g_quats = out->quats;
  a.g_opacity = out->opacity;
  a.g_sh = out->sh;
  a.g_means2d = out->means2d;
  a.accumulate = (cfg->flags & FE_FLAG_NO_ZERO_GRADS) ? 1 : 0;
  const int blocks = (int)((g->n + 255) / 256);
  return cfg->sh_dtype == FE_BF16 ? launch_bwd_typed<uint16_t>(cfg->sh_degree, a, blocks, s)
                                  : launch_bwd_typed<float>(cfg->sh_degree, a, blocks, s);
}

}  // namespace fe
