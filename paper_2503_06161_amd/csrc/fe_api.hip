// C ABI of libfe4dgs_rast.so: argument validation, state layout and the
// order of kernel launches.  See include/fe4dgs_rast.h for the contract.
#include "fe_common.h"

#include <new>
#include <vector>

#pragma clang fp contract(off)

namespace fe {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

bool compute_layout(const fe_config* cfg, const fe_camera* cam, int64_t n, Layout* L) {
  if (fe_validate(cfg, cam, n) != FE_OK) return false;
  L->n = n;
  L->cap = cfg->key_capacity;
  L->tiles_x = ceil_div(cam->width, cfg->tile_w);
  L->tiles_y = ceil_div(cam->height, cfg->tile_h);
  L->tiles = L->tiles_x * L->tiles_y;
  L->nblk = ceil_div(n, kBinChunk);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  // zeroed at the start of every forward: report, tile counts, ranges
  L->report = take(sizeof(unsigned long long) * 2 * kRepWords);
  L->tile_cnt = take(sizeof(uint32_t) * (size_t)L->tiles);
  L->ranges = take(sizeof(uint2) * (size_t)L->tiles);
  L->xy = take(sizeof(float2) * n);
  L->conic_o = take(sizeof(float4) * n);
  L->rgb = take(sizeof(float4) * n);
  L->box = take(sizeof(short4) * n);
  L->dkey = take(4 * n);
  L->count = take(4 * n);
  L->rel = take(L->tiles <= kBinLdsTiles ? 4 * (size_t)L->nblk * (size_t)L->tiles : 0);
  L->blk_sum = take(4 * (size_t)L->nblk);
  L->blk_off = take(4 * (size_t)L->nblk);
  L->blk_vis = take(4 * (size_t)L->nblk);
  L->keys = take(8 * (size_t)L->cap);
  L->keys_b = take(8 * (size_t)L->cap);
  L->gauss = take(4 * (size_t)L->cap);
  L->tile_maxlast = take(4 * (size_t)L->tiles);
  L->gofe = take(4 * (size_t)L->cap);
  L->epos = take(4 * (size_t)L->cap);
  L->eoff = take(4 * n);
  L->tile_order = take(4 * (size_t)L->tiles);
  L->total = o;
  return true;
}

StateView make_view(const Layout& L, void* base) {
  char* b = static_cast<char*>(base);
  StateView v;
  v.xy = reinterpret_cast<float2*>(b + L.xy);
  v.conic_o = reinterpret_cast<float4*>(b + L.conic_o);
  v.rgb = reinterpret_cast<float4*>(b + L.rgb);
  v.box = reinterpret_cast<short4*>(b + L.box);
  v.dkey = reinterpret_cast<uint32_t*>(b + L.dkey);
  v.count = reinterpret_cast<uint32_t*>(b + L.count);
  v.tile_cnt = reinterpret_cast<uint32_t*>(b + L.tile_cnt);
  v.rel = reinterpret_cast<uint32_t*>(b + L.rel);
  v.blk_sum = reinterpret_cast<uint32_t*>(b + L.blk_sum);
  v.blk_off = reinterpret_cast<uint32_t*>(b + L.blk_off);
  v.blk_vis = reinterpret_cast<uint32_t*>(b + L.blk_vis);
  v.keys = reinterpret_cast<unsigned long long*>(b + L.keys);
  v.keys_b = reinterpret_cast<unsigned long long*>(b + L.keys_b);
  v.gauss = reinterpret_cast<uint32_t*>(b + L.gauss);
  v.ranges = reinterpret_cast<uint2*>(b + L.ranges);
  v.report = reinterpret_cast<unsigned long long*>(b + L.report);
  v.tile_maxlast = reinterpret_cast<uint32_t*>(b + L.tile_maxlast);
  v.gofe = reinterpret_cast<uint32_t*>(b + L.gofe);
  v.epos = reinterpret_cast<uint32_t*>(b + L.epos);
  v.eoff = reinterpret_cast<uint32_t*>(b + L.eoff);
  v.tile_order = reinterpret_cast<uint32_t*>(b + L.tile_order);
  v.n = L.n;
  v.cap = L.cap;
  v.tiles_x = L.tiles_x;
  v.tiles_y = L.tiles_y;
  v.tiles = L.tiles;
  v.nblk = L.nblk;
  return v;
}

CamConst make_cam_const(const fe_camera* cam, const fe_config* cfg) {
  CamConst c;
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) c.R[r * 3 + k] = cam->world_to_cam[r * 4 + k];
    c.t[r] = cam->world_to_cam[r * 4 + 3];
  }
  for (int k = 0; k < 3; ++k) c.campos[k] = -((c.R[0 * 3 + k] * c.t[0] + c.R[1 * 3 + k] * c.t[1]) + c.R[2 * 3 + k] * c.t[2]);
  c.fx = cam->fx;
  c.fy = cam->fy;
  c.cx = cam->cx;
  c.cy = cam->cy;
  const double k = cfg->jacobian_clamp;
  if (k > 0.0) {
    c.limx = (k * (double)cam->width) / (2.0 * c.fx);
    c.limy = (k * (double)cam->height) / (2.0 * c.fy);
  } else {
    c.limx = 0.0;
    c.limy = 0.0;
  }
  c.near_plane = cam->near_plane;
  c.dilation = cfg->cov2d_dilation;
  c.width = cam->width;
  c.height = cam->height;
  return c;
}

static fe_status hip_status(hipError_t e) { return e == hipSuccess ? FE_OK : FE_ERR_HIP; }

// backward scratch: grad2d [n][12] | row_base [tiles + 1], tile order [tiles] | rowidx [cap] | rows [row_cap][RS]
struct BwdScratch {
  size_t grad2d, row_base, rowidx, rows, total;
  int64_t row_cap;
};

static bool bwd_scratch_layout(const fe_config* cfg, const fe_camera* cam, int64_t n, BwdScratch* b) {
  Layout L;
  if (!compute_layout(cfg, cam, n, &L)) return false;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  b->grad2d = take(sizeof(float) * 12 * (size_t)(n > 0 ? n : 1));
  b->row_cap = 0;
  b->row_base = b->rowidx = b->rows = o;
  if (cfg->variant != FE_VARIANT_VALU) {
    b->row_cap = cfg->row_capacity > 0 ? cfg->row_capacity : cfg->key_capacity;
    b->row_base = take(sizeof(uint32_t) * (2 * (size_t)L.tiles + 1));   // row offsets, then the launch order
    b->rowidx = take(sizeof(uint32_t) * (((size_t)L.cap + 3) & ~(size_t)3));   // whole 16-byte groups
    b->rows = take(sizeof(float) * (size_t)backward_row_stride(cfg->feat_dim) * (size_t)b->row_cap);
  }
  b->total = o;
  return true;
}

// optional per-stage events (recorded on the call's stream)
static void stage_mark(const fe_config* cfg, int stage, int end, hipStream_t s) {
  if (!cfg->stage_events) return;
  void* ev = cfg->stage_events[2 * stage + end];
  if (ev) (void)hipEventRecord(static_cast<hipEvent_t>(ev), s);
}

static fe_status check_gaussians(const fe_config* cfg, const fe_gaussians* g) {
  if (!g || g->n < 0) return FE_ERR_INVALID_ARG;
  if (g->n == 0) return FE_OK;
  if (!g->means || !g->scales || !g->quats || !g->opacity || !g->sh || !g->feat) return FE_ERR_INVALID_ARG;
  // element alignment everywhere; SH rows are read with 16-byte loads
  auto misaligned = [](const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; };
  if (misaligned(g->means, 4) || misaligned(g->scales, 4) || misaligned(g->quats, 4) || misaligned(g->opacity, 4) ||
      misaligned(g->sh, 16) || misaligned(g->feat, cfg->feat_dtype == FE_BF16 ? 2 : 4))
    return FE_ERR_INVALID_ARG;
  return FE_OK;
}

// forward up to the compositing: projection, binning and sorting
static fe_status forward_pre(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, void* state,
                             const Layout& L, hipStream_t s) {
  StateView v = make_view(L, state);
  hipError_t e;
  const size_t zero_words = (L.ranges + sizeof(uint2) * (size_t)L.tiles - L.report) / 4;
  if ((e = launch_zero_u32(reinterpret_cast<uint32_t*>(v.report), zero_words, s)) != hipSuccess) return FE_ERR_HIP;
  stage_mark(cfg, FE_STAGE_PROJECT, 0, s);
  if ((e = launch_project_fwd(make_cam_const(cam, cfg), cfg, g, v, s)) != hipSuccess) return FE_ERR_HIP;
  stage_mark(cfg, FE_STAGE_PROJECT, 1, s);
  stage_mark(cfg, FE_STAGE_SORT, 0, s);
  if ((e = launch_sort_and_bin(cfg, v, s)) != hipSuccess) return FE_ERR_HIP;
  stage_mark(cfg, FE_STAGE_SORT, 1, s);
  return FE_OK;
}

static fe_status forward_impl(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                              const fe_images* out, void* state, const Layout& L, hipStream_t s) {
  const fe_status st = forward_pre(cfg, cam, g, state, L, s);
  if (st != FE_OK) return st;
  StateView v = make_view(L, state);
  stage_mark(cfg, FE_STAGE_COMPOSITE, 0, s);
  const hipError_t e = cfg->variant == FE_VARIANT_VALU ? launch_composite_fwd(cfg, cam, g, v, out, s)
                                                       : launch_composite_fwd_mfma(cfg, cam, g, v, out, s);
  stage_mark(cfg, FE_STAGE_COMPOSITE, 1, s);
  return hip_status(e);
}

// backward of the matrix-core form around its compositing kernel: row
// offsets of the tiles before, the per-Gaussian sums and the projection
// backward after
struct BwdBuffers {
  float* grad2d;
  uint32_t* row_base;
  uint32_t* rowidx;
  float* rows;
  int64_t row_cap;
};

static BwdBuffers bwd_buffers(const fe_config* cfg, const fe_camera* cam, int64_t n, void* scratch) {
  BwdScratch bs;
  bwd_scratch_layout(cfg, cam, n, &bs);
  char* sb = static_cast<char*>(scratch);
  BwdBuffers b;
  b.grad2d = reinterpret_cast<float*>(sb + bs.grad2d);
  b.row_base = reinterpret_cast<uint32_t*>(sb + bs.row_base);
  b.rowidx = reinterpret_cast<uint32_t*>(sb + bs.rowidx);
  b.rows = reinterpret_cast<float*>(sb + bs.rows);
  b.row_cap = bs.row_cap;
  return b;
}

static fe_status backward_pre(const Layout& L, const void* state, const BwdBuffers& b, hipStream_t s) {
  StateView v = make_view(L, const_cast<void*>(state));
  return hip_status(launch_backward_prep(v.tile_maxlast, b.row_base, v.tiles, L.tiles_x, b.rowidx, v.report, L.cap, s));
}

static fe_status backward_post(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g, const Layout& L,
                               const void* state, const BwdBuffers& b, const fe_grads* out, hipStream_t s) {
  StateView v = make_view(L, const_cast<void*>(state));
  stage_mark(cfg, FE_STAGE_REDUCE, 0, s);
  if (launch_reduce_rows(cfg, v, b.rowidx, b.rows, b.grad2d, out->feat, s) != hipSuccess) return FE_ERR_HIP;
  stage_mark(cfg, FE_STAGE_REDUCE, 1, s);
  stage_mark(cfg, FE_STAGE_PROJECT_BWD, 0, s);
  const hipError_t e = launch_project_bwd(make_cam_const(cam, cfg), cfg, g, v, b.grad2d, out, s);
  stage_mark(cfg, FE_STAGE_PROJECT_BWD, 1, s);
  return hip_status(e);
}

static fe_status backward_impl(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                               const fe_images* fwd, const void* state, const Layout& L, const float* d_rgb,
                               const float* d_feat, const float* d_depth, const fe_grads* out, void* scratch,
                               hipStream_t s) {
  StateView v = make_view(L, const_cast<void*>(state));
  const BwdBuffers b = bwd_buffers(cfg, cam, g->n, scratch);
  hipError_t e;
  if (cfg->variant != FE_VARIANT_VALU) {
    fe_status st = backward_pre(L, state, b, s);
    if (st != FE_OK) return st;
    stage_mark(cfg, FE_STAGE_COMPOSITE_BWD, 0, s);
    if ((e = launch_composite_bwd_mfma(cfg, cam, g, v, fwd, d_rgb, d_feat, d_depth, b.row_base, b.rows, b.row_cap,
                                       b.rowidx, s)) != hipSuccess)
      return FE_ERR_HIP;
    stage_mark(cfg, FE_STAGE_COMPOSITE_BWD, 1, s);
    return backward_post(cfg, cam, g, L, state, b, out, s);
  }
  if ((e = launch_zero_u32(reinterpret_cast<uint32_t*>(b.grad2d), (size_t)12 * g->n, s)) != hipSuccess)
    return FE_ERR_HIP;
  if (!(cfg->flags & FE_FLAG_NO_ZERO_GRADS)) {
    if ((e = launch_zero_u32(reinterpret_cast<uint32_t*>(out->feat), (size_t)cfg->feat_dim * g->n, s)) != hipSuccess)
      return FE_ERR_HIP;
  }
  stage_mark(cfg, FE_STAGE_COMPOSITE_BWD, 0, s);
  if ((e = launch_composite_bwd(cfg, cam, g, v, fwd, d_rgb, d_feat, d_depth, b.grad2d, out->feat, s)) != hipSuccess)
    return FE_ERR_HIP;
  stage_mark(cfg, FE_STAGE_COMPOSITE_BWD, 1, s);
  stage_mark(cfg, FE_STAGE_PROJECT_BWD, 0, s);
  e = launch_project_bwd(make_cam_const(cam, cfg), cfg, g, v, b.grad2d, out, s);
  stage_mark(cfg, FE_STAGE_PROJECT_BWD, 1, s);
  return hip_status(e);
}

}  // namespace fe

using namespace fe;

extern "C" {

int fe_abi_version(void) { return FE4DGS_ABI_VERSION; }

const char* fe_status_string(fe_status s) {
  switch (s) {
    case FE_OK: return "ok";
    case FE_ERR_INVALID_ARG: return "invalid argument";
    case FE_ERR_UNSUPPORTED: return "unsupported configuration";
    case FE_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case FE_ERR_KEY_OVERFLOW: return "sort key capacity exceeded";
    case FE_ERR_HIP: return "HIP runtime error";
    case FE_ERR_ROW_OVERFLOW: return "backward row capacity exceeded";
  }
  return "unknown status";
}

fe_status fe_validate(const fe_config* cfg, const fe_camera* cam, int64_t n) {
  if (!cfg || !cam || n < 0) return FE_ERR_INVALID_ARG;
  if (cam->width < 1 || cam->height < 1) return FE_ERR_INVALID_ARG;
  if (cam->width > 32767 || cam->height > 32767) return FE_ERR_UNSUPPORTED;
  if (!(cam->fx > 0.f) || !(cam->fy > 0.f)) return FE_ERR_INVALID_ARG;
  const int tw = cfg->tile_w, th = cfg->tile_h;
  if (!(tw == 8 || tw == 16 || tw == 32)) return FE_ERR_UNSUPPORTED;
  const int nt = tw * th;
  if (th < 1 || (nt != 64 && nt != 128 && nt != 256)) return FE_ERR_UNSUPPORTED;
  // threads per tile: 0 (library choice), one per pixel, or two per pixel
  // where the wave-specialized kernels exist in both directions (matrix-core
  // variant, BF16 features, D <= 128)
  if (cfg->threads_per_tile != 0 && cfg->threads_per_tile != nt) {
    if (cfg->threads_per_tile != 2 * nt) return FE_ERR_UNSUPPORTED;
    if (cfg->variant == FE_VARIANT_VALU || cfg->feat_dtype != FE_BF16 || cfg->feat_dim > 128)
      return FE_ERR_UNSUPPORTED;
  }
  if (cfg->sh_degree < 0) return FE_ERR_INVALID_ARG;
  if (cfg->sh_degree > 3) return FE_ERR_UNSUPPORTED;
  if (cfg->feat_dim < 1) return FE_ERR_INVALID_ARG;
  if (cfg->feat_dim > 256) return FE_ERR_UNSUPPORTED;
  if ((cfg->sh_dtype != FE_F32 && cfg->sh_dtype != FE_BF16) ||
      (cfg->feat_dtype != FE_F32 && cfg->feat_dtype != FE_BF16))
    return FE_ERR_INVALID_ARG;
  if (cfg->key_capacity < 0 || cfg->key_capacity > 0x7FFFFFFFll) return FE_ERR_INVALID_ARG;
  if (n > kMaxGaussians) return FE_ERR_UNSUPPORTED;
  if (cfg->variant != FE_VARIANT_AUTO && cfg->variant != FE_VARIANT_VALU && cfg->variant != FE_VARIANT_MFMA)
    return FE_ERR_UNSUPPORTED;
  return FE_OK;
}

size_t fe_state_bytes(const fe_config* cfg, const fe_camera* cam, int64_t n) {
  Layout L;
  if (!compute_layout(cfg, cam, n, &L)) return 0;
  return L.total;
}

fe_status fe_state_layout_get(const fe_config* cfg, const fe_camera* cam, int64_t n, fe_state_layout* out) {
  if (!out) return FE_ERR_INVALID_ARG;
  const fe_status st = fe_validate(cfg, cam, n);
  if (st != FE_OK) return st;
  Layout L;
  compute_layout(cfg, cam, n, &L);
  out->total = L.total;
  out->xy = L.xy;
  out->conic_opacity = L.conic_o;
  out->rgb = L.rgb;
  out->box = L.box;
  out->depth_key = L.dkey;
  out->tile_count = L.count;
  out->sorted_gauss = L.gauss;
  out->ranges = L.ranges;
  out->report = L.report;
  return FE_OK;
}

size_t fe_backward_scratch_bytes(const fe_config* cfg, const fe_camera* cam, int64_t n) {
  BwdScratch b;
  if (!bwd_scratch_layout(cfg, cam, n, &b)) return 0;
  return b.total;
}

fe_status fe_render_forward(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                            const fe_images* out, void* state, size_t state_bytes, void* stream) {
  fe_status st = fe_validate(cfg, cam, g ? g->n : -1);
  if (st != FE_OK) return st;
  if ((st = check_gaussians(cfg, g)) != FE_OK) return st;
  if (!out || !out->rgb || !out->feat || !out->final_T || !out->n_contrib || !state) return FE_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(state) % 256 != 0) return FE_ERR_INVALID_ARG;   // regions are 256-byte aligned
  Layout L;
  compute_layout(cfg, cam, g->n, &L);
  if (state_bytes < L.total) return FE_ERR_WORKSPACE_TOO_SMALL;
  return forward_impl(cfg, cam, g, out, state, L, static_cast<hipStream_t>(stream));
}

fe_status fe_render_backward(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                             const fe_images* fwd, const void* state, size_t state_bytes,
                             const float* d_rgb, const float* d_feat, const float* d_depth, const fe_grads* out,
                             void* scratch, size_t scratch_bytes, void* stream) {
  fe_status st = fe_validate(cfg, cam, g ? g->n : -1);
  if (st != FE_OK) return st;
  if ((st = check_gaussians(cfg, g)) != FE_OK) return st;
  if (!fwd || !fwd->final_T || !fwd->n_contrib || !state || !d_rgb || !d_feat || !out || !scratch ||
      reinterpret_cast<uintptr_t>(state) % 256 != 0 || reinterpret_cast<uintptr_t>(scratch) % 256 != 0)
    return FE_ERR_INVALID_ARG;
  if (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh || !out->feat)
    return FE_ERR_INVALID_ARG;
  Layout L;
  compute_layout(cfg, cam, g->n, &L);
  if (state_bytes < L.total) return FE_ERR_WORKSPACE_TOO_SMALL;
  if (scratch_bytes < fe_backward_scratch_bytes(cfg, cam, g->n)) return FE_ERR_WORKSPACE_TOO_SMALL;
  if (g->n == 0) return FE_OK;
  return backward_impl(cfg, cam, g, fwd, state, L, d_rgb, d_feat, d_depth, out, scratch,
                       static_cast<hipStream_t>(stream));
}

// one partial (dW, db, loss) per workgroup of the persistent decoder grid,
// then the sign masks (2 bits per output value)
static size_t decoder_partial_bytes(int32_t in_dim, int target_dtype) {
  const int grid = decoder_grid_size(in_dim, target_dtype);
  return grid < 1 ? 0 : align256((size_t)grid * decoder_partial_floats(in_dim) * sizeof(float));
}

size_t fe_decoder_workspace_bytes(int32_t in_dim, int64_t pixels) {
  if ((in_dim != 32 && in_dim != 64 && in_dim != 128) || pixels < 1) return 0;
  const size_t a = decoder_partial_bytes(in_dim, FE_F32), b = decoder_partial_bytes(in_dim, FE_BF16);
  if (!a || !b) return 0;
  return (a > b ? a : b) + decoder_sign_bytes(pixels);
}

fe_status fe_decoder_l1(const fe_decoder* d, void* workspace, size_t workspace_bytes, void* stream) {
  if (!d || !workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FE_ERR_INVALID_ARG;
  if (d->in_dim != 32 && d->in_dim != 64 && d->in_dim != 128) return FE_ERR_UNSUPPORTED;
  if (d->target_dtype != FE_F32 && d->target_dtype != FE_BF16) return FE_ERR_INVALID_ARG;
  if (d->pixels < 1 || d->pixels > ((int64_t)1 << 24)) return FE_ERR_INVALID_ARG;
  if (!d->feat || !d->weight || !d->bias || !d->target || !d->loss || !d->d_weight || !d->d_bias)
    return FE_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(d->weight) % 16 != 0) return FE_ERR_INVALID_ARG;
  int grid = decoder_grid_size(d->in_dim, d->target_dtype);
  if (grid < 1) return FE_ERR_HIP;
  // at least 16 pixel blocks per workgroup, so that small maps do not pay
  // for a full grid of partial gradients
  const int64_t blocks = (d->pixels + 31) / 32, need = (blocks + 15) / 16;
  if (need < grid) grid = (int)need;
  const size_t part = decoder_partial_bytes(d->in_dim, d->target_dtype);
  if (workspace_bytes < part + decoder_sign_bytes(d->pixels)) return FE_ERR_WORKSPACE_TOO_SMALL;
  char* ws = static_cast<char*>(workspace);
  return hip_status(launch_decoder_l1(d, grid, reinterpret_cast<float*>(ws), ws + part,
                                      static_cast<hipStream_t>(stream)));
}

fe_status fe_read_report(const void* state, size_t state_bytes, fe_report* out, void* stream) {
  if (!state || !out || state_bytes < sizeof(unsigned long long) * kRepWords) return FE_ERR_INVALID_ARG;
  unsigned long long w[kRepWords];
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(w, state, sizeof(w), hipMemcpyDeviceToHost, s) != hipSuccess) return FE_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return FE_ERR_HIP;
  out->status = (int32_t)(w[kRepStatus] != 0 ? w[kRepStatus] : w[kRepBwdStatus]);
  out->backward_status = (int32_t)w[kRepBwdStatus];
  out->keys_needed = (int64_t)w[kRepKeys];
  out->n_visible = (int64_t)w[kRepVisible];
  out->n_culled_nonfinite = (int64_t)w[kRepNonFinite];
  out->rows_needed = (int64_t)w[kRepRows];
  return (fe_status)out->status;
}

// ------------------------------------------------------------------------
// Batched frames captured into one HIP graph.
//
// Where the wave-specialized compositing kernels apply (BF16 features,
// D <= 128, frames of one image size), the compositing of all frames runs as
// one persistent launch per direction: the per-frame stages before it run on
// parallel branches, a single workgroup then builds a queue of every
// (frame, tile) item ordered longest first, and the persistent workgroups take
// items from it.  Otherwise every frame runs its own kernels.
// ------------------------------------------------------------------------
struct MultiLayout {
  size_t rec_f, rec_b, rng, walk, items_f, items_b, qwords, total;
};

struct fe_batch_plan {
  fe_config cfg;
  int32_t frames;
  int32_t mode;
  std::vector<fe_camera> cams;
  std::vector<fe_gaussians> g;
  std::vector<fe_images> out;
  std::vector<const float*> d_rgb, d_feat, d_depth;
  std::vector<fe_grads> grads;
  std::vector<Layout> layouts;
  std::vector<size_t> state_off, scratch_off;
  bool persistent;
  size_t multi_off;
  MultiLayout ml;
  int grid_f, grid_b;
  char* ws;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};

static bool batch_persistent(const fe_config* cfg, const fe_camera* cams, int32_t frames) {
  if ((cfg->flags & FE_FLAG_BATCH_PER_FRAME) || !composite_persistent_supported(cfg)) return false;
  for (int f = 1; f < frames; ++f)
    if (cams[f].width != cams[0].width || cams[f].height != cams[0].height) return false;
  return true;
}

static size_t multi_layout(int32_t frames, int64_t tiles, MultiLayout* m) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  m->rec_f = take(frames * composite_fwd_record_bytes());
  m->rec_b = take(frames * composite_bwd_record_bytes());
  m->rng = take(frames * sizeof(void*));
  m->walk = take(frames * sizeof(void*));
  m->items_f = take((size_t)frames * tiles * sizeof(uint2));
  m->items_b = take((size_t)frames * tiles * sizeof(uint2));
  m->qwords = take(4 * sizeof(uint32_t));   // forward count, head; backward count, head
  m->total = o;
  return o;
}

static size_t batch_layout(const fe_config* cfg, const fe_camera* cams, int32_t frames, const int64_t* n,
                           std::vector<Layout>* layouts, std::vector<size_t>* st_off,
                           std::vector<size_t>* sc_off, size_t* multi_off = nullptr, MultiLayout* ml = nullptr) {
  size_t o = 0;
  int64_t tiles = 0;
  for (int f = 0; f < frames; ++f) {
    Layout L;
    if (!compute_layout(cfg, &cams[f], n[f], &L)) return 0;
    tiles = L.tiles;
    if (layouts) layouts->push_back(L);
    if (st_off) st_off->push_back(o);
    o = align256(o + L.total);
    if (sc_off) sc_off->push_back(o);
    o = align256(o + fe_backward_scratch_bytes(cfg, &cams[f], n[f]));
  }
  if (batch_persistent(cfg, cams, frames)) {
    MultiLayout m;
    if (multi_off) *multi_off = o;
    o = align256(o + multi_layout(frames, tiles, &m));
    if (ml) *ml = m;
  }
  return o;
}

size_t fe_batch_workspace_bytes(const fe_config* cfg, const fe_camera* cams, int32_t frames, const int64_t* n) {
  if (!cfg || !cams || !n || frames < 1) return 0;
  return batch_layout(cfg, cams, frames, n, nullptr, nullptr, nullptr);
}

fe_status fe_batch_plan_create(const fe_config* cfg, const fe_camera* cams, int32_t frames,
                               const fe_gaussians* g, const fe_images* out,
                               const float* const* d_rgb, const float* const* d_feat,
                               const float* const* d_depth, const fe_grads* grads, int32_t mode, void* workspace,
                               size_t workspace_bytes, fe_batch_plan** plan) {
  if (!plan) return FE_ERR_INVALID_ARG;
  *plan = nullptr;
  if (!cfg || !cams || frames < 1 || !g || !out || !workspace) return FE_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FE_ERR_INVALID_ARG;
  if (mode != FE_MODE_FORWARD && mode != FE_MODE_BACKWARD && mode != FE_MODE_FORWARD_BACKWARD)
    return FE_ERR_INVALID_ARG;
  const bool bwd = (mode & FE_MODE_BACKWARD) != 0;
  if (bwd && (!d_rgb || !d_feat || !grads)) return FE_ERR_INVALID_ARG;
  std::vector<int64_t> n(frames);
  for (int f = 0; f < frames; ++f) {
    fe_status st = fe_validate(cfg, &cams[f], g[f].n);
    if (st != FE_OK) return st;
    if ((st = check_gaussians(cfg, &g[f])) != FE_OK) return st;
    if (!out[f].rgb || !out[f].feat || !out[f].final_T || !out[f].n_contrib) return FE_ERR_INVALID_ARG;
    if (bwd) {
      if (!d_rgb[f] || !d_feat[f]) return FE_ERR_INVALID_ARG;
      const fe_grads& gr = grads[f];   // a frame without Gaussians has no gradients
      if (g[f].n > 0 && (!gr.means || !gr.scales || !gr.quats || !gr.opacity || !gr.sh || !gr.feat))
        return FE_ERR_INVALID_ARG;
    }
    n[f] = g[f].n;
  }
  fe_batch_plan* p = new (std::nothrow) fe_batch_plan();
  if (!p) return FE_ERR_INVALID_ARG;
  p->multi_off = 0;
  const size_t need = batch_layout(cfg, cams, frames, n.data(), &p->layouts, &p->state_off, &p->scratch_off,
                                   &p->multi_off, &p->ml);
  if (workspace_bytes < need) {
    delete p;
    return FE_ERR_WORKSPACE_TOO_SMALL;
  }
  p->cfg = *cfg;
  p->cfg.stage_events = nullptr;
  p->frames = frames;
  p->mode = mode;
  p->cams.assign(cams, cams + frames);
  p->g.assign(g, g + frames);
  p->out.assign(out, out + frames);
  if (bwd) {
    p->d_rgb.assign(d_rgb, d_rgb + frames);
    p->d_feat.assign(d_feat, d_feat + frames);
    if (d_depth)
      p->d_depth.assign(d_depth, d_depth + frames);
    else
      p->d_depth.assign(frames, nullptr);
    p->grads.assign(grads, grads + frames);
  }
  p->persistent = batch_persistent(cfg, cams, frames);
  p->grid_f = p->grid_b = 0;
  if (p->persistent) {
    p->grid_f = composite_fwd_persistent_grid(cfg);
    p->grid_b = composite_bwd_persistent_grid(cfg);
    if (p->grid_f < 1 || p->grid_b < 1) {
      delete p;
      return FE_ERR_HIP;
    }
  }
  p->ws = static_cast<char*>(workspace);
  p->graph = nullptr;
  p->exec = nullptr;
  p->captured = false;
  *plan = p;
  return FE_OK;
}

// Frames are independent: frame f's stages are enqueued on branch stream
// f % kBranches, forked from and joined back into the capture stream, so the
// captured graph has parallel chains the GPU may overlap.
constexpr int kBranches = 4;

struct Branches {
  int n = 0;
  hipStream_t s[kBranches] = {};
  std::vector<hipEvent_t> events;
  bool create(int frames) {
    n = frames < kBranches ? frames : kBranches;
    for (int b = 0; b < n; ++b)
      if (hipStreamCreateWithFlags(&s[b], hipStreamNonBlocking) != hipSuccess) return false;
    return true;
  }
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    events.push_back(e);
    return e;
  }
  // the branches wait for everything enqueued on cs so far
  bool fork(hipStream_t cs) {
    hipEvent_t e = event();
    if (!e || hipEventRecord(e, cs) != hipSuccess) return false;
    for (int b = 0; b < n; ++b)
      if (hipStreamWaitEvent(s[b], e, 0) != hipSuccess) return false;
    return true;
  }
  // cs waits for everything enqueued on the branches so far
  bool join(hipStream_t cs) {
    bool ok = true;
    for (int b = 0; b < n; ++b) {
      hipEvent_t e = event();
      ok = ok && e && hipEventRecord(e, s[b]) == hipSuccess && hipStreamWaitEvent(cs, e, 0) == hipSuccess;
    }
    return ok;
  }
  ~Branches() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (int b = 0; b < kBranches; ++b)
      if (s[b]) (void)hipStreamDestroy(s[b]);
  }
};

static fe_status frame_enqueue(fe_batch_plan* p, int f, hipStream_t s) {
  fe_status st = FE_OK;
  if (p->mode & FE_MODE_FORWARD)
    st = forward_impl(&p->cfg, &p->cams[f], &p->g[f], &p->out[f], p->ws + p->state_off[f], p->layouts[f], s);
  if (st == FE_OK && (p->mode & FE_MODE_BACKWARD) && p->g[f].n > 0)
    st = backward_impl(&p->cfg, &p->cams[f], &p->g[f], &p->out[f], p->ws + p->state_off[f], p->layouts[f],
                       p->d_rgb[f], p->d_feat[f], p->d_depth[f], &p->grads[f], p->ws + p->scratch_off[f], s);
  return st;
}

// Frame records and the per-frame pointer tables of the persistent path,
// written once before the capture.
static fe_status upload_multi(fe_batch_plan* p) {
  const int F = p->frames;
  const bool bwd = (p->mode & FE_MODE_BACKWARD) != 0;
  char* m = p->ws + p->multi_off;
  const size_t rf = composite_fwd_record_bytes(), rb = composite_bwd_record_bytes();
  std::vector<char> recf(F * rf), recb(bwd ? F * rb : 0);
  std::vector<const void*> rng(F), walk(F);
  for (int f = 0; f < F; ++f) {
    StateView v = make_view(p->layouts[f], p->ws + p->state_off[f]);
    composite_fwd_record(&p->cfg, &p->cams[f], &p->g[f], v, &p->out[f], recf.data() + f * rf);
    if (bwd) {
      const BwdBuffers b = bwd_buffers(&p->cfg, &p->cams[f], p->g[f].n, p->ws + p->scratch_off[f]);
      composite_bwd_record(&p->cfg, &p->cams[f], &p->g[f], v, &p->out[f], p->d_rgb[f], p->d_feat[f], p->d_depth[f],
                           b.row_base, b.rows, b.row_cap, b.rowidx, recb.data() + f * rb);
    }
    rng[f] = v.ranges;
    walk[f] = v.tile_maxlast;
  }
  bool ok = hipMemcpy(m + p->ml.rec_f, recf.data(), recf.size(), hipMemcpyHostToDevice) == hipSuccess;
  if (bwd) ok = ok && hipMemcpy(m + p->ml.rec_b, recb.data(), recb.size(), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(m + p->ml.rng, rng.data(), F * sizeof(void*), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(m + p->ml.walk, walk.data(), F * sizeof(void*), hipMemcpyHostToDevice) == hipSuccess;
  return ok ? FE_OK : FE_ERR_HIP;
}

static fe_status composite_all(fe_batch_plan* p, bool backward, hipStream_t cs) {
  char* m = p->ws + p->multi_off;
  uint32_t* qw = reinterpret_cast<uint32_t*>(m + p->ml.qwords) + (backward ? 2 : 0);
  TileQueueBuild qb;
  qb.frames = p->frames;
  qb.tiles = (int32_t)p->layouts[0].tiles;
  qb.ranges = reinterpret_cast<const uint2* const*>(m + p->ml.rng);
  qb.walk = backward ? reinterpret_cast<const uint32_t* const*>(m + p->ml.walk) : nullptr;
  qb.items = reinterpret_cast<uint2*>(m + (backward ? p->ml.items_b : p->ml.items_f));
  qb.count = qw;
  qb.head = qw + 1;
  if (launch_build_tile_queue(qb, cs) != hipSuccess) return FE_ERR_HIP;
  TileQueue q{qb.items, qb.count, qb.head};
  const hipError_t e = backward ? launch_composite_bwd_persistent(&p->cfg, m + p->ml.rec_b, q, p->grid_b, cs)
                                : launch_composite_fwd_persistent(&p->cfg, m + p->ml.rec_f, q, p->grid_f, cs);
  return hip_status(e);
}

static fe_status batch_enqueue(fe_batch_plan* p, hipStream_t cs, Branches& br) {
  fe_status st = FE_OK;
  if (!p->persistent) {
    if (!br.fork(cs)) return FE_ERR_HIP;
    for (int f = 0; st == FE_OK && f < p->frames; ++f) st = frame_enqueue(p, f, br.s[f % br.n]);
    // always join the branches so that the capture ends cleanly
    return br.join(cs) ? st : FE_ERR_HIP;
  }
  auto per_frame = [&](auto&& stage) {
    if (!br.fork(cs)) return FE_ERR_HIP;
    fe_status r = FE_OK;
    for (int f = 0; r == FE_OK && f < p->frames; ++f) r = stage(f, br.s[f % br.n]);
    return br.join(cs) ? r : FE_ERR_HIP;
  };
  if (p->mode & FE_MODE_FORWARD) {
    st = per_frame([&](int f, hipStream_t s) {
      return forward_pre(&p->cfg, &p->cams[f], &p->g[f], p->ws + p->state_off[f], p->layouts[f], s);
    });
    if (st == FE_OK) st = composite_all(p, false, cs);
  }
  if (st == FE_OK && (p->mode & FE_MODE_BACKWARD)) {
    auto buffers = [&](int f) { return bwd_buffers(&p->cfg, &p->cams[f], p->g[f].n, p->ws + p->scratch_off[f]); };
    st = per_frame([&](int f, hipStream_t s) {
      return p->g[f].n > 0 ? backward_pre(p->layouts[f], p->ws + p->state_off[f], buffers(f), s) : FE_OK;
    });
    if (st == FE_OK) st = composite_all(p, true, cs);
    if (st == FE_OK)
      st = per_frame([&](int f, hipStream_t s) {
        return p->g[f].n > 0 ? backward_post(&p->cfg, &p->cams[f], &p->g[f], p->layouts[f],
                                             p->ws + p->state_off[f], buffers(f), &p->grads[f], s)
                             : FE_OK;
      });
  }
  return st;
}

fe_status fe_batch_launch(fe_batch_plan* p, void* stream) {
  if (!p) return FE_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!p->captured) {
    if (p->persistent) {
      const fe_status st = upload_multi(p);
      if (st != FE_OK) return st;
    }
    // capture on a private non-default stream so that the caller's stream may be
    // the legacy default stream
    Branches br;
    if (!br.create(p->frames)) return FE_ERR_HIP;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return FE_ERR_HIP;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return FE_ERR_HIP;
    }
    const fe_status st = batch_enqueue(p, cs, br);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != FE_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess || !graph) return FE_ERR_HIP;
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return FE_ERR_HIP;
    }
    p->graph = graph;
    p->exec = exec;
    p->captured = true;
  }
  return hip_status(hipGraphLaunch(p->exec, s));
}

fe_status fe_batch_read_report(fe_batch_plan* p, int32_t f, fe_report* out, void* stream) {
  if (!p || f < 0 || f >= p->frames) return FE_ERR_INVALID_ARG;
  return fe_read_report(p->ws + p->state_off[f], p->layouts[f].total, out, stream);
}

void fe_batch_plan_destroy(fe_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

}  // extern "C"
