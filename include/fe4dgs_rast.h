/*
 * fe4dgs_rast.h -- C ABI of the MI355X (gfx950) tile rasterizer for
 * feature-distilled 4D Gaussian splatting (FeatureEndo-4DGS).
 *
 * What the library computes (the paper's Sec. 3.3, "Differentiable Rendering
 * and Loss Functions", and Sec. 3.1):
 *   - each deformed Gaussian G_t (eq. 6) is projected: Sigma = R S S^T R^T
 *     (eq. 2) and Sigma' = J W Sigma W^T J^T (eq. 9), plus a 0.3 px^2
 *     dilation of the diagonal;
 *   - it is binned into screen tiles by its 3-sigma pixel box, and every
 *     tile's list is ordered front to back (by view-space depth, ties by
 *     Gaussian index);
 *   - every pixel blends colour, depth and the D semantic channels front to
 *     back with the same weights alpha_i prod_{j<i}(1 - alpha_j) (eqs. 7 and
 *     8; colour, depth and semantics in one pass, Sec. 3 overview), where
 *     alpha_i = min(0.99, o_i exp(-q/2)) (eq. 1 in 2-D), q = d^T Sigma'^-1 d,
 *     Gaussians with q > 9 or outside their box are ignored, alpha < 1/255 is
 *     skipped, and a pixel stops before the Gaussian that would take its
 *     transmittance below 1e-4;
 *   - the backward pass returns the derivative of that forward with respect to
 *     every Gaussian parameter (the paper trains them all with Adam).
 *
 * Conventions
 *   - pixel (i, j) samples (i + 0.5, j + 0.5); u = fx (tx / tz) + cx.
 *   - world_to_cam is a row-major 3x4 [R | t]; camera looks along +z.
 *   - quaternions are (w, x, y, z), any non-zero norm (normalised inside).
 *   - scales are linear (already exponentiated); opacity is in (0, 1).
 *   - SH: real orthonormal basis without the Condon-Shortley phase, degree
 *     0..3, coefficient index l^2 + l + m, layout [n][(L+1)^2][3];
 *     colour = max(0, sum_k sh_k Y_k(dir) + 0.5), dir = normalise(mu - campos).
 *   - images are planar float32: rgb [3][H][W], feat [D][H][W],
 *     depth [H][W] (sum of the weights times each Gaussian's view-space depth
 *     tz; background 0), final_T [H][W], n_contrib [H][W] (1 + list position
 *     of the last blended Gaussian in the pixel's tile list).
 *   - BF16 storage is accepted for sh and feat only (round-to-nearest-even
 *     bfloat16, passed as uint16 bit patterns).  Blending, transmittance and
 *     every accumulation are float32; the matrix-core contractions use exact
 *     bf16 parts in the forward and two-part splits (about 16 significant
 *     bits per product) in the backward; the forward projection geometry is
 *     float64 (it decides keys and boxes), its backward float32; every
 *     gradient is float32.
 *
 * Ownership and asynchrony
 *   - every pointer in the structs below is DEVICE memory owned by the caller;
 *     the library never allocates device memory in these calls and keeps no
 *     global mutable state.  Calls only enqueue work on `stream` (a
 *     hipStream_t, NULL = default stream) and return; results are ready when
 *     the stream is.  Distinct state buffers may be used concurrently.
 *   - argument errors are detected on the host before anything is enqueued
 *     and returned synchronously; conditions only the device can see (sort
 *     key overflow, non-finite inputs) are recorded in the state's report and
 *     read with fe_read_report().  No C++ exception crosses the ABI.
 */
#ifndef FE4DGS_RAST_H
#define FE4DGS_RAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FE4DGS_ABI_VERSION 6

typedef enum fe_status {
  FE_OK = 0,
  FE_ERR_INVALID_ARG = 1,        /* NULL pointer, bad size, bad enum value      */
  FE_ERR_UNSUPPORTED = 2,        /* feat_dim > 256, sh_degree > 3, W/H > 32767,
                                    n > 2^23 Gaussians, tile shapes other than
                                    8/16/32 wide with 64/128/256 pixels        */
  FE_ERR_WORKSPACE_TOO_SMALL = 3,/* state / scratch / workspace below *_bytes() */
  FE_ERR_KEY_OVERFLOW = 4,       /* device: more (tile, Gaussian) keys than
                                    key_capacity; outputs are invalid and
                                    report.keys_needed holds the count needed  */
  FE_ERR_HIP = 5,                /* a HIP runtime call failed                  */
  FE_ERR_ROW_OVERFLOW = 6        /* device: the backward needed more partial
                                    rows than row_capacity; gradients are
                                    invalid and report.rows_needed holds the
                                    count needed                               */
} fe_status;

typedef enum fe_dtype { FE_F32 = 0, FE_BF16 = 1 } fe_dtype;

/* Pinhole camera (identity pose in every workload of the paper's data). */
typedef struct fe_camera {
  int32_t width, height;         /* pixels, 1..32767                           */
  float fx, fy, cx, cy;          /* focal lengths and principal point, pixels  */
  float world_to_cam[12];        /* row-major 3x4 [R | t]                       */
  float near_plane;              /* cull when tz <= near_plane (0.2 typical)   */
} fe_camera;

/* Rasterizer configuration. */
typedef struct fe_config {
  int32_t tile_w, tile_h;        /* tile shape in pixels; tile_w * tile_h must
                                    be 64, 128 or 256 and tile_w one of
                                    8, 16, 32                                  */
  int32_t threads_per_tile;      /* threads of the compositing workgroup of a
                                    tile: tile_w * tile_h (one per pixel:
                                    every wave walks its pixels and runs the
                                    contractions), 2 * tile_w * tile_h (two
                                    per pixel: walker waves beside matrix-core
                                    waves; matrix-core variant, BF16 features,
                                    feat_dim <= 128), or
                                    0 = the two-per-pixel kernels wherever
                                    they exist; other values are
                                    FE_ERR_UNSUPPORTED                         */
  int32_t sh_degree;             /* 0..3                                        */
  int32_t feat_dim;              /* D, 1..256                                   */
  int32_t sh_dtype, feat_dtype;  /* fe_dtype                                    */
  float bg_rgb[3];               /* colour background (feature background is 0)*/
  float cov2d_dilation;          /* added to Sigma'_xx and Sigma'_yy (0.3)      */
  float jacobian_clamp;          /* J evaluated at tx/tz clamped to
                                    +-k W / (2 fx) (1.3); 0 disables            */
  int64_t key_capacity;          /* maximum number of (tile, Gaussian) keys    */
  int64_t row_capacity;          /* backward partial rows (matrix-core variant);
                                    0 = key_capacity (always sufficient)       */
  uint32_t flags;                /* FE_FLAG_*                                   */
  int32_t variant;               /* compositing kernel variant (FE_VARIANT_*)  */
  void* const* stage_events;     /* optional timing: NULL, or an array of
                                    2 * FE_STAGE_COUNT hipEvent_t (entries may be
                                    NULL); events[2s] / events[2s+1] are recorded
                                    on the call's stream before / after stage s */
} fe_config;

/* Stages recorded by fe_config.stage_events. */
#define FE_STAGE_PROJECT 0          /* projection forward                         */
#define FE_STAGE_SORT 1             /* tile binning and per-tile depth sort       */
#define FE_STAGE_COMPOSITE 2        /* per-tile blending forward                  */
#define FE_STAGE_COMPOSITE_BWD 3    /* per-tile blending backward                 */
#define FE_STAGE_REDUCE 4           /* per-Gaussian reduction of tile partials    */
#define FE_STAGE_PROJECT_BWD 5      /* projection backward                        */
#define FE_STAGE_COUNT 6

#define FE_FLAG_NO_ZERO_GRADS 0x1u  /* backward accumulates into *out instead of
                                       overwriting it                           */
#define FE_FLAG_BATCH_PER_FRAME 0x2u  /* batch plans: every frame runs its own
                                       compositing kernels (frames on parallel
                                       graph branches) instead of the
                                       persistent multi-frame launches          */

#define FE_VARIANT_AUTO 0           /* library default                          */
#define FE_VARIANT_VALU 1           /* vector-ALU blending in both directions   */
#define FE_VARIANT_MFMA 2           /* D-channel contractions on the matrix cores
                                       (bf16 parts, exact float32 products)     */

/* Packed Gaussian arrays (device, SoA, contiguous).  `sh` must be 16-byte
 * aligned (rows are read with 16-byte loads); the other arrays need their
 * element alignment.  Misaligned pointers give FE_ERR_INVALID_ARG. */
typedef struct fe_gaussians {
  int64_t n;
  const float* means;            /* [n][3]                                      */
  const float* scales;           /* [n][3] linear                               */
  const float* quats;            /* [n][4] (w, x, y, z)                          */
  const float* opacity;          /* [n]                                          */
  const void* sh;                /* [n][(L+1)^2][3] float or bf16 bits          */
  const void* feat;              /* [n][D] float or bf16 bits                   */
} fe_gaussians;

/* Forward outputs (device). */
typedef struct fe_images {
  float* rgb;                    /* [3][H][W]                                   */
  float* feat;                   /* [D][H][W]                                   */
  float* final_T;                /* [H][W]                                      */
  int32_t* n_contrib;            /* [H][W]                                      */
  float* depth;                  /* [H][W], or NULL (not written)               */
} fe_images;

/* Backward outputs (device, float32; overwritten unless FE_FLAG_NO_ZERO_GRADS). */
typedef struct fe_grads {
  float* means;                  /* [n][3]                                      */
  float* scales;                 /* [n][3]                                      */
  float* quats;                  /* [n][4]                                      */
  float* opacity;                /* [n]                                          */
  float* sh;                     /* [n][(L+1)^2][3]                              */
  float* feat;                   /* [n][D]                                      */
  float* means2d;                /* optional [n][2] dL/d(u, v); may be NULL     */
} fe_grads;

/* Device-side report, read back with fe_read_report(). */
typedef struct fe_report {
  int32_t status;                /* the forward's status (FE_OK or
                                    FE_ERR_KEY_OVERFLOW) if it is not FE_OK,
                                    else backward_status                       */
  int32_t backward_status;       /* the last backward of this state: FE_OK or
                                    FE_ERR_ROW_OVERFLOW (cleared when a
                                    backward starts, and by a new forward)     */
  int64_t keys_needed;           /* number of (tile, Gaussian) keys the frame has */
  int64_t n_visible;             /* Gaussians that emitted at least one key     */
  int64_t n_culled_nonfinite;    /* Gaussians culled for non-finite parameters  */
  int64_t rows_needed;           /* sum over tiles of the longest pixel walk
                                    (matrix-core variant; sizes the backward)   */
} fe_report;

/* Byte offsets of the regions of a forward state buffer (for tests and
 * tools; every offset is 256-byte aligned).  The sorted array holds
 * report.keys_needed valid entries (at most key_capacity): the lists of the
 * tiles one after another, tile t at [ranges[t].x, ranges[t].y), each in
 * ascending (float32 depth bits, Gaussian index) order. */
typedef struct fe_state_layout {
  size_t total;
  size_t xy;                     /* float2 [n]    pixel position (u, v)         */
  size_t conic_opacity;          /* float4 [n]    conic (A, B, C), opacity      */
  size_t rgb;                    /* float4 [n]    colour and view-space depth
                                                  (r, g, b, tz)                 */
  size_t box;                    /* int16x4 [n]   pixel box (i0, j0, i1, j1)    */
  size_t depth_key;              /* uint32 [n]    float32 depth bits of each
                                                  Gaussian (culled: 0xFFFFFFFF) */
  size_t tile_count;             /* uint32 [n]    tiles touched                 */
  size_t sorted_gauss;           /* uint32 [cap]  Gaussian index of each key    */
  size_t ranges;                 /* uint32x2 [tiles] [start, end) per tile      */
  size_t report;                 /* device report words                         */
} fe_state_layout;

int         fe_abi_version(void);
const char* fe_status_string(fe_status s);

/* Validate a configuration and camera (host only, no GPU needed). */
fe_status fe_validate(const fe_config* cfg, const fe_camera* cam, int64_t n);

/* Size and layout of the forward state for n Gaussians (host only).
 * Returns 0 (and fills nothing) when the arguments are invalid. */
size_t    fe_state_bytes(const fe_config* cfg, const fe_camera* cam, int64_t n);
fe_status fe_state_layout_get(const fe_config* cfg, const fe_camera* cam, int64_t n,
                              fe_state_layout* out);

/* Scratch needed by fe_render_backward (host only).  With the matrix-core
 * variant it holds one partial-gradient row of round_up(D + 9, 32) floats
 * (whole 128-byte lines) for each (tile, list position) the backward walks;
 * the forward's report.rows_needed gives the exact count for a frame, and
 * row_capacity bounds it. */
size_t    fe_backward_scratch_bytes(const fe_config* cfg, const fe_camera* cam, int64_t n);

/* Forward render of one camera.  `state` (device, 256-byte aligned,
 * state_bytes >= fe_state_bytes) receives the projected record, the sorted key
 * lists and the report, and must be passed unchanged to fe_render_backward.
 * A misaligned state returns FE_ERR_INVALID_ARG. */
fe_status fe_render_forward(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                            const fe_images* out, void* state, size_t state_bytes, void* stream);

/* Backward of fe_render_forward for upstream gradients d_rgb [3][H][W],
 * d_feat [D][H][W] and d_depth [H][W] (device float32; d_depth may be NULL for
 * no depth gradient; none flows into final_T / n_contrib).
 * `fwd` must be the images that forward wrote (final_T and n_contrib are
 * read).  `scratch` (device, 256-byte aligned, >= fe_backward_scratch_bytes)
 * holds per-Gaussian screen-space gradients; a misaligned scratch returns
 * FE_ERR_INVALID_ARG. */
fe_status fe_render_backward(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                             const fe_images* fwd, const void* state, size_t state_bytes,
                             const float* d_rgb, const float* d_feat, const float* d_depth,
                             const fe_grads* out, void* scratch, size_t scratch_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fe_render_backward with its scratch in a library-held device array of
 * FE_NOALLOC_SCRATCH_BYTES per GPU (allocated when the library's device code
 * is loaded on that GPU, held until the process ends).  Same arguments and
 * results as fe_render_backward without scratch / scratch_bytes; the device
 * is the current one (the stream must belong to it).  Returns
 * FE_ERR_WORKSPACE_TOO_SMALL, before enqueuing anything, when
 * fe_backward_scratch_bytes() exceeds FE_NOALLOC_SCRATCH_BYTES: set
 * row_capacity to the forward's report.rows_needed (or a bound of it) rather
 * than leaving it at key_capacity.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race;
 * calls in order on one stream do not.  Calls no allocating routine. */
#define FE_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
fe_status fe_render_backward_noalloc(const fe_config* cfg, const fe_camera* cam, const fe_gaussians* g,
                                     const fe_images* fwd, const void* state, size_t state_bytes,
                                     const float* d_rgb, const float* d_feat, const float* d_depth,
                                     const fe_grads* out, void* stream);

/* ------------------------------------------------------------------------
 * Semantic decoder and feature loss (Sec. 3.3, eq. 10), fused: the rendered
 * feature map z [in_dim][pixels] (planar float32, as fe_render_forward writes
 * it) goes through the pointwise convolution z' = W z + b (W [256][in_dim]
 * row-major, b [256]) and is compared with the target map t [256][pixels] by
 * L = (1 / pixels) sum_x |z'(x) - t(x)|_1 (the target at the render
 * resolution).  One call returns L and its gradients, with
 * s = sign(z' - t) (sign(0) = 0): d_feat = W^T s / pixels (ready to be the
 * backward's d_feat), d_weight = s z^T / pixels, d_bias = sum_x s / pixels;
 * `decoded` (optional) receives z'.  Products are taken from bf16 parts of
 * the float32 operands (about 16 significant bits per product), sums in
 * float32.  in_dim is 32, 64 or 128 (else FE_ERR_UNSUPPORTED); target_dtype
 * FE_F32 or FE_BF16; 1 <= pixels <= 2^24; weight 16-byte aligned (else
 * FE_ERR_INVALID_ARG).  All pointers are device memory; d_feat and decoded may
 * be NULL; no output may overlap an input.  Launches asynchronously on
 * `stream`; results are ready when the stream reaches the end of the call.  The workspace (256-byte aligned, >= fe_decoder_workspace_bytes;
 * 0 for unsupported sizes) holds one partial gradient per workgroup and the
 * residual signs (2 bits per output value).
 * ---------------------------------------------------------------------- */
typedef struct fe_decoder {
  int32_t in_dim;                /* D of the feature map                        */
  int32_t target_dtype;          /* fe_dtype of `target`                        */
  int64_t pixels;                /* H * W >= 1                                  */
  const float* feat;             /* [in_dim][pixels]                            */
  const float* weight;           /* [256][in_dim]                               */
  const float* bias;             /* [256]                                       */
  const void* target;            /* [256][pixels]                               */
  float* loss;                   /* [1]                                         */
  float* d_feat;                 /* [in_dim][pixels] or NULL                    */
  float* d_weight;               /* [256][in_dim]                               */
  float* d_bias;                 /* [256]                                       */
  float* decoded;                /* [256][pixels] or NULL                       */
} fe_decoder;

size_t    fe_decoder_workspace_bytes(int32_t in_dim, int64_t pixels);
fe_status fe_decoder_l1(const fe_decoder* d, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * FST deformation module (Sec. 3.2, eqs. 4-6; appendix "FST Deformation
 * Module"): G_t from the canonical Gaussians at time t, as the rasterizer's
 * input.  Per Gaussian:
 *   f  = HexPlane(mu, t): the coordinates (x, y, z, t) are mapped to [-1, 1]
 *        (space by the box [lo, hi], time by 2t - 1) and clamped; for each of
 *        the four levels the six coordinate-pair planes (x,y), (x,z), (x,t),
 *        (y,z), (y,t), (z,t) are sampled bilinearly (grid end points on -1
 *        and 1) and multiplied channel by channel; the levels' products are
 *        concatenated (f has 4C entries);
 *   h  = F_out(f): eight affine layers of width W, ReLU between them;
 *   h_g = B2(relu(B1(relu(h)))) (W -> W -> W/2) and
 *   dg = H(relu(h_g)) (W/2 -> d_g) for g = mu, rot, scale, opacity
 *        (d = 3, 4, 3, 1);
 *   dz = E2(relu(E1([h_mu | h_rot | h_scale | h_opacity]))) (2W -> W -> N);
 *   G_t = (mu + dmu, q + dq, exp(log s + ds), sigmoid(logit o + do), z + dz).
 * Grid points of coordinate k at level l: base_res[k] * level_mult[l] for
 * space, base_res[3] for time.  HexPlane arithmetic in float32 (coordinates
 * and interpolation weights in float64); the affine layers on the matrix
 * cores from two-part bf16 splits of activations and weights (products of
 * order <= 1, about 16 significant bits) with float32 accumulation.
 * Supported: channels 32 or 64, width 64, feat_dim a multiple of 16 up to
 * 256 (else FE_ERR_UNSUPPORTED).
 * ---------------------------------------------------------------------- */
typedef struct fe_deform_net {
  int32_t channels;              /* C, channels of every HexPlane plane         */
  int32_t width;                 /* W of F_out                                  */
  int32_t feat_dim;              /* N, channels of the semantic update          */
  int32_t base_res[4];           /* grid points of x, y, z, t at multiplier 1   */
  int32_t level_mult[4];         /* spatial multipliers of the four levels      */
  float lo[3];                   /* box of the spatial coordinates              */
  float hi[3];                   /* (hi > lo on every axis)                     */
  const float* planes;           /* device, fe_deform_plane_floats() floats:
                                    level by level, pairs in the order above,
                                    each plane [res_b][res_a][C]               */
  const float* weights;          /* device, fe_deform_weight_floats() floats:
                                    layers F_out 1..8, then per branch g (mu,
                                    rot, scale, opacity) B1, B2, H, then E1, E2;
                                    each layer weight [out][in] row-major, then
                                    bias [out]                                 */
} fe_deform_net;

typedef struct fe_deform_io {
  int64_t n;                     /* Gaussians, >= 0                             */
  float t;                       /* time in [0, 1] (clamped)                    */
  int32_t out_feat_dtype;        /* fe_dtype of out_feat                        */
  const float* means;            /* [n][3]                                      */
  const float* quats;            /* [n][4] (w, x, y, z)                         */
  const float* log_scales;       /* [n][3]                                      */
  const float* logit_opacity;    /* [n]                                         */
  const float* feat;             /* [n][N] float32                              */
  float* out_means;              /* [n][3]                                      */
  float* out_quats;              /* [n][4], not normalised                      */
  float* out_scales;             /* [n][3], linear                              */
  float* out_opacity;            /* [n], in (0, 1)                              */
  void* out_feat;                /* [n][N] of out_feat_dtype                    */
} fe_deform_io;

/* Sizes of the flat parameter arrays (host only; 0 if unsupported). */
size_t fe_deform_plane_floats(const fe_deform_net* net);
size_t fe_deform_weight_floats(const fe_deform_net* net);
/* Workspace of fe_deform_forward: the weights split into bf16 parts. */
size_t fe_deform_workspace_bytes(const fe_deform_net* net);

/* G_t for io->n Gaussians at time io->t.  All arrays are device memory; the
 * workspace (256-byte aligned) is overwritten; outputs must not overlap
 * inputs.  Enqueued on `stream`. */
fe_status fe_deform_forward(const fe_deform_net* net, const fe_deform_io* io, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Copy the device report of `state` to the host.  Synchronises `stream`.
 * Returns report->status as the call's status (FE_ERR_KEY_OVERFLOW when the
 * frame needed more keys than key_capacity, FE_ERR_ROW_OVERFLOW when a
 * backward of this state needed more rows than row_capacity; a backward may
 * write this status into the state's report). */
fe_status fe_read_report(const void* state, size_t state_bytes, fe_report* out, void* stream);

/* ------------------------------------------------------------------------
 * Batched frames (many timestamps / views, uneven Gaussian counts) replayed
 * as one captured HIP graph.  The plan binds every buffer at creation; the
 * caller rewrites the Gaussian arrays / upstream gradients in place between
 * launches.  Frames are independent renders that share nothing but the
 * stream; per-frame results equal fe_render_forward / fe_render_backward on
 * that frame alone.
 *
 * With BF16 features, feat_dim <= 128, the matrix-core variant and frames of
 * one image size, the compositing of all frames runs as one persistent launch
 * per direction: after the per-frame projection and sorting, one workgroup
 * orders every (frame, tile) item longest first (list length forward, walk
 * length backward; empty walks are left out) and the persistent workgroups,
 * one or more per compute unit, take items from that queue until it is empty.
 * Otherwise each frame runs its own kernels inside the graph.  The workspace
 * then also holds the queues and one argument record per frame (written by
 * the first fe_batch_launch, before it captures).
 * ---------------------------------------------------------------------- */
typedef struct fe_batch_plan fe_batch_plan;

#define FE_MODE_FORWARD 1
#define FE_MODE_BACKWARD 2
#define FE_MODE_FORWARD_BACKWARD 3

/* Workspace for `frames` frames with n[f] Gaussians each (host only). */
size_t fe_batch_workspace_bytes(const fe_config* cfg, const fe_camera* cams, int32_t frames,
                                const int64_t* n);

/* Create a plan.  Arrays of length `frames`: cams, g, out, d_rgb, d_feat,
 * d_depth, grads (d_rgb / d_feat / grads may be NULL for FE_MODE_FORWARD;
 * d_depth, or any of its entries, may be NULL for no depth gradient; the gradient
 * pointers of a frame with n == 0 may be NULL).  Returns FE_ERR_HIP when the
 * device cannot be queried for the persistent launch size.  The plan
 * owns host memory and HIP graph handles only; `workspace` (256-byte
 * aligned, else FE_ERR_INVALID_ARG) stays the caller's.  The first
 * fe_batch_launch captures the graph. */
fe_status fe_batch_plan_create(const fe_config* cfg, const fe_camera* cams, int32_t frames,
                               const fe_gaussians* g, const fe_images* out,
                               const float* const* d_rgb, const float* const* d_feat,
                               const float* const* d_depth, const fe_grads* grads, int32_t mode, void* workspace,
                               size_t workspace_bytes, fe_batch_plan** plan);

/* Enqueue one replay of every frame on `stream` (capturing on first use). */
fe_status fe_batch_launch(fe_batch_plan* plan, void* stream);

/* Report of frame f (synchronises `stream`). */
fe_status fe_batch_read_report(fe_batch_plan* plan, int32_t f, fe_report* out, void* stream);

void fe_batch_plan_destroy(fe_batch_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* FE4DGS_RAST_H */
