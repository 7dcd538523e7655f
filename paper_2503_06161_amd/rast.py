"""Python binding of libfe4dgs_rast.so.

Argument marshalling only: every step of the rasterizer runs in the HIP
library; PyTorch provides device memory and the stream.  The library must be
built (``python -m paper_2503_06161_amd.build``); importing this module
without it raises, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe4dgs_rast.so")

(FE_OK, FE_ERR_INVALID_ARG, FE_ERR_UNSUPPORTED, FE_ERR_WORKSPACE_TOO_SMALL, FE_ERR_KEY_OVERFLOW, FE_ERR_HIP,
 FE_ERR_ROW_OVERFLOW) = range(7)
FE_F32, FE_BF16 = 0, 1
FE_FLAG_NO_ZERO_GRADS = 1
FE_FLAG_BATCH_PER_FRAME = 2
FE_VARIANT_AUTO, FE_VARIANT_VALU, FE_VARIANT_MFMA = 0, 1, 2
FE_MODE_FORWARD, FE_MODE_BACKWARD, FE_MODE_FORWARD_BACKWARD = 1, 2, 3
STAGES = ("project", "sort", "composite", "composite_bwd", "reduce", "project_bwd")


class RasterError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_status_string(status)} ({status})")


class fe_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("world_to_cam", C.c_float * 12),
                ("near_plane", C.c_float)]


class fe_config(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("threads_per_tile", C.c_int32),
                ("sh_degree", C.c_int32), ("feat_dim", C.c_int32), ("sh_dtype", C.c_int32),
                ("feat_dtype", C.c_int32), ("bg_rgb", C.c_float * 3), ("cov2d_dilation", C.c_float),
                ("jacobian_clamp", C.c_float), ("key_capacity", C.c_int64), ("row_capacity", C.c_int64),
                ("flags", C.c_uint32),
                ("variant", C.c_int32), ("stage_events", C.c_void_p)]


class fe_gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("feat", C.c_void_p)]


class fe_images(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("feat", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("depth", C.c_void_p)]


class fe_grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p), ("opacity", C.c_void_p),
                ("sh", C.c_void_p), ("feat", C.c_void_p), ("means2d", C.c_void_p)]


class fe_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("backward_status", C.c_int32), ("keys_needed", C.c_int64),
                ("n_visible", C.c_int64), ("n_culled_nonfinite", C.c_int64), ("rows_needed", C.c_int64)]


class fe_decoder(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("target_dtype", C.c_int32), ("pixels", C.c_int64), ("feat", C.c_void_p),
                ("weight", C.c_void_p), ("bias", C.c_void_p), ("target", C.c_void_p), ("loss", C.c_void_p),
                ("d_feat", C.c_void_p), ("d_weight", C.c_void_p), ("d_bias", C.c_void_p), ("decoded", C.c_void_p)]


class fe_deform_net(C.Structure):
    _fields_ = [("channels", C.c_int32), ("width", C.c_int32), ("feat_dim", C.c_int32),
                ("base_res", C.c_int32 * 4), ("level_mult", C.c_int32 * 4), ("lo", C.c_float * 3),
                ("hi", C.c_float * 3), ("planes", C.c_void_p), ("weights", C.c_void_p)]


class fe_deform_io(C.Structure):
    _fields_ = [("n", C.c_int64), ("t", C.c_float), ("out_feat_dtype", C.c_int32), ("means", C.c_void_p),
                ("quats", C.c_void_p), ("log_scales", C.c_void_p), ("logit_opacity", C.c_void_p),
                ("feat", C.c_void_p), ("out_means", C.c_void_p), ("out_quats", C.c_void_p),
                ("out_scales", C.c_void_p), ("out_opacity", C.c_void_p), ("out_feat", C.c_void_p)]


class fe_state_layout(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in ("total", "xy", "conic_opacity", "rgb", "box", "depth_key",
                                          "tile_count", "sorted_gauss", "ranges", "report")]


EXPORTS = {
    "fe_abi_version": (C.c_int, []),
    "fe_status_string": (C.c_char_p, [C.c_int]),
    "fe_validate": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int64]),
    "fe_state_bytes": (C.c_size_t, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int64]),
    "fe_state_layout_get": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int64,
                                      C.POINTER(fe_state_layout)]),
    "fe_backward_scratch_bytes": (C.c_size_t, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int64]),
    "fe_render_forward": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.POINTER(fe_gaussians),
                                    C.POINTER(fe_images), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fe_render_backward": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.POINTER(fe_gaussians),
                                     C.POINTER(fe_images), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.POINTER(fe_grads), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fe_render_backward_noalloc": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.POINTER(fe_gaussians),
                                             C.POINTER(fe_images), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.POINTER(fe_grads), C.c_void_p]),
    "fe_read_report": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(fe_report), C.c_void_p]),
    "fe_batch_workspace_bytes": (C.c_size_t, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int32,
                                              C.POINTER(C.c_int64)]),
    "fe_batch_plan_create": (C.c_int, [C.POINTER(fe_config), C.POINTER(fe_camera), C.c_int32,
                                       C.POINTER(fe_gaussians), C.POINTER(fe_images), C.POINTER(C.c_void_p),
                                       C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(fe_grads), C.c_int32,
                                       C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "fe_batch_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fe_batch_read_report": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(fe_report), C.c_void_p]),
    "fe_batch_plan_destroy": (None, [C.c_void_p]),
    "fe_decoder_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64]),
    "fe_decoder_l1": (C.c_int, [C.POINTER(fe_decoder), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fe_deform_plane_floats": (C.c_size_t, [C.POINTER(fe_deform_net)]),
    "fe_deform_weight_floats": (C.c_size_t, [C.POINTER(fe_deform_net)]),
    "fe_deform_workspace_bytes": (C.c_size_t, [C.POINTER(fe_deform_net)]),
    "fe_deform_forward": (C.c_int, [C.POINTER(fe_deform_net), C.POINTER(fe_deform_io), C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2503_06161_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.fe_abi_version() != 6:
        raise ImportError("libfe4dgs_rast.so ABI version mismatch")
    _lib = lib
    return lib


def _status_string(s: int) -> str:
    try:
        return load_library().fe_status_string(s).decode()
    except Exception:  # library not loadable: still report the number
        return "status"


# ---------------------------------------------------------------------------
@dataclass
class Settings:
    """Rasterizer settings (fe_config).  ``key_capacity=None`` sizes the sort
    buffers from the frame and grows them when a frame needs more."""
    sh_degree: int = 3
    feat_dim: int = 32
    tile_w: int = 16
    tile_h: int = 16
    sh_dtype: str = "f32"
    feat_dtype: str = "f32"
    bg: tuple = (0.0, 0.0, 0.0)
    dilation: float = 0.3
    jacobian_clamp: float = 1.3
    key_capacity: int | None = None
    row_capacity: int | None = None  # None: the forward's reported need (or key_capacity)
    variant: int = FE_VARIANT_AUTO
    threads_per_tile: int = 0       # 0: library choice; tile pixels or twice that (fe_config.threads_per_tile)
    flags: int = 0
    stage_events: object = None     # optional ctypes array of 2*len(STAGES) hipEvent_t handles

    def to_c(self, cap: int, rows: int = 0) -> fe_config:
        c = fe_config()
        c.tile_w, c.tile_h, c.threads_per_tile = self.tile_w, self.tile_h, self.threads_per_tile
        c.sh_degree, c.feat_dim = self.sh_degree, self.feat_dim
        c.sh_dtype = FE_BF16 if self.sh_dtype == "bf16" else FE_F32
        c.feat_dtype = FE_BF16 if self.feat_dtype == "bf16" else FE_F32
        for k in range(3):
            c.bg_rgb[k] = float(self.bg[k])
        c.cov2d_dilation = self.dilation
        c.jacobian_clamp = self.jacobian_clamp
        c.key_capacity = int(cap)
        c.row_capacity = int(rows)
        c.flags = self.flags
        c.variant = self.variant
        c.stage_events = C.cast(self.stage_events, C.c_void_p) if self.stage_events is not None else None
        return c


def camera_c(cam) -> fe_camera:
    c = fe_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w = np.asarray(cam.world_to_cam, np.float32).reshape(-1)
    for k in range(12):
        c.world_to_cam[k] = float(w[k])
    c.near_plane = float(getattr(cam, "near", 0.2))
    return c


def _stream_handle(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _check(status: int, what: str):
    if status != FE_OK:
        raise RasterError(status, what)


def _ptr(t: torch.Tensor | None):
    return None if t is None else t.data_ptr()


def _req(t: torch.Tensor, dtype, shape, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def default_capacity(n: int) -> int:
    return max(4096, 16 * n)


@dataclass
class ForwardResult:
    rgb: torch.Tensor
    feat: torch.Tensor
    final_T: torch.Tensor
    n_contrib: torch.Tensor
    state: torch.Tensor
    cfg: fe_config
    cam: fe_camera
    report: dict | None = None
    depth: torch.Tensor | None = None


def _gaussians_c(means, scales, quats, opacity, sh, feat, st: Settings):
    n = means.shape[0]
    K = (st.sh_degree + 1) ** 2
    shdt = torch.bfloat16 if st.sh_dtype == "bf16" else torch.float32
    fdt = torch.bfloat16 if st.feat_dtype == "bf16" else torch.float32
    _req(means, torch.float32, (n, 3), "means")
    _req(scales, torch.float32, (n, 3), "scales")
    _req(quats, torch.float32, (n, 4), "quats")
    _req(opacity, torch.float32, (n,), "opacity")
    _req(sh, shdt, (n, K, 3), "sh")
    _req(feat, fdt, (n, st.feat_dim), "feat")
    g = fe_gaussians()
    g.n = n
    g.means, g.scales, g.quats, g.opacity = _ptr(means), _ptr(scales), _ptr(quats), _ptr(opacity)
    g.sh, g.feat = _ptr(sh), _ptr(feat)
    return g


def read_report(state: torch.Tensor, stream=None) -> dict:
    lib = load_library()
    r = fe_report()
    lib.fe_read_report(C.c_void_p(state.data_ptr()), state.numel(), C.byref(r), C.c_void_p(_stream_handle(stream)))
    return dict(status=r.status, backward_status=r.backward_status, keys_needed=r.keys_needed,
                n_visible=r.n_visible, n_culled_nonfinite=r.n_culled_nonfinite, rows_needed=r.rows_needed)


def state_layout(cam, st: Settings, n: int, cap: int) -> dict:
    lib = load_library()
    lay = fe_state_layout()
    _check(lib.fe_state_layout_get(C.byref(st.to_c(cap)), C.byref(camera_c(cam)), n, C.byref(lay)),
           "fe_state_layout_get")
    return {k: getattr(lay, k) for k, _ in fe_state_layout._fields_}


def render_forward(means, scales, quats, opacity, sh, feat, cam, st: Settings, check: bool = True,
                   stream=None, state: torch.Tensor | None = None, out: dict | None = None) -> ForwardResult:
    """Forward render of one camera through fe_render_forward.  With
    ``check`` the report is read back (one stream synchronisation) and a
    key-capacity overflow either grows the buffers and re-renders (automatic
    capacity) or raises."""
    lib = load_library()
    n = means.shape[0]
    dev = means.device
    cam_c = camera_c(cam)
    cap = st.key_capacity if st.key_capacity is not None else default_capacity(n)
    H, W, D = cam_c.height, cam_c.width, st.feat_dim
    g = _gaussians_c(means, scales, quats, opacity, sh, feat, st)
    for _attempt in range(3):
        cfg = st.to_c(cap)
        sb = lib.fe_state_bytes(C.byref(cfg), C.byref(cam_c), n)
        if sb == 0:
            _check(lib.fe_validate(C.byref(cfg), C.byref(cam_c), n), "fe_validate")
        if state is None or state.numel() < sb:
            state = torch.empty(sb, dtype=torch.uint8, device=dev)
        if out is None:
            out = dict(rgb=torch.empty(3, H, W, device=dev), feat=torch.empty(D, H, W, device=dev),
                       final_T=torch.empty(H, W, device=dev),
                       n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev),
                       depth=torch.empty(H, W, device=dev))
        im = fe_images(_ptr(out["rgb"]), _ptr(out["feat"]), _ptr(out["final_T"]), _ptr(out["n_contrib"]),
                       _ptr(out.get("depth")))
        _check(lib.fe_render_forward(C.byref(cfg), C.byref(cam_c), C.byref(g), C.byref(im),
                                     C.c_void_p(state.data_ptr()), state.numel(),
                                     C.c_void_p(_stream_handle(stream))), "fe_render_forward")
        rep = None
        if check:
            rep = read_report(state, stream)
            if rep["status"] == FE_ERR_KEY_OVERFLOW:
                if st.key_capacity is None:
                    cap = int(rep["keys_needed"] * 1.25) + 1024
                    state = None
                    continue
                raise RasterError(FE_ERR_KEY_OVERFLOW, f"fe_render_forward needs {rep['keys_needed']} keys")
            _check(rep["status"], "fe_render_forward (device)")
        return ForwardResult(out["rgb"], out["feat"], out["final_T"], out["n_contrib"], state, cfg, cam_c, rep,
                             out.get("depth"))
    raise RasterError(FE_ERR_KEY_OVERFLOW, "fe_render_forward: capacity did not converge")


def render_backward(fwd: ForwardResult, means, scales, quats, opacity, sh, feat, d_rgb, d_feat,
                    st: Settings, stream=None, grads: dict | None = None, scratch: torch.Tensor | None = None,
                    want_means2d: bool = False, check: bool = True, d_depth=None) -> dict:
    """Gradients of <d_rgb, rgb> + <d_feat, feat> (+ <d_depth, depth>) for
    every input (float32).
    With ``check`` the report is read back (one stream synchronisation) and a
    backward that ran out of partial rows (a ``row_capacity`` below the
    frame's need) raises instead of returning invalid gradients."""
    lib = load_library()
    n = means.shape[0]
    dev = means.device
    K = (st.sh_degree + 1) ** 2
    H, W, D = fwd.cam.height, fwd.cam.width, st.feat_dim
    _req(d_rgb, torch.float32, (3, H, W), "d_rgb")
    _req(d_feat, torch.float32, (D, H, W), "d_feat")
    if d_depth is not None:
        _req(d_depth, torch.float32, (H, W), "d_depth")
    g = _gaussians_c(means, scales, quats, opacity, sh, feat, st)
    if grads is None:
        grads = dict(means=torch.empty(n, 3, device=dev), scales=torch.empty(n, 3, device=dev),
                     quats=torch.empty(n, 4, device=dev), opacity=torch.empty(n, device=dev),
                     sh=torch.empty(n, K, 3, device=dev), feat=torch.empty(n, D, device=dev))
        if want_means2d:
            grads["means2d"] = torch.empty(n, 2, device=dev)
    cfg = fe_config.from_buffer_copy(fwd.cfg)
    cfg.stage_events = C.cast(st.stage_events, C.c_void_p) if st.stage_events is not None else None
    if st.row_capacity is not None:
        cfg.row_capacity = int(st.row_capacity)
    elif fwd.report is not None:
        cfg.row_capacity = max(int(fwd.report["rows_needed"]), 1)
    sc_bytes = lib.fe_backward_scratch_bytes(C.byref(cfg), C.byref(fwd.cam), n)
    if scratch is None or scratch.numel() < sc_bytes:
        scratch = torch.empty(max(sc_bytes, 1), dtype=torch.uint8, device=dev)
    gr = fe_grads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]), _ptr(grads["opacity"]),
                  _ptr(grads["sh"]), _ptr(grads["feat"]), _ptr(grads.get("means2d")))
    im = fe_images(_ptr(fwd.rgb), _ptr(fwd.feat), _ptr(fwd.final_T), _ptr(fwd.n_contrib), _ptr(fwd.depth))
    _check(lib.fe_render_backward(C.byref(cfg), C.byref(fwd.cam), C.byref(g), C.byref(im),
                                  C.c_void_p(fwd.state.data_ptr()), fwd.state.numel(),
                                  C.c_void_p(d_rgb.data_ptr()), C.c_void_p(d_feat.data_ptr()),
                                  C.c_void_p(_ptr(d_depth)), C.byref(gr),
                                  C.c_void_p(scratch.data_ptr()), scratch.numel(),
                                  C.c_void_p(_stream_handle(stream))), "fe_render_backward")
    grads["_scratch"] = scratch
    if check:
        rep = read_report(fwd.state, stream)
        if rep["backward_status"] == FE_ERR_ROW_OVERFLOW:
            raise RasterError(FE_ERR_ROW_OVERFLOW, f"fe_render_backward needs {rep['rows_needed']} rows, "
                                                   f"row_capacity is {cfg.row_capacity}")
        _check(rep["status"], "fe_render_backward (device)")
    return grads


NOALLOC_SCRATCH_BYTES = 256 << 20    # FE_NOALLOC_SCRATCH_BYTES


def render_backward_noalloc(fwd: ForwardResult, means, scales, quats, opacity, sh, feat, d_rgb, d_feat,
                            st: Settings, grads: dict, stream=None, check: bool = True, d_depth=None) -> dict:
    """fe_render_backward_noalloc: the backward with its scratch in the
    library's per-GPU array (nothing is allocated; ``grads`` are the caller's
    float32 output buffers).  Raises FE_ERR_WORKSPACE_TOO_SMALL when the
    frame's scratch exceeds NOALLOC_SCRATCH_BYTES."""
    lib = load_library()
    H, W, D = fwd.cam.height, fwd.cam.width, st.feat_dim
    _req(d_rgb, torch.float32, (3, H, W), "d_rgb")
    _req(d_feat, torch.float32, (D, H, W), "d_feat")
    if d_depth is not None:
        _req(d_depth, torch.float32, (H, W), "d_depth")
    g = _gaussians_c(means, scales, quats, opacity, sh, feat, st)
    cfg = fe_config.from_buffer_copy(fwd.cfg)
    cfg.stage_events = None
    if st.row_capacity is not None:
        cfg.row_capacity = int(st.row_capacity)
    elif fwd.report is not None:
        cfg.row_capacity = max(int(fwd.report["rows_needed"]), 1)
    gr = fe_grads(_ptr(grads["means"]), _ptr(grads["scales"]), _ptr(grads["quats"]), _ptr(grads["opacity"]),
                  _ptr(grads["sh"]), _ptr(grads["feat"]), _ptr(grads.get("means2d")))
    im = fe_images(_ptr(fwd.rgb), _ptr(fwd.feat), _ptr(fwd.final_T), _ptr(fwd.n_contrib), _ptr(fwd.depth))
    _check(lib.fe_render_backward_noalloc(C.byref(cfg), C.byref(fwd.cam), C.byref(g), C.byref(im),
                                          C.c_void_p(fwd.state.data_ptr()), fwd.state.numel(),
                                          C.c_void_p(d_rgb.data_ptr()), C.c_void_p(d_feat.data_ptr()),
                                          C.c_void_p(_ptr(d_depth)), C.byref(gr),
                                          C.c_void_p(_stream_handle(stream))), "fe_render_backward_noalloc")
    if check:
        rep = read_report(fwd.state, stream)
        if rep["backward_status"] == FE_ERR_ROW_OVERFLOW:
            raise RasterError(FE_ERR_ROW_OVERFLOW, "fe_render_backward_noalloc: row capacity exceeded")
        _check(rep["status"], "fe_render_backward_noalloc (device)")
    return grads


class RasterizeFE(torch.autograd.Function):
    """Differentiable rasterization: (means, scales, quats, opacity, sh,
    feat) -> (rgb [3,H,W], feat [D,H,W], depth [H,W]).  final_T and n_contrib
    are returned as non-differentiable outputs."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, feat, cam, st: Settings):
        fwd = render_forward(means, scales, quats, opacity, sh, feat, cam, st)
        ctx.save_for_backward(means, scales, quats, opacity, sh, feat)
        ctx.fwd = fwd
        ctx.st = st
        ctx.mark_non_differentiable(fwd.final_T, fwd.n_contrib)
        return fwd.rgb, fwd.feat, fwd.depth, fwd.final_T, fwd.n_contrib

    @staticmethod
    def backward(ctx, g_rgb, g_feat, g_depth, _g_T, _g_n):
        means, scales, quats, opacity, sh, feat = ctx.saved_tensors
        fwd = ctx.fwd
        H, W = fwd.cam.height, fwd.cam.width
        if g_rgb is None:
            g_rgb = torch.zeros(3, H, W, device=means.device)
        if g_feat is None:
            g_feat = torch.zeros(ctx.st.feat_dim, H, W, device=means.device)
        gr = render_backward(fwd, means, scales, quats, opacity, sh, feat, g_rgb.contiguous().float(),
                             g_feat.contiguous().float(), ctx.st,
                             d_depth=None if g_depth is None else g_depth.contiguous().float())
        ctx.fp32_grads = gr   # the float32 buffers, before any dtype cast
        return (gr["means"], gr["scales"], gr["quats"], gr["opacity"], gr["sh"].to(sh.dtype),
                gr["feat"].to(feat.dtype), None, None)


def rasterize(means, scales, quats, opacity, sh, feat, cam, st: Settings):
    """Differentiable render; returns (rgb, feat, depth, final_T, n_contrib)."""
    return RasterizeFE.apply(means, scales, quats, opacity, sh, feat, cam, st)


# ---------------------------------------------------------------------------
# Semantic decoder + L1 feature loss (Sec. 3.3, eq. 10)

DECODER_CHANNELS = 256


def decoder_workspace_bytes(in_dim: int, pixels: int) -> int:
    return int(load_library().fe_decoder_workspace_bytes(int(in_dim), int(pixels)))


def decoder_l1(feat, weight, bias, target, d_feat: bool = True, decoded: bool = False, workspace=None,
               stream=None) -> dict:
    """fe_decoder_l1: feat [D,H,W] float32, weight [256,D] float32, bias
    [256] float32, target [256,H,W] float32 or bfloat16 (all on the GPU).
    Returns loss [1] and d_weight [256,D], d_bias [256], plus d_feat [D,H,W]
    and decoded [256,H,W] when asked for (float32 tensors)."""
    lib = load_library()
    if feat.dim() != 3:
        raise ValueError("feat must be [D, H, W]")
    D, H, W = feat.shape
    _req(feat, torch.float32, (D, H, W), "feat")
    _req(weight, torch.float32, (DECODER_CHANNELS, D), "weight")
    _req(bias, torch.float32, (DECODER_CHANNELS,), "bias")
    if target.dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("target must be float32 or bfloat16")
    _req(target, target.dtype, (DECODER_CHANNELS, H, W), "target")
    dev = feat.device
    out = dict(loss=torch.empty(1, device=dev), d_weight=torch.empty(DECODER_CHANNELS, D, device=dev),
               d_bias=torch.empty(DECODER_CHANNELS, device=dev))
    if d_feat:
        out["d_feat"] = torch.empty(D, H, W, device=dev)
    if decoded:
        out["decoded"] = torch.empty(DECODER_CHANNELS, H, W, device=dev)
    need = decoder_workspace_bytes(D, H * W)
    if need == 0:
        raise RasterError(FE_ERR_UNSUPPORTED, "fe_decoder_workspace_bytes")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    d = fe_decoder(D, FE_BF16 if target.dtype == torch.bfloat16 else FE_F32, H * W, feat.data_ptr(),
                   weight.data_ptr(), bias.data_ptr(), target.data_ptr(), out["loss"].data_ptr(),
                   _ptr(out.get("d_feat")), out["d_weight"].data_ptr(), out["d_bias"].data_ptr(),
                   _ptr(out.get("decoded")))
    _check(lib.fe_decoder_l1(C.byref(d), C.c_void_p(workspace.data_ptr()), workspace.numel(),
                             C.c_void_p(_stream_handle(stream))), "fe_decoder_l1")
    return out


class DecoderL1(torch.autograd.Function):
    """L_feat(feat, weight, bias; target) as a differentiable scalar: the
    fused call computes the loss and its gradients together; backward scales
    them by the incoming gradient."""

    @staticmethod
    def forward(ctx, feat, weight, bias, target):
        r = decoder_l1(feat.contiguous().float(), weight.contiguous().float(), bias.contiguous().float(),
                       target.contiguous())
        ctx.save_for_backward(r["d_feat"], r["d_weight"], r["d_bias"])
        ctx.dtypes = (feat.dtype, weight.dtype, bias.dtype)
        return r["loss"][0]

    @staticmethod
    def backward(ctx, g):
        df, dw, db = ctx.saved_tensors
        return (df * g).to(ctx.dtypes[0]), (dw * g).to(ctx.dtypes[1]), (db * g).to(ctx.dtypes[2]), None


def decoder_loss(feat, weight, bias, target):
    """Differentiable L_feat of a rendered feature map (eq. 10)."""
    return DecoderL1.apply(feat, weight, bias, target)


# ---------------------------------------------------------------------------
# FST deformation module (Sec. 3.2, eqs. 4-6)

DEFORM_BRANCHES = ("mu", "rot", "scale", "opacity")


class DeformNet:
    """Device copy of the deformation parameters in the library's flat
    layout: ``planes[l][p]`` ([res_b, res_a, C] arrays, levels and
    coordinate pairs in the header's order) and ``layers`` (weight [out, in],
    bias [out] pairs under 'out', 'branch_<g>', 'head_<g>', 'sem')."""

    def __init__(self, planes, layers, lo, hi, channels, width, feat_dim, base_res=(64, 64, 64, 100),
                 levels=(1, 2, 4, 8), device="cuda"):
        lib = load_library()
        self.net = fe_deform_net()
        self.net.channels, self.net.width, self.net.feat_dim = int(channels), int(width), int(feat_dim)
        self.net.base_res[:] = [int(r) for r in base_res]
        self.net.level_mult[:] = [int(m) for m in levels]
        self.net.lo[:] = [float(v) for v in lo]
        self.net.hi[:] = [float(v) for v in hi]
        n_planes = lib.fe_deform_plane_floats(C.byref(self.net))
        n_weights = lib.fe_deform_weight_floats(C.byref(self.net))
        if n_planes == 0 or n_weights == 0:
            raise RasterError(FE_ERR_UNSUPPORTED, "fe_deform_net")
        flat = [np.ascontiguousarray(p, dtype=np.float32).ravel() for lvl in planes for p in lvl]
        order = list(layers["out"])
        for g in DEFORM_BRANCHES:
            order += list(layers["branch_" + g]) + [layers["head_" + g]]
        order += list(layers["sem"])
        wflat = [np.ascontiguousarray(a, dtype=np.float32).ravel() for w, b in order for a in (w, b)]
        pf, wf = np.concatenate(flat), np.concatenate(wflat)
        if pf.size != n_planes or wf.size != n_weights:
            raise ValueError(f"parameter sizes {pf.size}/{wf.size} do not match the layout {n_planes}/{n_weights}")
        self.planes = torch.from_numpy(pf).to(device)
        self.weights = torch.from_numpy(wf).to(device)
        self.net.planes, self.net.weights = self.planes.data_ptr(), self.weights.data_ptr()
        self.workspace = torch.empty(lib.fe_deform_workspace_bytes(C.byref(self.net)), dtype=torch.uint8,
                                     device=device)
        self.feat_dim = int(feat_dim)


def deform_forward(net: DeformNet, means, quats, log_scales, logit_opacity, feat, t: float, out_feat_dtype="f32",
                   out=None, stream=None) -> dict:
    """fe_deform_forward: G_t (means, quats, scales, opacity, feat) of n
    canonical Gaussians at time t.  Inputs are float32 CUDA tensors; feat is
    [n, N].  ``out`` may hold preallocated output tensors."""
    lib = load_library()
    n = means.shape[0]
    N = net.feat_dim
    _req(means, torch.float32, (n, 3), "means")
    _req(quats, torch.float32, (n, 4), "quats")
    _req(log_scales, torch.float32, (n, 3), "log_scales")
    _req(logit_opacity, torch.float32, (n,), "logit_opacity")
    _req(feat, torch.float32, (n, N), "feat")
    dev = means.device
    fdt = torch.bfloat16 if out_feat_dtype == "bf16" else torch.float32
    if out is None:
        out = dict(means=torch.empty(n, 3, device=dev), quats=torch.empty(n, 4, device=dev),
                   scales=torch.empty(n, 3, device=dev), opacity=torch.empty(n, device=dev),
                   feat=torch.empty(n, N, dtype=fdt, device=dev))
    io = fe_deform_io(n, float(t), FE_BF16 if fdt == torch.bfloat16 else FE_F32, means.data_ptr(), quats.data_ptr(),
                      log_scales.data_ptr(), logit_opacity.data_ptr(), feat.data_ptr(), out["means"].data_ptr(),
                      out["quats"].data_ptr(), out["scales"].data_ptr(), out["opacity"].data_ptr(),
                      out["feat"].data_ptr())
    _check(lib.fe_deform_forward(C.byref(net.net), C.byref(io), C.c_void_p(net.workspace.data_ptr()),
                                 net.workspace.numel(), C.c_void_p(_stream_handle(stream))), "fe_deform_forward")
    return out
