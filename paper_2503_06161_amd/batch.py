"""Many frames (timestamps / views) with uneven Gaussian counts rendered as
one captured HIP graph through the fe_batch_* entry points.

The plan binds every buffer at creation; deforming a scene means writing the
new parameters into the same tensors and calling ``launch()`` again.
Argument marshalling only: the graph is built and replayed by the library.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import rast


class BatchRenderer:
    """frames: list of dicts with device tensors means, scales, quats,
    opacity, sh, feat (one frame each); cams: list of cameras; d_rgb / d_feat
    (/ d_depth, optional): lists of upstream gradients (needed for the
    backward modes)."""

    def __init__(self, frames, cams, st: rast.Settings, mode=rast.FE_MODE_FORWARD_BACKWARD, d_rgb=None,
                 d_feat=None, capacity_margin=1.25, d_depth=None):
        lib = rast.load_library()
        self.lib = lib
        self.frames = frames
        self.cams = cams
        self.st = st
        self.mode = mode
        F = len(frames)
        dev = frames[0]["means"].device
        args = lambda f: (f["means"], f["scales"], f["quats"], f["opacity"], f["sh"], f["feat"])
        # size the sort keys and partial rows from one checked render of every frame
        keys, rows = 0, 0
        if st.key_capacity is None or st.row_capacity is None:
            for f, cam in zip(frames, cams):
                probe = rast.render_forward(*args(f), cam, rast.Settings(**{**st.__dict__, "stage_events": None}))
                keys = max(keys, probe.report["keys_needed"])
                rows = max(rows, probe.report["rows_needed"])
        cap = st.key_capacity if st.key_capacity is not None else int(keys * capacity_margin) + 1024
        rcap = st.row_capacity if st.row_capacity is not None else int(rows * capacity_margin) + 1024
        self.cfg = st.to_c(cap, rcap)
        self.cams_c = (rast.fe_camera * F)(*[rast.camera_c(c) for c in cams])
        self.g_c = (rast.fe_gaussians * F)(*[rast._gaussians_c(*args(f), st) for f in frames])
        self.out = []
        for cam in cams:
            H, W = int(cam.height), int(cam.width)
            self.out.append(dict(rgb=torch.empty(3, H, W, device=dev), feat=torch.empty(st.feat_dim, H, W, device=dev),
                                 final_T=torch.empty(H, W, device=dev),
                                 n_contrib=torch.empty(H, W, dtype=torch.int32, device=dev),
                                 depth=torch.empty(H, W, device=dev)))
        self.out_c = (rast.fe_images * F)(*[rast.fe_images(o["rgb"].data_ptr(), o["feat"].data_ptr(),
                                                            o["final_T"].data_ptr(), o["n_contrib"].data_ptr(),
                                                            o["depth"].data_ptr())
                                             for o in self.out])
        bwd = (mode & rast.FE_MODE_BACKWARD) != 0
        self.grads = []
        if bwd:
            K = (st.sh_degree + 1) ** 2
            for f in frames:
                n = f["means"].shape[0]
                self.grads.append(dict(means=torch.empty(n, 3, device=dev), scales=torch.empty(n, 3, device=dev),
                                       quats=torch.empty(n, 4, device=dev), opacity=torch.empty(n, device=dev),
                                       sh=torch.empty(n, K, 3, device=dev), feat=torch.empty(n, st.feat_dim, device=dev)))
            self.grads_c = (rast.fe_grads * F)(*[rast.fe_grads(*[g[k].data_ptr() for k in
                                                                 ("means", "scales", "quats", "opacity", "sh", "feat")],
                                                               None) for g in self.grads])
            self.d_rgb, self.d_feat = list(d_rgb), list(d_feat)
            self.d_depth = list(d_depth) if d_depth is not None else [None] * F
            self.drgb_c = (C.c_void_p * F)(*[t.data_ptr() for t in self.d_rgb])
            self.dfeat_c = (C.c_void_p * F)(*[t.data_ptr() for t in self.d_feat])
            self.ddepth_c = (C.c_void_p * F)(*[None if t is None else t.data_ptr() for t in self.d_depth])
        else:
            self.grads_c, self.drgb_c, self.dfeat_c, self.ddepth_c = None, None, None, None
        ns = (C.c_int64 * F)(*[f["means"].shape[0] for f in frames])
        wb = lib.fe_batch_workspace_bytes(C.byref(self.cfg), self.cams_c, F, ns)
        if wb == 0:
            raise rast.RasterError(rast.FE_ERR_INVALID_ARG, "fe_batch_workspace_bytes")
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=dev)
        plan = C.c_void_p()
        rast._check(lib.fe_batch_plan_create(C.byref(self.cfg), self.cams_c, F, self.g_c, self.out_c,
                                             self.drgb_c, self.dfeat_c, self.ddepth_c, self.grads_c, mode,
                                             C.c_void_p(self.workspace.data_ptr()), wb, C.byref(plan)),
                    "fe_batch_plan_create")
        self.plan = plan

    def launch(self, stream=None):
        rast._check(self.lib.fe_batch_launch(self.plan, C.c_void_p(rast._stream_handle(stream))), "fe_batch_launch")

    def report(self, f, stream=None) -> dict:
        r = rast.fe_report()
        self.lib.fe_batch_read_report(self.plan, f, C.byref(r), C.c_void_p(rast._stream_handle(stream)))
        return dict(status=r.status, keys_needed=r.keys_needed, n_visible=r.n_visible,
                    n_culled_nonfinite=r.n_culled_nonfinite, rows_needed=r.rows_needed)

    def close(self):
        if self.plan:
            self.lib.fe_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
