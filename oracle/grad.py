"""Gradients of the float64 oracle, and a central finite-difference harness.

Test infrastructure only (see the package docstring).

The paper trains every Gaussian parameter with Adam through the
differentiable rasterizer (Sec. 3.4 and 4.1), so the backward is the
derivative of the forward as defined in ``raster`` and ``project``.  It is
obtained here by reverse-mode differentiation of that same float64 graph
(torch autograd), one tile at a time for the blending and once for the
projection.  Discrete choices (culling, boxes, sort order, the skip and stop
tests) are piecewise constant and contribute nothing; the 0.99 opacity
clamp, the colour clamp at 0 and the clamped Jacobian coordinates pass zero.

``fd_gradient`` takes central differences with step h = h_rel max(1, |x|)
and accepts a sample only when the discrete trace of the forward (included
Gaussians per pixel, clamp flags, boxes, culling, key order) is the same at
x - h, x and x + h.
"""
from __future__ import annotations

import numpy as np
import torch

from .project import project, round_projected, OracleCamera, OracleConfig, F64
from .raster import bin_gaussians, tile_pixels, composite_tile, render_forward


def render_backward(means, scales, quats, opacity, sh, feat, cam, cfg: OracleConfig, d_rgb, d_feat,
                    parity=True, tiles=None, d_depth=None):
    """Gradient of L = <d_rgb, rgb> + <d_feat, feat_image> (+ <d_depth,
    depth_image>) with respect to every input.  Returns a dict with float64
    numpy arrays for means, scales, quats, opacity, sh, feat and the
    intermediate projected-record gradients (xy, conic, opacity2d, rgb2d,
    depth2d)."""
    cam = cam if isinstance(cam, OracleCamera) else OracleCamera.from_any(cam)
    cfg = cfg.f32()
    leaf = lambda a: torch.tensor(np.asarray(a), dtype=F64, requires_grad=True)
    mu, s, q, op, shc, ft = (leaf(means), leaf(scales), leaf(quats), leaf(opacity), leaf(sh), leaf(feat))
    p = project(mu, s, q, op, shc, cam, cfg)
    pr = round_projected(p) if parity else p
    lists = bin_gaussians(pr, cam, cfg)
    n, D = mu.shape[0], ft.shape[1]
    g_xy = torch.zeros(n, 2, dtype=F64)
    g_con = torch.zeros(n, 3, dtype=F64)
    g_op = torch.zeros(n, dtype=F64)
    g_rgb = torch.zeros(n, 3, dtype=F64)
    g_ft = torch.zeros(n, D, dtype=F64)
    g_dep = torch.zeros(n, dtype=F64)
    drgb = torch.as_tensor(np.asarray(d_rgb), dtype=F64)
    dfeat = torch.as_tensor(np.asarray(d_feat), dtype=F64)
    ddep = torch.as_tensor(np.asarray(d_depth), dtype=F64) if d_depth is not None else None
    xy_d, con_d, op_d, rgb_d = (pr["xy"].detach(), pr["conic"].detach(), pr["opacity"].detach(),
                                pr["rgb"].detach())
    dep_d = pr["depth"].detach()
    ft_d = ft.detach()
    it = range(lists.tiles_x * lists.tiles_y) if tiles is None else tiles
    for t in it:
        s0, e0 = lists.ranges[t]
        if e0 == s0:
            continue
        pi, pj = tile_pixels(t, lists, cam, cfg)
        gi = torch.as_tensor(lists.gidx[s0:e0])
        xs = [xy_d[gi].clone().requires_grad_(), con_d[gi].clone().requires_grad_(),
              op_d[gi].clone().requires_grad_(), rgb_d[gi].clone().requires_grad_(),
              ft_d[gi].clone().requires_grad_(), dep_d[gi].clone().requires_grad_()]
        r = composite_tile(pi, pj, xs[0], xs[1], xs[2], xs[3], xs[4], pr["box"][gi], cfg.bg, depth=xs[5])
        loss = (r["rgb"] * drgb[:, pj, pi].T).sum() + (r["feat"] * dfeat[:, pj, pi].T).sum()
        if ddep is not None:
            loss = loss + (r["depth"] * ddep[pj, pi]).sum()
        gs = torch.autograd.grad(loss, xs, allow_unused=True)
        for acc, gg in zip((g_xy, g_con, g_op, g_rgb, g_ft, g_dep), gs):
            if gg is not None:
                acc.index_add_(0, gi, gg)
    torch.autograd.backward([pr["xy"], pr["conic"], pr["rgb"], pr["opacity"], pr["depth"]],
                            [g_xy, g_con, g_rgb, g_op, g_dep])
    z = lambda t: np.zeros(t.shape) if t.grad is None else t.grad.numpy().copy()
    return dict(means=z(mu), scales=z(s), quats=z(q), opacity=z(op), sh=z(shc), feat=g_ft.numpy().copy(),
                xy=g_xy.numpy(), conic=g_con.numpy(), opacity2d=g_op.numpy(), rgb2d=g_rgb.numpy(),
                depth2d=g_dep.numpy(), lists=lists, proj=pr)


def render_loss(params: dict, cam, cfg: OracleConfig, d_rgb, d_feat, parity=False, d_depth=None):
    """Scalar <d_rgb, rgb> + <d_feat, feat> (+ <d_depth, depth>) of the pure
    float64 forward, and the forward's discrete trace."""
    out = render_forward(params["means"], params["scales"], params["quats"], params["opacity"],
                         params["sh"], params["feat"], cam, cfg, parity=parity, trace=True)
    loss = float((out["rgb"].numpy() * np.asarray(d_rgb, np.float64)).sum()
                 + (out["feat"].numpy() * np.asarray(d_feat, np.float64)).sum())
    if d_depth is not None:
        loss += float((out["depth"].numpy() * np.asarray(d_depth, np.float64)).sum())
    return loss, out["trace"]


def fd_gradient(params: dict, name: str, flat_indices, cam, cfg, d_rgb, d_feat, h_rel=1e-6, d_depth=None):
    """Central differences of ``render_loss`` for chosen entries of one
    parameter.  Returns (grads, valid) float64 / bool arrays."""
    base = {k: np.array(v, dtype=np.float64, copy=True) for k, v in params.items()}
    _, tr0 = render_loss(base, cam, cfg, d_rgb, d_feat, d_depth=d_depth)
    grads = np.zeros(len(flat_indices))
    valid = np.zeros(len(flat_indices), dtype=bool)
    for n_, fi in enumerate(flat_indices):
        arr = base[name].reshape(-1)
        x0 = arr[fi]
        h = h_rel * max(1.0, abs(x0))
        arr[fi] = x0 + h
        lp, tp = render_loss(base, cam, cfg, d_rgb, d_feat, d_depth=d_depth)
        arr[fi] = x0 - h
        lm, tm = render_loss(base, cam, cfg, d_rgb, d_feat, d_depth=d_depth)
        arr[fi] = x0
        grads[n_] = (lp - lm) / (2 * h)
        valid[n_] = (tp == tr0) and (tm == tr0)
    return grads, valid
