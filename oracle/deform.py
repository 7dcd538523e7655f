"""FST deformation module in float64 (Sec. 3.2, eqs. 4-6; appendix "FST
Deformation Module" and the hyper-parameter table).

Test infrastructure only (see the package docstring).

A Gaussian with centre mu at time t is encoded by a multi-resolution
HexPlane into a feature f, decoded by the MLP F_out into h in R^W, and four
branches predict the geometric updates; the semantic updater F_feat turns the
branches' features into the feature update (eq. 5) and G_t is assembled as in
eq. (6).  Readings of what the paper leaves open (each one is stated again
where it is used):

* HexPlane: the six planes are the coordinate pairs of (x, y, z, t) in the
  order (x,y), (x,z), (x,t), (y,z), (y,t), (z,t); plane (a, b) is a grid of
  res_b rows by res_a columns with C channels.  Per resolution level the six
  planes' samples are multiplied channel by channel; the levels' products are
  concatenated in the order of the multipliers [1, 2, 4, 8], so f has 4 C
  entries.  A spatial coordinate has 64 m grid points at level m, time has
  100 at every level.
* Sampling: the spatial coordinates are mapped to [-1, 1] by a caller-given
  axis-aligned box and time t in [0, 1] to 2 t - 1, clamped to [-1, 1];
  bilinear interpolation with the grid's first and last points on -1 and 1.
* F_out: eight affine layers of width W with ReLU between them (none after
  the last).
* Branch g in (mu, R, S, o): h_g = B2(relu(B1(relu(h)))), B1: W -> W,
  B2: W -> W/2 (two linear layers down to W/2); the head is
  dg = H(relu(h_g)), H: W/2 -> d_g with d = (3, 4, 3, 1).
* u_all = [h_mu | h_R | h_S | h_o] has 4 (W/2) = 2W entries (the appendix's
  W/2 branch width; Sec. 3.2 prints 4W).
* F_feat: dz = E2(relu(E1(u_all))), E1: 2W -> W, E2: W -> N.
* eq. (6) in the optimiser's parameters: mu + dmu; q + dq (left unnormalised,
  the rasterizer normalises); scale exp(log s + ds); opacity
  sigmoid(logit o + do); z' = z + dz.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64
PLANE_PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
LEVELS = (1, 2, 4, 8)
BASE_RES = (64, 64, 64, 100)
BRANCHES = ("mu", "rot", "scale", "opacity")
BRANCH_DIMS = {"mu": 3, "rot": 4, "scale": 3, "opacity": 1}


def resolution(level_mult: int, coord: int, base=BASE_RES) -> int:
    """Grid points of coordinate ``coord`` at level multiplier ``level_mult``
    (space is refined, time is not)."""
    return base[coord] * level_mult if coord < 3 else base[coord]


def normalized_coords(means, t, lo, hi):
    """(x, y, z, t) mapped to [-1, 1]: space by the box [lo, hi], time t in
    [0, 1] by 2 t - 1; clamped to the box."""
    m = torch.as_tensor(np.asarray(means), dtype=F64)
    lo = torch.as_tensor(np.asarray(lo), dtype=F64)
    hi = torch.as_tensor(np.asarray(hi), dtype=F64)
    u = 2.0 * (m - lo) / (hi - lo) - 1.0
    ut = torch.full((m.shape[0], 1), 2.0 * float(t) - 1.0, dtype=F64)
    return torch.cat([u, ut], 1).clamp(-1.0, 1.0)


def bilinear(plane, ua, ub):
    """Sample plane [rows = res_b][cols = res_a][C] at (ua, ub) in [-1, 1]^2
    with the grid's end points on -1 and 1.  Returns [n, C]."""
    g = torch.as_tensor(np.asarray(plane), dtype=F64)
    rb, ra = g.shape[0], g.shape[1]
    x = (ua + 1.0) / 2.0 * (ra - 1)
    y = (ub + 1.0) / 2.0 * (rb - 1)
    x0 = torch.floor(x).clamp(0, ra - 2).long()
    y0 = torch.floor(y).clamp(0, rb - 2).long()
    wx = (x - x0.to(F64))[:, None]
    wy = (y - y0.to(F64))[:, None]
    return ((1 - wx) * (1 - wy) * g[y0, x0] + wx * (1 - wy) * g[y0, x0 + 1]
            + (1 - wx) * wy * g[y0 + 1, x0] + wx * wy * g[y0 + 1, x0 + 1])


def hexplane_features(means, t, planes, lo, hi):
    """f [n, 4 C]: per level the channel-wise product of the six planes'
    samples, levels concatenated.  ``planes[l][p]`` is level l's plane for
    pair PLANE_PAIRS[p]."""
    u = normalized_coords(means, t, lo, hi)
    feats = []
    for lvl in planes:
        prod = None
        for p, (a, b) in enumerate(PLANE_PAIRS):
            s = bilinear(lvl[p], u[:, a], u[:, b])
            prod = s if prod is None else prod * s
        feats.append(prod)
    return torch.cat(feats, 1)


def _affine(x, layer):
    w, b = layer
    return x @ torch.as_tensor(np.asarray(w), dtype=F64).T + torch.as_tensor(np.asarray(b), dtype=F64)


def deform_mlp(f, layers):
    """The MLPs on features f [n, 4 C].  ``layers`` holds (weight [out, in],
    bias [out]) pairs: 'out' (8 layers of F_out), 'branch_<g>' (B1, B2),
    'head_<g>' (H), 'sem' (E1, E2).  Returns h, the branch features, the
    updates d<g> and dz (float64 tensors)."""
    x = torch.as_tensor(f, dtype=F64) if not torch.is_tensor(f) else f.to(F64)
    out_layers = layers["out"]
    for i, layer in enumerate(out_layers):
        x = _affine(x if i == 0 else torch.relu(x), layer)
    h = x
    res = {"h": h}
    hg = []
    for g in BRANCHES:
        b1, b2 = layers["branch_" + g]
        y = _affine(torch.relu(_affine(torch.relu(h), b1)), b2)
        res["h_" + g] = y
        res["d_" + g] = _affine(torch.relu(y), layers["head_" + g])
        hg.append(y)
    u_all = torch.cat(hg, 1)
    e1, e2 = layers["sem"]
    res["d_feat"] = _affine(torch.relu(_affine(u_all, e1)), e2)
    return res


def deform_gaussians(means, quats, log_scales, logit_opacity, feat, t, params):
    """G_t of eq. (6).  ``params``: dict with 'planes', 'lo', 'hi', 'layers'.
    Returns float64 numpy arrays means [n,3], quats [n,4], scales [n,3]
    (linear), opacity [n] in (0, 1), feat [n, N], plus the MLP's
    intermediates."""
    f = hexplane_features(means, t, params["planes"], params["lo"], params["hi"])
    r = deform_mlp(f, params["layers"])
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=F64)
    out = dict(
        means=(T(means) + r["d_mu"]).numpy(),
        quats=(T(quats) + r["d_rot"]).numpy(),
        scales=torch.exp(T(log_scales) + r["d_scale"]).numpy(),
        opacity=torch.sigmoid(T(logit_opacity) + r["d_opacity"][:, 0]).numpy(),
        feat=(T(feat) + r["d_feat"]).numpy(),
        f=f.numpy(),
    )
    out.update({k: v.numpy() for k, v in r.items()})
    return out
