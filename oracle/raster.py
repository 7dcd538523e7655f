"""Tile binning and front-to-back compositing in float64 (eqs. 1, 7, 8).

Test infrastructure only (see the package docstring).

Binning (a tile rasterizer is an acceleration structure, so its result is
fixed by the per-pixel definition below; binning only has to reproduce the
key order exactly):
* every visible Gaussian emits one key per tile of its pixel box's tile
  rectangle; key = (tile_id << 32) | bits(float32 depth), tile_id =
  ty * tiles_x + tx; keys ascend, equal keys by Gaussian index ascending.

Per pixel p with centre (i + 1/2, j + 1/2), over the Gaussians of p's tile
in key order, starting from T = 1, C = 0, Z = 0:
* d = p - (u, v); q = d^T conic d              (exponent of eq. 1)
* the Gaussian counts only if p lies inside its pixel box and q <= 9
* alpha = min(0.99, o exp(-q / 2)); alpha < 1/255 is skipped
* T' = T (1 - alpha); if T' < 1e-4 the pixel stops and this Gaussian is
  excluded
* C += alpha T c, Z += alpha T f (eqs. 7-8, same weights), T = T'
* the depth image takes the same weights on the view-space depth t_z of each
  Gaussian (colour, depth and features are rendered in one pass, Sec. 3,
  method overview): Dp += alpha T t_z
and rgb = C + T bg, feature = Z (feature background 0), depth = Dp (depth
background 0), final T = T, n_contrib = 1 + list position of the last
included Gaussian (0 if none).
"""
from __future__ import annotations

from dataclasses import dataclass
import hashlib
import itertools
import numpy as np
import torch

from .project import project, round_projected, OracleCamera, OracleConfig, F64

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_STOP = 1e-4
Q_MAX = 9.0


@dataclass
class TileLists:
    tiles_x: int
    tiles_y: int
    tile_of: np.ndarray   # [K] int64, sorted
    gidx: np.ndarray      # [K] int64
    ranges: np.ndarray    # [tiles, 2] int64 [start, end)
    depth_bits: np.ndarray  # [K] uint32

    @property
    def k(self) -> int:
        return int(self.gidx.shape[0])


def depth_bits(depth64: torch.Tensor) -> np.ndarray:
    return depth64.detach().to(torch.float32).numpy().view(np.uint32)


def bin_gaussians(proj: dict, cam: OracleCamera, cfg: OracleConfig) -> TileLists:
    tiles_x = -(-cam.width // cfg.tile_w)
    tiles_y = -(-cam.height // cfg.tile_h)
    rect = proj["rect"].numpy()
    count = proj["count"].numpy()
    dbits = depth_bits(proj["depth"])
    gid, tid = [], []
    for g in np.nonzero(count > 0)[0]:
        tx0, ty0, tx1, ty1 = rect[g]
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                gid.append(g)
                tid.append(ty * tiles_x + tx)
    gid = np.asarray(gid, dtype=np.int64)
    tid = np.asarray(tid, dtype=np.int64)
    db = dbits[gid] if gid.size else np.zeros(0, np.uint32)
    order = np.lexsort((gid, db, tid))      # primary tile, then depth bits, then index
    tid, gid, db = tid[order], gid[order], db[order]
    ntiles = tiles_x * tiles_y
    starts = np.searchsorted(tid, np.arange(ntiles), side="left")
    ends = np.searchsorted(tid, np.arange(ntiles), side="right")
    return TileLists(tiles_x, tiles_y, tid, gid, np.stack([starts, ends], 1), db)


def tile_pixels(tile: int, lists: TileLists, cam: OracleCamera, cfg: OracleConfig):
    tx, ty = tile % lists.tiles_x, tile // lists.tiles_x
    jj, ii = np.meshgrid(np.arange(cfg.tile_h), np.arange(cfg.tile_w), indexing="ij")
    pi = (tx * cfg.tile_w + ii).reshape(-1)
    pj = (ty * cfg.tile_h + jj).reshape(-1)
    keep = (pi < cam.width) & (pj < cam.height)
    return pi[keep], pj[keep]


def composite_tile(pi, pj, xy, conic, op, rgb, feat, box, bg, amb_delta=None, depth=None):
    """Blend one tile.  pi, pj: [P] int pixel indices; per-Gaussian tensors
    [L, ...] in list order (``depth`` [L] view-space depths, optional).
    Differentiable in xy, conic, op, rgb, feat, depth."""
    P, L = len(pi), xy.shape[0]
    pit = torch.as_tensor(pi, dtype=torch.int64)
    pjt = torch.as_tensor(pj, dtype=torch.int64)
    px = pit.to(F64)[:, None] + 0.5
    py = pjt.to(F64)[:, None] + 0.5
    dx = px - xy[None, :, 0]
    dy = py - xy[None, :, 1]
    q = (conic[None, :, 0] * dx * dx + 2.0 * conic[None, :, 1] * dx * dy) + conic[None, :, 2] * dy * dy
    inbox = ((pit[:, None] >= box[None, :, 0]) & (pit[:, None] <= box[None, :, 2])
             & (pjt[:, None] >= box[None, :, 1]) & (pjt[:, None] <= box[None, :, 3]))
    g = torch.exp(-0.5 * q)
    a = torch.clamp(op[None, :] * g, max=ALPHA_MAX)
    qd, ad = q.detach(), a.detach()
    active = inbox & (qd <= Q_MAX) & (ad >= ALPHA_MIN)
    a_act = torch.where(active, ad, torch.zeros_like(ad))
    t_after = torch.cumprod(1.0 - a_act, dim=1)
    incl = active & (t_after >= T_STOP)
    a_inc = torch.where(incl, a, torch.zeros_like(a))
    one_minus = 1.0 - a_inc
    t_incl = torch.cumprod(one_minus, dim=1)
    t_before = torch.cat([torch.ones(P, 1, dtype=F64), t_incl[:, :-1]], dim=1) if L > 0 else t_incl
    w = a_inc * t_before
    C = w @ rgb
    Z = w @ feat
    Dp = w @ depth if depth is not None else None
    T = t_incl[:, -1] if L > 0 else torch.ones(P, dtype=F64)
    out_rgb = C + T[:, None] * torch.as_tensor(bg, dtype=F64)[None, :]
    pos = torch.arange(1, L + 1, dtype=torch.int64)[None, :]
    ncon = torch.where(incl, pos, torch.zeros_like(pos)).max(dim=1).values if L > 0 else torch.zeros(P, dtype=torch.int64)
    aclamp = incl & ((op[None, :] * g).detach() > ALPHA_MAX)
    res = dict(rgb=out_rgb, feat=Z, T=T, n_contrib=ncon, w=w, incl=incl, aclamp=aclamp, depth=Dp)
    if amb_delta is not None:
        dq, da, dt = amb_delta
        stop_hit = active & (t_after < T_STOP)
        # positions up to and including the first stop
        if L > 0:
            first_stop = torch.where(stop_hit.any(1), stop_hit.to(torch.int64).argmax(1), torch.full((P,), L))
        else:
            first_stop = torch.zeros(P, dtype=torch.int64)
        upto = torch.arange(L)[None, :] <= first_stop[:, None]
        near_q = inbox & ((qd - Q_MAX).abs() <= dq * Q_MAX)
        near_a = inbox & (qd <= Q_MAX * (1 + dq)) & ((ad - ALPHA_MIN).abs() <= da * ALPHA_MIN)
        near_t = active & ((t_after - T_STOP).abs() <= dt * T_STOP)
        res["near"] = dict(q=near_q & upto, a=near_a & upto, t=near_t & upto)
        res["ambiguous"] = ((near_q | near_a | near_t) & upto).any(1)
    return res


def composite(proj: dict, feat: torch.Tensor, lists: TileLists, cam: OracleCamera, cfg: OracleConfig,
              amb_delta=None, keep_weights=False, tiles=None, trace=False):
    """Render all tiles (or the listed ones) from a projected record."""
    H, W = cam.height, cam.width
    D = feat.shape[1]
    rgb = torch.zeros(3, H, W, dtype=F64)
    Z = torch.zeros(D, H, W, dtype=F64)
    Dimg = torch.zeros(H, W, dtype=F64)
    T = torch.ones(H, W, dtype=F64)
    ncon = torch.zeros(H, W, dtype=torch.int64)
    amb = torch.zeros(H, W, dtype=torch.bool)
    near = {}
    weights = {}
    tr = hashlib.sha1() if trace else None
    xy, conic, op, col = proj["xy"].detach(), proj["conic"].detach(), proj["opacity"].detach(), proj["rgb"].detach()
    dep = proj["depth"].detach()
    box = proj["box"]
    featd = feat.detach()
    it = range(lists.tiles_x * lists.tiles_y) if tiles is None else tiles
    for t in it:
        pi, pj = tile_pixels(t, lists, cam, cfg)
        s, e = lists.ranges[t]
        gi = torch.as_tensor(lists.gidx[s:e])
        r = composite_tile(pi, pj, xy[gi], conic[gi], op[gi], col[gi], featd[gi], box[gi], cfg.bg, amb_delta,
                           depth=dep[gi])
        rgb[:, pj, pi] = r["rgb"].T
        Z[:, pj, pi] = r["feat"].T
        Dimg[pj, pi] = r["depth"]
        T[pj, pi] = r["T"]
        ncon[pj, pi] = r["n_contrib"]
        if amb_delta is not None:
            amb[pj, pi] = r["ambiguous"]
            if r["ambiguous"].any():
                near[t] = (pi, pj, r["near"])
        if keep_weights:
            weights[t] = (pi, pj, gi.numpy(), r["w"].numpy(), r["incl"].numpy())
        if tr is not None:
            tr.update(np.packbits(r["incl"].numpy()).tobytes())
            tr.update(np.packbits(r["aclamp"].numpy()).tobytes())
    return dict(rgb=rgb, feat=Z, depth=Dimg, final_T=T, n_contrib=ncon, ambiguous=amb, near=near, weights=weights,
                trace=tr.hexdigest() if tr is not None else None)


def render_forward(means, scales, quats, opacity, sh, feat, cam, cfg: OracleConfig, parity=True,
                   amb_delta=None, keep_weights=False, tiles=None, trace=False):
    """Full forward: project, (parity mode) round the projected record to
    float32 once, bin, blend.  ``feat`` is used as given (float64 widening of
    its stored values)."""
    cam = cam if isinstance(cam, OracleCamera) else OracleCamera.from_any(cam)
    cfg = cfg.f32()
    with torch.no_grad():
        p = project(means, scales, quats, opacity, sh, cam, cfg)
        pr = round_projected(p) if parity else p
        lists = bin_gaussians(pr, cam, cfg)
        f = torch.as_tensor(np.asarray(feat), dtype=F64)
        out = composite(pr, f, lists, cam, cfg, amb_delta=amb_delta, keep_weights=keep_weights, tiles=tiles,
                        trace=trace)
        if trace:
            h = hashlib.sha1(out["trace"].encode())
            for k in ("visible", "box", "rect", "xclamped"):
                h.update(pr[k].numpy().tobytes())
            h.update((pr["rgb_raw"].numpy() < 0).tobytes())
            h.update(lists.gidx.tobytes())
            out["trace"] = h.hexdigest()
    out["proj"] = pr
    out["lists"] = lists
    out["cam"] = cam
    out["cfg"] = cfg
    return out


def brute_force_render(proj: dict, feat, cam: OracleCamera, cfg: OracleConfig):
    """Tile-free reference: per pixel, every visible Gaussian whose pixel box
    holds the pixel, ordered by (float32 depth bits, index), blended with the
    same rules in a plain sequential loop.  Tiny scenes only."""
    H, W = cam.height, cam.width
    feat = np.asarray(feat, dtype=np.float64)
    D = feat.shape[1]
    xy = proj["xy"].detach().numpy()
    conic = proj["conic"].detach().numpy()
    op = proj["opacity"].detach().numpy()
    col = proj["rgb"].detach().numpy()
    dep = proj["depth"].detach().numpy()
    box = proj["box"].numpy()
    vis = proj["visible"].numpy()
    db = depth_bits(proj["depth"])
    bg = np.asarray(cfg.bg, dtype=np.float64)
    rgb = np.zeros((3, H, W))
    Z = np.zeros((D, H, W))
    Dimg = np.zeros((H, W))
    Tf = np.ones((H, W))
    lists = {}
    cand = np.nonzero(vis)[0]
    for j in range(H):
        for i in range(W):
            m = cand[(box[cand, 0] <= i) & (box[cand, 2] >= i) & (box[cand, 1] <= j) & (box[cand, 3] >= j)]
            order = m[np.lexsort((m, db[m]))]
            T = 1.0
            C = np.zeros(3)
            z = np.zeros(D)
            dsum = 0.0
            used, ws = [], []
            for g in order:
                dx = (i + 0.5) - xy[g, 0]
                dy = (j + 0.5) - xy[g, 1]
                q = (conic[g, 0] * dx * dx + 2.0 * conic[g, 1] * dx * dy) + conic[g, 2] * dy * dy
                if q > Q_MAX:
                    continue
                a = min(ALPHA_MAX, op[g] * np.exp(-0.5 * q))
                if a < ALPHA_MIN:
                    continue
                Tn = T * (1.0 - a)
                if Tn < T_STOP:
                    break
                w = a * T
                C = C + w * col[g]
                z = z + w * feat[g]
                dsum += w * dep[g]
                used.append(int(g))
                ws.append(w)
                T = Tn
            rgb[:, j, i] = C + T * bg
            Z[:, j, i] = z
            Dimg[j, i] = dsum
            Tf[j, i] = T
            lists[(i, j)] = (used, ws)
    return dict(rgb=rgb, feat=Z, depth=Dimg, final_T=Tf, lists=lists)


def pixel_variants(i, j, proj: dict, feat, lists: TileLists, cam: OracleCamera, cfg: OracleConfig,
                   near: dict, max_flips=3):
    """All outcomes of one pixel when each near-threshold decision (from
    ``composite(..., amb_delta)``) may go either way.  Returns a list of
    (rgb[3], feat[D], T, n_contrib, depth) or None if too many decisions are near."""
    tiles_x = lists.tiles_x
    t = (j // cfg.tile_h) * tiles_x + (i // cfg.tile_w)
    pis, pjs, nr = near
    k = int(np.nonzero((pis == i) & (pjs == j))[0][0])
    cands = []
    for kind in ("q", "a", "t"):
        for pos in np.nonzero(nr[kind][k].numpy())[0]:
            cands.append((int(pos), kind))
    if len(cands) > max_flips:
        return None
    s, e = lists.ranges[t]
    gl = lists.gidx[s:e]
    xy = proj["xy"].detach().numpy()
    conic = proj["conic"].detach().numpy()
    op = proj["opacity"].detach().numpy()
    col = proj["rgb"].detach().numpy()
    dep = proj["depth"].detach().numpy()
    box = proj["box"].numpy()
    feat = np.asarray(feat, dtype=np.float64)
    bg = np.asarray(cfg.bg, dtype=np.float64)
    outs = []
    for mask in itertools.product([False, True], repeat=len(cands)):
        flips = {c for c, f in zip(cands, mask) if f}
        T, C, z, last, dsum = 1.0, np.zeros(3), np.zeros(feat.shape[1]), 0, 0.0
        for pos, g in enumerate(gl):
            if not (box[g, 0] <= i <= box[g, 2] and box[g, 1] <= j <= box[g, 3]):
                continue
            dx = (i + 0.5) - xy[g, 0]
            dy = (j + 0.5) - xy[g, 1]
            q = (conic[g, 0] * dx * dx + 2.0 * conic[g, 1] * dx * dy) + conic[g, 2] * dy * dy
            if (q > Q_MAX) != ((pos, "q") in flips):
                continue
            a = min(ALPHA_MAX, op[g] * np.exp(-0.5 * q))
            if (a < ALPHA_MIN) != ((pos, "a") in flips):
                continue
            Tn = T * (1.0 - a)
            if (Tn < T_STOP) != ((pos, "t") in flips):
                break
            w = a * T
            C = C + w * col[g]
            z = z + w * feat[g]
            dsum += w * dep[g]
            T = Tn
            last = pos + 1
        outs.append((C + T * bg, z, T, last, dsum))
    return outs
