"""Helpers shared by the GPU parity tests: move a seeded scene to the GPU,
run the HIP path through the C ABI, read back the state, and compare with
the FP64 oracle under the acceptance rules for near-threshold decisions."""
from __future__ import annotations

import numpy as np
import torch

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import bf16_round, crop_camera
import oracle
from oracle.raster import pixel_variants

# relative half-widths of the near-threshold windows: q vs 9, alpha vs 1/255, T' vs 1e-4
AMB_DELTA = (2e-6, 2e-6, 1e-5)


def settings_for(sc, tile=(16, 16), dtype="f32", **kw):
    return rast.Settings(sh_degree=sc.sh_degree, feat_dim=sc.feat_dim, tile_w=tile[0], tile_h=tile[1],
                         sh_dtype=dtype, feat_dtype=dtype, **kw)


def stored_inputs(sc, dtype="f32"):
    """Inputs as the GPU stores them (BF16-rounded SH / features for the BF16 form)."""
    sh = sc.sh if dtype == "f32" else bf16_round(sc.sh)
    feat = sc.feat if dtype == "f32" else bf16_round(sc.feat)
    return dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=sh, feat=feat)


def to_device(sc, dtype="f32", dev="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    lo = torch.bfloat16 if dtype == "bf16" else torch.float32
    return dict(means=t(sc.means), scales=t(sc.scales), quats=t(sc.quats), opacity=t(sc.opacity),
                sh=t(sc.sh).to(lo).contiguous(), feat=t(sc.feat).to(lo).contiguous())


def gpu_forward(sc, st, cam=None, dev_in=None, check=True):
    d = dev_in if dev_in is not None else to_device(sc, st.feat_dtype)
    fwd = rast.render_forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              cam if cam is not None else sc.cam, st, check=check)
    torch.cuda.synchronize()
    return fwd, d


def read_state(fwd, n, st, cam):
    lay = rast.state_layout(cam, st, n, fwd.cfg.key_capacity)
    s = fwd.state
    view = lambda off, dt, count: s[off: off + count * torch.tensor([], dtype=dt).element_size()].view(dt)
    rep = rast.read_report(s)
    k = int(rep["keys_needed"]) if rep["status"] == 0 else 0
    out = dict(
        xy=view(lay["xy"], torch.float32, 2 * n).reshape(n, 2).cpu().numpy(),
        conic_o=view(lay["conic_opacity"], torch.float32, 4 * n).reshape(n, 4).cpu().numpy(),
        rgb=view(lay["rgb"], torch.float32, 4 * n).reshape(n, 4).cpu().numpy(),
        box=view(lay["box"], torch.int16, 4 * n).reshape(n, 4).cpu().numpy().astype(np.int64),
        depth_key=view(lay["depth_key"], torch.int32, n).cpu().numpy().view(np.uint32),
        count=view(lay["tile_count"], torch.int32, n).cpu().numpy(),
        gauss=view(lay["sorted_gauss"], torch.int32, max(k, 1)).cpu().numpy()[:k],
        report=rep,
    )
    nt = -(-cam.width // st.tile_w) * -(-cam.height // st.tile_h)
    out["ranges"] = view(lay["ranges"], torch.int32, 2 * nt).reshape(nt, 2).cpu().numpy().astype(np.int64)
    return out


def oracle_cfg(sc, st):
    return oracle.OracleConfig(tile_w=st.tile_w, tile_h=st.tile_h, sh_degree=sc.sh_degree, bg=tuple(st.bg),
                               dilation=st.dilation, jacobian_clamp=st.jacobian_clamp)


def oracle_forward(sc, st, cam=None, tiles=None):
    inp = stored_inputs(sc, st.feat_dtype)
    return oracle.render_forward(**inp, cam=cam if cam is not None else sc.cam, cfg=oracle_cfg(sc, st),
                                 parity=True, amb_delta=AMB_DELTA, tiles=tiles)


def compare_projection(gs, orc, n):
    p = orc["proj"]
    vis = p["visible"].numpy()
    assert np.array_equal(gs["count"], p["count"].numpy().astype(np.int32)), "tile counts differ"
    # depth keys: float32 depth bits of every Gaussian (culled: all ones)
    keys = p["depth"].numpy().astype(np.float32).view(np.uint32).copy()
    keys[~vis] = 0xFFFFFFFF
    assert np.array_equal(gs["depth_key"], keys), "depth keys differ"
    assert np.array_equal(gs["box"][vis], p["box"].numpy()[vis]), "pixel boxes differ"
    xy = p["xy"].numpy().astype(np.float32)
    con = p["conic"].numpy().astype(np.float32)
    rgb = p["rgb"].numpy().astype(np.float32)
    np.testing.assert_array_equal(gs["xy"][vis], xy[vis])
    np.testing.assert_allclose(gs["conic_o"][vis, :3], con[vis], rtol=2e-7, atol=0)
    np.testing.assert_array_equal(gs["conic_o"][vis, 3], p["opacity"].numpy().astype(np.float32)[vis])
    np.testing.assert_allclose(gs["rgb"][vis, :3], rgb[vis], rtol=1e-6, atol=1e-7)
    # the report's visible count (summed over the binning workgroups)
    assert gs["report"]["n_visible"] == int(vis.sum()), (gs["report"]["n_visible"], int(vis.sum()))
    return int(vis.sum())


def compare_keys(gs, orc):
    L = orc["lists"]
    assert gs["report"]["keys_needed"] == L.k
    np.testing.assert_array_equal(gs["gauss"].astype(np.int64), L.gidx)
    # tiles laid out in id order: the ranges are the oracle's, empty ones included
    np.testing.assert_array_equal(gs["ranges"], L.ranges)


def compare_images(fwd, orc, sc, st, tiles=None, tol=1e-5, feat_in=None):
    """Normwise relative error of rgb / feat / final_T over pixels without a
    near-threshold decision; near-threshold pixels must match one of the
    oracle's branch variants.  Returns a dict of statistics."""
    g_rgb = fwd.rgb.double().cpu().numpy()
    g_feat = fwd.feat.double().cpu().numpy()
    g_T = fwd.final_T.double().cpu().numpy()
    g_n = fwd.n_contrib.cpu().numpy()
    g_d = fwd.depth.double().cpu().numpy() if getattr(fwd, "depth", None) is not None else None
    o_d = orc["depth"].numpy()
    o_rgb, o_feat = orc["rgb"].numpy(), orc["feat"].numpy()
    o_T, o_n = orc["final_T"].numpy(), orc["n_contrib"].numpy()
    H, W = o_T.shape
    mask = np.ones((H, W), bool)
    if tiles is not None:
        mask[:] = False
        tx = -(-W // st.tile_w)
        for t in tiles:
            x0, y0 = (t % tx) * st.tile_w, (t // tx) * st.tile_h
            mask[y0:y0 + st.tile_h, x0:x0 + st.tile_w] = True
    amb = orc["ambiguous"].numpy() & mask
    clean = mask & ~amb
    stats = {}
    for name, g, o in (("rgb", g_rgb, o_rgb), ("feat", g_feat, o_feat)):
        ref = max(np.abs(o[:, mask]).max(), 1e-30)
        err = np.abs(g - o)[:, clean].max() / ref if clean.any() else 0.0
        stats[name] = err
        assert err <= tol, (name, err)
    if g_d is not None:
        ref = max(np.abs(o_d[mask]).max(), 1e-30)
        err = np.abs(g_d - o_d)[clean].max() / ref if clean.any() else 0.0
        stats["depth"] = err
        assert err <= tol, ("depth", err)
    errT = np.abs(g_T - o_T)[clean].max() if clean.any() else 0.0
    stats["final_T"] = errT
    assert errT <= tol, ("final_T", errT)
    bad_n = int((g_n != o_n)[clean].sum())
    stats["n_contrib_mismatch"] = bad_n
    assert bad_n == 0, ("n_contrib", bad_n)
    # near-threshold pixels: accept any branch outcome
    unresolved = 0
    feat_in = stored_inputs(sc, st.feat_dtype)["feat"] if feat_in is None else feat_in
    ref_r = max(np.abs(o_rgb[:, mask]).max(), 1e-30)
    ref_f = max(np.abs(o_feat[:, mask]).max(), 1e-30)
    ref_d = max(np.abs(o_d[mask]).max(), 1e-30)
    for j, i in zip(*np.nonzero(amb)):
        t = (j // st.tile_h) * (-(-W // st.tile_w)) + i // st.tile_w
        vs = pixel_variants(int(i), int(j), orc["proj"], feat_in, orc["lists"], orc["cam"], orc["cfg"],
                            orc["near"][t])
        ok = False
        if vs is not None:
            for (vr, vf, vT, vn, vd) in vs:
                if (np.abs(vr - g_rgb[:, j, i]).max() <= tol * ref_r and np.abs(vf - g_feat[:, j, i]).max() <= tol * ref_f
                        and abs(vT - g_T[j, i]) <= tol and (g_d is None or abs(vd - g_d[j, i]) <= tol * ref_d)):
                    ok = True
                    break
        unresolved += 0 if ok else 1
    stats["ambiguous"] = int(amb.sum())
    stats["unresolved"] = unresolved
    assert unresolved == 0, stats
    return stats


def oracle_backward(sc, st, d_rgb, d_feat, cam=None, tiles=None, d_depth=None):
    inp = stored_inputs(sc, st.feat_dtype)
    return oracle.render_backward(**inp, cam=cam if cam is not None else sc.cam, cfg=oracle_cfg(sc, st),
                                  d_rgb=d_rgb, d_feat=d_feat, parity=True, tiles=tiles, d_depth=d_depth)


def depth_grad(H, W, seed, std=1e-3):
    """An upstream depth-image gradient (its own generator, so the other
    draws of a test are unchanged)."""
    return np.random.default_rng(10_000 + seed).normal(0, std, (H, W)).astype(np.float32)


def screen_grads(gr, n):
    """The backward's per-Gaussian screen-space sums from its scratch:
    u v A B C opacity r g b depth."""
    g2 = gr["_scratch"][: 48 * n].view(torch.float32).reshape(n, 12).cpu().numpy()
    return dict(xy=g2[:, 0:2], conic=g2[:, 2:5], opacity2d=g2[:, 5], rgb2d=g2[:, 6:9], depth2d=g2[:, 9])


SCREEN_KEYS = ("xy", "conic", "opacity2d", "rgb2d", "depth2d")


def normwise(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


GRAD_KEYS = ("means", "scales", "quats", "opacity", "sh", "feat")


def grad_errors(g, o):
    """(normwise L2 relative, max |g - o| / max |o|) of one gradient group;
    a group whose reference is exactly zero must be zero too."""
    g = np.asarray(g.detach().double().cpu().numpy() if isinstance(g, torch.Tensor) else g, np.float64).reshape(-1)
    o = np.asarray(o, np.float64).reshape(-1)
    ref = np.abs(o).max() if o.size else 0.0
    if ref == 0.0:
        return (0.0, 0.0) if not np.abs(g).max(initial=0.0) else (np.inf, np.inf)
    return normwise(g, o), float(np.abs(g - o).max() / ref)


def check_grads(gr, ob, keys=GRAD_KEYS, tol=1e-4, tol_inf=1e-4):
    """Every gradient group against the oracle: normwise L2 relative error
    below ``tol`` and the largest element error below ``tol_inf`` times the
    group's largest reference magnitude (a few wrong Gaussians with small
    gradients cannot hide in the norm)."""
    errs = {}
    for k in keys:
        nw, inf = grad_errors(gr[k], ob[k])
        errs[k] = (nw, inf)
        assert nw < tol and inf < tol_inf, (k, nw, inf)
    print("[grads] normwise / max-element:", {k: (f"{a:.2e}", f"{b:.2e}") for k, (a, b) in errs.items()}, flush=True)
    return errs
