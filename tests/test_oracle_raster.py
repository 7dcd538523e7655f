"""Pins for the oracle's blending (eqs. 1, 7, 8) and binning: closed-form
images, ordering, the alpha rules, tile-free brute force, feature/colour
equivalence, linearity and the transmittance invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import render_forward, brute_force_render, project, bin_gaussians
from oracle.raster import pixel_variants
from tests.oracle_helpers import cam, gaussians, cfg

Y00 = 0.5 / math.sqrt(math.pi)


def _grid(w, h):
    ii, jj = np.meshgrid(np.arange(w), np.arange(h), indexing="xy")
    return ii + 0.5, jj + 0.5


def test_single_isotropic_gaussian_closed_form():
    f, s, z, o = 32.0, 0.08, 2.0, 0.8
    c = cam(32, 32, f=f)
    col, fv = np.array([0.9, 0.4, 0.2]), np.array([1.5, -2.0, 0.25])
    g = gaussians([[0, 0, z]], [s, s, s], opacity=o, colors=col, feat=[fv])
    out = render_forward(**g, cam=c, cfg=cfg(bg=(0.1, 0.2, 0.3)), parity=False)
    s32, o32 = float(np.float32(s)), float(np.float32(o))
    var = (f * s32 / z) ** 2 + float(np.float32(0.3))
    X, Yp = _grid(32, 32)
    q = ((X - 16) ** 2 + (Yp - 16) ** 2) / var
    a = np.minimum(0.99, o32 * np.exp(-0.5 * q))
    a = np.where((q <= 9) & (a >= 1 / 255), a, 0.0)
    bg = np.array([np.float32(0.1), np.float32(0.2), np.float32(0.3)], np.float64)
    col32 = np.maximum(0, Y00 * ((col - 0.5) / Y00).astype(np.float32) + 0.5)
    rgb = a[None] * col32[:, None, None] + (1 - a)[None] * bg[:, None, None]
    np.testing.assert_allclose(out["rgb"].numpy(), rgb, atol=1e-12)
    np.testing.assert_allclose(out["feat"].numpy(), a[None] * fv.astype(np.float32)[:, None, None], atol=1e-12)
    np.testing.assert_allclose(out["final_T"].numpy(), 1 - a, atol=1e-15)
    # depth image: the same weights on the view-space depth, background 0
    np.testing.assert_allclose(out["depth"].numpy(), a * z, atol=1e-12)


def test_rotated_anisotropic_gaussian_closed_form():
    # rotation about the optical axis by th, on axis: Sigma' = (f/z)^2 R2 diag(sx^2, sy^2) R2^T + 0.3 I
    f, z, th = 40.0, 2.5, 0.6
    sx, sy = float(np.float32(0.09)), float(np.float32(0.03))
    c = cam(40, 40, f=f)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    g = gaussians([[0, 0, z]], [[sx, sy, 0.01]], quats=[q], opacity=0.7, colors=[0.6, 0.6, 0.6], feat=[[1.0, 2.0]])
    out = render_forward(**g, cam=c, cfg=cfg(), parity=False)
    qq = np.asarray(g["quats"][0], np.float64)
    qq /= np.linalg.norm(qq)
    ang = 2 * math.atan2(qq[3], qq[0])
    R2 = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
    S2 = (f / z) ** 2 * R2 @ np.diag([sx * sx, sy * sy]) @ R2.T + float(np.float32(0.3)) * np.eye(2)
    Ci = np.linalg.inv(S2)
    X, Yp = _grid(40, 40)
    dx, dy = X - 20, Yp - 20
    qv = Ci[0, 0] * dx * dx + 2 * Ci[0, 1] * dx * dy + Ci[1, 1] * dy * dy
    a = np.minimum(0.99, float(np.float32(0.7)) * np.exp(-0.5 * qv))
    a = np.where((qv <= 9) & (a >= 1 / 255), a, 0.0)
    np.testing.assert_allclose(out["feat"][1].numpy(), 2.0 * a, atol=1e-10)
    assert abs(Ci[0, 1]) > 1e-3   # the off-diagonal term matters here


def test_two_gaussians_front_to_back_order():
    c = cam(16, 16, f=16.0)
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    for z1, z2 in ((2.0, 3.0), (3.0, 2.0)):
        # same screen position: scale the second so both have the same footprint
        g = gaussians([[0, 0, z1], [0, 0, z2]], [[0.1 * z1 / 2] * 3, [0.1 * z2 / 2] * 3],
                      opacity=[0.6, 0.5], colors=[c1, c2], feat=[[1.0, 0.0], [0.0, 1.0]])
        out = render_forward(**g, cam=c, cfg=cfg(), parity=False)
        p = out["proj"]
        a = []
        for k in range(2):
            A = p["conic"][k, 0].item()
            a.append(min(0.99, p["opacity"][k].item() * math.exp(-0.5 * A * 0.5)))   # pixel (8,8): d = (0.5,0.5)
        fr, bk = (0, 1) if z1 < z2 else (1, 0)
        expect = a[fr] * np.eye(2)[fr] + (1 - a[fr]) * a[bk] * np.eye(2)[bk]
        np.testing.assert_allclose(out["feat"][:, 8, 8].numpy(), expect, rtol=1e-12)
        zs = (z1, z2)
        np.testing.assert_allclose(out["depth"][8, 8].item(), a[fr] * zs[fr] + (1 - a[fr]) * a[bk] * zs[bk],
                                   rtol=1e-12)


def test_stop_rule_excludes_the_stopping_gaussian():
    # four identical Gaussians at alpha = 0.95: T = .05, .0025, 1.25e-4 are kept,
    # the fourth would take T below 1e-4 and is excluded
    c = cam(8, 8, f=8.0)
    g = gaussians([[0, 0, 2.0 + 0.01 * k] for k in range(4)], [[2.0 * (2.0 + 0.01 * k) / 2] * 3 for k in range(4)],
                  opacity=0.95, colors=[0.8, 0.5, 0.3], feat=np.ones((4, 2)))
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=False)
    p = out["proj"]
    a = [min(0.99, p["opacity"][k].item() * math.exp(-0.5 * (p["conic"][k, 0].item() * 0.5))) for k in range(4)]
    # pixel (4, 4): offset (0.5, 0.5) from the centre (4, 4)
    T = 1.0
    fe = 0.0
    for k in range(3):
        fe += a[k] * T
        T *= 1 - a[k]
    assert out["n_contrib"][4, 4].item() == 3
    np.testing.assert_allclose(out["feat"][0, 4, 4].item(), fe, rtol=1e-13)
    np.testing.assert_allclose(out["final_T"][4, 4].item(), T, rtol=1e-13)
    assert T >= 1e-4 and T * (1 - a[3]) < 1e-4
    assert abs(fe - (1 - 0.05 ** 3)) < 0.01


def test_skip_and_clamp_rules():
    c = cam(8, 8, f=8.0)
    # opacity so small that alpha < 1/255 everywhere: nothing changes
    g = gaussians([[0, 0, 2.0]], [[0.3, 0.3, 0.3]], opacity=0.999 / 255, colors=[1, 1, 1], feat=[[1.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=False)
    assert float(out["feat"].abs().max()) == 0.0 and float(out["final_T"].min()) == 1.0
    assert int(out["n_contrib"].max()) == 0
    # opacity 1 at the centre: o G >= 0.99 gives exactly 0.99
    g = gaussians([[0, 0, 2.0]], [[2.0, 2.0, 2.0]], opacity=1.0, colors=[1, 1, 1], feat=[[1.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=False)
    assert out["feat"][0, 4, 4].item() == 0.99
    assert out["final_T"][4, 4].item() == 1.0 - 0.99


def _random_scene(seed, n=120, w=40, h=36, f=36.0, d=5, sh_degree=1):
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(-0.7, 0.7, n), rng.uniform(-0.6, 0.6, n), rng.uniform(1.5, 4.0, n)], 1)
    g = gaussians(mu, np.exp(rng.normal(-2.9, 0.5, (n, 3))), quats=rng.normal(size=(n, 4)),
                  opacity=1 / (1 + np.exp(-rng.normal(size=n))), feat=rng.normal(size=(n, d)),
                  sh_degree=sh_degree)
    g["sh"][:] = rng.normal(0, 0.3, g["sh"].shape)
    g["sh"][:, 0, :] += 1.0
    return g, cam(w, h, f=f)


@pytest.mark.parametrize("seed", [0, 1])
def test_tiled_equals_brute_force(seed):
    g, c = _random_scene(seed)
    cf = cfg(tile=8, sh_degree=1, bg=(0.2, 0.1, 0.05))
    out = render_forward(**g, cam=c, cfg=cf, parity=True, keep_weights=True)
    bf = brute_force_render(out["proj"], g["feat"], out["cam"], out["cfg"])
    # weights and included Gaussians identical bit for bit; images to float64 rounding
    for t, (pi, pj, gi, w, incl) in out["weights"].items():
        for k in range(len(pi)):
            used, ws = bf["lists"][(int(pi[k]), int(pj[k]))]
            assert list(gi[incl[k]]) == used
            assert np.array_equal(w[k][incl[k]], np.asarray(ws))
    assert np.array_equal(out["final_T"].numpy(), bf["final_T"])
    np.testing.assert_allclose(out["rgb"].numpy(), bf["rgb"], atol=1e-14)
    np.testing.assert_allclose(out["feat"].numpy(), bf["feat"], atol=1e-13)
    np.testing.assert_allclose(out["depth"].numpy(), bf["depth"], atol=1e-13)


def test_image_independent_of_tile_shape():
    g, c = _random_scene(2)
    outs = [render_forward(**g, cam=c, cfg=cfg(tile=t, sh_degree=1), parity=True) for t in (4, 8, 16)]
    o2 = render_forward(**g, cam=c, cfg=__import__("oracle").OracleConfig(tile_w=16, tile_h=4, sh_degree=1),
                        parity=True)
    for o in outs[1:] + [o2]:
        assert np.array_equal(o["final_T"].numpy(), outs[0]["final_T"].numpy())
        np.testing.assert_allclose(o["feat"].numpy(), outs[0]["feat"].numpy(), atol=1e-14)


def test_features_equal_colour_and_linearity():
    g, c = _random_scene(3, sh_degree=0)
    cf = cfg(tile=8, sh_degree=0)
    p = project(**g, cam=c, cfg=cf)
    g3 = dict(g, feat=p["rgb"].numpy())                 # D = 3 features equal to the colours
    out = render_forward(**{k: np.asarray(v, np.float64) for k, v in g3.items()}, cam=c, cfg=cf, parity=False)
    np.testing.assert_allclose(out["feat"].numpy(), out["rgb"].numpy(), atol=1e-14)
    rng = np.random.default_rng(5)
    f1, f2 = rng.normal(size=g["feat"].shape), rng.normal(size=g["feat"].shape)
    r = lambda f: render_forward(**dict(g, feat=f), cam=c, cfg=cf, parity=False)["feat"].numpy()
    np.testing.assert_allclose(r(f1 + f2), r(f1) + r(f2), atol=1e-13)
    perm = rng.permutation(f1.shape[1])
    np.testing.assert_allclose(r(f1[:, perm]), r(f1)[perm], atol=1e-15)


def test_transmittance_invariants():
    g, c = _random_scene(4, n=300)
    out = render_forward(**g, cam=c, cfg=cfg(tile=8, sh_degree=1), parity=True, keep_weights=True)
    T = out["final_T"].numpy()
    assert T.min() >= 1e-4 and T.max() <= 1.0
    for t, (pi, pj, gi, w, incl) in out["weights"].items():
        assert (w >= 0).all()
        np.testing.assert_allclose(w.sum(1), 1 - T[pj, pi], atol=1e-14)


def test_binning_keys_cover_every_pixel_and_are_sorted():
    g, c = _random_scene(5, n=200)
    cf = cfg(tile=8, sh_degree=1)
    out = render_forward(**g, cam=c, cfg=cf, parity=True)
    L, p = out["lists"], out["proj"]
    key = (L.tile_of.astype(np.uint64) << np.uint64(32)) | L.depth_bits.astype(np.uint64)
    assert np.all(np.diff(key.astype(np.float64)) >= 0)
    same = np.nonzero(np.diff(key) == 0)[0]
    assert np.all(L.gidx[same] < L.gidx[same + 1])
    box = p["box"].numpy()
    for t in range(L.tiles_x * L.tiles_y):
        s, e = L.ranges[t]
        members = set(L.gidx[s:e].tolist())
        tx, ty = t % L.tiles_x, t // L.tiles_x
        for gg in np.nonzero(p["visible"].numpy())[0]:
            i0, j0, i1, j1 = box[gg]
            overlaps = not (i1 < tx * 8 or i0 > tx * 8 + 7 or j1 < ty * 8 or j0 > ty * 8 + 7)
            assert overlaps == (gg in members)


def test_ambiguity_variants_cover_both_branches():
    # a pixel exactly at the q = 9 boundary: both outcomes are offered
    c = cam(8, 8, f=8.0)
    g = gaussians([[0, 0, 2.0]], [[0.3, 0.3, 0.3]], opacity=0.9, colors=[1, 1, 1], feat=[[1.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=True, amb_delta=(0.3, 1e-5, 1e-5))
    amb = out["ambiguous"].numpy()
    assert amb.any()
    j, i = [int(v[0]) for v in np.nonzero(amb)]
    tile = (j // 8) * out["lists"].tiles_x + i // 8
    vs = pixel_variants(i, j, out["proj"], g["feat"], out["lists"], out["cam"], out["cfg"], out["near"][tile])
    fe = sorted(v[1][0] for v in vs)
    assert fe[0] == 0.0 and fe[-1] > 0.0


def _variants_at(out, g, i, j, tile=8):
    t = (j // tile) * out["lists"].tiles_x + i // tile
    vs = pixel_variants(i, j, out["proj"], g["feat"], out["lists"], out["cam"], out["cfg"], out["near"][t])
    assert vs is not None
    return sorted(vs, key=lambda v: v[2])      # by final transmittance


def test_ambiguity_variants_alpha_branch():
    # alpha exactly at the 1/255 skip threshold (Gaussian centred on pixel
    # (4, 4), opacity 1/255): one outcome includes it, the other skips it
    c = cam(8, 8, f=40.0, cx=4.5, cy=4.5)
    col, fv = [0.8, 0.5, 0.2], [2.0, -1.0]
    g = gaussians([[0, 0, 2.0]], [[0.02, 0.02, 0.02]], opacity=1.0 / 255.0, colors=col, feat=[fv])
    bg = (0.1, 0.2, 0.3)
    out = render_forward(**g, cam=c, cfg=cfg(tile=8, bg=bg), parity=True, amb_delta=(1e-5, 1e-5, 1e-5))
    amb = out["ambiguous"].numpy()
    assert amb[4, 4] and amb.sum() == 1
    near = out["near"][0][2]
    assert near["a"].any() and not near["q"].any() and not near["t"].any()
    vs = _variants_at(out, g, 4, 4)
    assert len(vs) == 2
    a = float(np.float32(1.0 / 255.0))
    # the projected colour (pinned by the SH tests), as the blend sees it
    col32 = out["proj"]["rgb"][0].numpy()
    np.testing.assert_allclose(col32, col, rtol=1e-6)
    bg32 = np.asarray([float(np.float32(b)) for b in bg])
    (r_in, f_in, T_in, n_in, d_in), (r_sk, f_sk, T_sk, n_sk, d_sk) = vs
    np.testing.assert_allclose(r_in, a * col32 + (1 - a) * bg32, rtol=1e-12)
    np.testing.assert_allclose(f_in, a * np.asarray(fv), rtol=1e-12)
    assert abs(T_in - (1 - a)) < 1e-15 and n_in == 1
    np.testing.assert_allclose(r_sk, bg32, rtol=1e-15)
    assert np.all(f_sk == 0) and T_sk == 1.0 and n_sk == 0
    assert abs(d_in - a * 2.0) < 1e-15 and d_sk == 0.0


def test_ambiguity_variants_stop_branch():
    # two Gaussians centred on pixel (4, 4), both clamped at alpha = 0.99:
    # the transmittance after the second is 0.01^2, at the 1e-4 stop
    # threshold; one outcome blends both, the other stops before the second
    c = cam(8, 8, f=40.0, cx=4.5, cy=4.5)
    c1, c2 = [0.9, 0.1, 0.4], [0.2, 0.7, 0.6]
    g = gaussians([[0, 0, 2.0], [0, 0, 2.5]], [[0.05, 0.05, 0.05]], opacity=0.995, colors=[c1, c2],
                  feat=[[1.0, 0.0], [0.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=True, amb_delta=(1e-5, 1e-5, 1e-5))
    amb = out["ambiguous"].numpy()
    assert amb[4, 4] and amb.sum() == 1
    near = out["near"][0][2]
    assert near["t"].any() and not near["a"].any()
    vs = _variants_at(out, g, 4, 4)
    assert len(vs) == 2
    k1, k2 = out["proj"]["rgb"][0].numpy(), out["proj"]["rgb"][1].numpy()
    np.testing.assert_allclose(k1, c1, rtol=1e-6)
    np.testing.assert_allclose(k2, c2, rtol=1e-6)
    a, t1 = 0.99, 1.0 - 0.99
    (r_both, f_both, T_both, n_both, d_both), (r_stop, f_stop, T_stop, n_stop, d_stop) = vs
    np.testing.assert_allclose(r_both, a * k1 + t1 * a * k2, rtol=1e-12)
    np.testing.assert_allclose(f_both, [a, t1 * a], rtol=1e-12)
    assert abs(T_both - t1 * t1) < 1e-18 and n_both == 2
    np.testing.assert_allclose(r_stop, a * k1, rtol=1e-12)
    np.testing.assert_allclose(f_stop, [a, 0.0], rtol=1e-12, atol=0)
    assert abs(T_stop - t1) < 1e-16 and n_stop == 1
    np.testing.assert_allclose([d_both, d_stop], [a * 2.0 + t1 * a * 2.5, a * 2.0], rtol=1e-12)


def test_round_projected_is_one_float32_rounding_with_identity_gradient():
    from oracle.project import round_projected
    rng = np.random.default_rng(3)
    vals = {k: torch.tensor(rng.normal(0, 50, shape), dtype=torch.float64, requires_grad=True)
            for k, shape in (("xy", (7, 2)), ("conic", (7, 3)), ("rgb", (7, 3)), ("depth", (7,)), ("opacity", (7,)))}
    box = torch.tensor(rng.integers(0, 9, (7, 4)))
    p = dict(vals, box=box, n=7)
    r = round_projected(p)
    for k, v in vals.items():
        # numpy's float64 -> float32 cast rounds to nearest, ties to even
        np.testing.assert_array_equal(r[k].detach().numpy(), v.detach().numpy().astype(np.float32).astype(np.float64))
        assert r[k].dtype == torch.float64
    assert r["box"] is box and r["n"] == 7
    w = {k: torch.tensor(rng.normal(size=tuple(v.shape)), dtype=torch.float64) for k, v in vals.items()}
    sum((r[k] * w[k]).sum() for k in vals).backward()
    for k, v in vals.items():
        assert torch.equal(v.grad, w[k])        # the rounding passes gradients through unchanged


def test_equal_depths_blend_in_index_order():
    # two Gaussians at the same depth (identical sort keys) centred on pixel
    # (4, 4): the lower index is in front, rgb = a0 c0 + (1 - a0) a1 c1
    c = cam(8, 8, f=40.0, cx=4.5, cy=4.5)
    c0, c1 = [0.9, 0.2, 0.1], [0.1, 0.3, 0.8]
    g = gaussians([[0, 0, 2.0], [0, 0, 2.0]], [[0.03, 0.03, 0.03], [0.05, 0.05, 0.05]], opacity=[0.6, 0.3],
                  colors=[c0, c1], feat=[[1.0, 0.0], [0.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=True)
    L = out["lists"]
    assert L.gidx.tolist() == [0, 1] and L.depth_bits[0] == L.depth_bits[1]
    k0, k1 = out["proj"]["rgb"][0].numpy(), out["proj"]["rgb"][1].numpy()
    a0, a1 = float(np.float32(0.6)), float(np.float32(0.3))
    np.testing.assert_allclose(out["rgb"][:, 4, 4].numpy(), a0 * k0 + (1 - a0) * a1 * k1, rtol=1e-12)
    np.testing.assert_allclose(out["feat"][:, 4, 4].numpy(), [a0, (1 - a0) * a1], rtol=1e-12)
    # the same scene with the two Gaussians listed the other way round
    gs = {k: v[::-1].copy() for k, v in g.items()}
    out2 = render_forward(**gs, cam=c, cfg=cfg(tile=8), parity=True)
    np.testing.assert_allclose(out2["rgb"][:, 4, 4].numpy(), a1 * k1 + (1 - a1) * a0 * k0, rtol=1e-12)


def test_negative_colour_is_clamped_to_zero():
    # a DC coefficient whose colour Y00 k + 1/2 is negative in one channel:
    # that channel is 0 (colour = max(0, sum k Y + 1/2)), the others unchanged
    c = cam(8, 8, f=40.0, cx=4.5, cy=4.5)
    g = gaussians([[0, 0, 2.0]], [[0.05, 0.05, 0.05]], opacity=0.5, colors=[-0.3, 0.4, 0.7], feat=[[1.0, 1.0]])
    out = render_forward(**g, cam=c, cfg=cfg(tile=8), parity=False)
    col = out["proj"]["rgb"][0].numpy()
    assert col[0] == 0.0
    np.testing.assert_allclose(col[1:], [0.4, 0.7], rtol=1e-6)
    assert float(out["rgb"][0].abs().max()) == 0.0
    a = float(np.float32(0.5))
    np.testing.assert_allclose(out["rgb"][1:, 4, 4].numpy(), a * col[1:], rtol=1e-12)
