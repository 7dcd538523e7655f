"""Pins for the oracle's FST deformation module (Sec. 3.2, eqs. 4-6):
bilinear sampling against torch's grid_sample (align_corners, border) and
against affine planes it must reproduce exactly, grid nodes, the box and time
normalisation, the per-level plane product and level order, the MLP stack
against torch.nn layers assembled from the stated architecture, and the
identity update when the last layers are zero."""
import numpy as np
import pytest
import torch

from oracle import deform as od
from paper_2503_06161_amd.scenes import deform_inputs

SMALL_RES = (5, 6, 7, 4)


def test_bilinear_matches_grid_sample():
    rng = np.random.default_rng(0)
    plane = rng.normal(size=(9, 13, 5))                      # rows = res_b, cols = res_a
    ua = torch.as_tensor(rng.uniform(-1.2, 1.2, 200), dtype=torch.float64)
    ub = torch.as_tensor(rng.uniform(-1.2, 1.2, 200), dtype=torch.float64)
    got = od.bilinear(plane, ua.clamp(-1, 1), ub.clamp(-1, 1))
    inp = torch.as_tensor(plane, dtype=torch.float64).permute(2, 0, 1)[None]
    grid = torch.stack([ua, ub], -1)[None, :, None, :]
    ref = torch.nn.functional.grid_sample(inp, grid, mode="bilinear", padding_mode="border",
                                          align_corners=True)[0, :, :, 0].T
    torch.testing.assert_close(got, ref, rtol=1e-12, atol=1e-12)


def test_bilinear_reproduces_affine_planes_and_nodes():
    rng = np.random.default_rng(1)
    ra, rb, C = 11, 7, 3
    al, be, ga = rng.normal(size=C), rng.normal(size=C), rng.normal(size=C)
    xa = -1 + 2 * np.arange(ra) / (ra - 1)
    yb = -1 + 2 * np.arange(rb) / (rb - 1)
    plane = al + be * xa[None, :, None] + ga * yb[:, None, None]
    ua = torch.as_tensor(rng.uniform(-1, 1, 50), dtype=torch.float64)
    ub = torch.as_tensor(rng.uniform(-1, 1, 50), dtype=torch.float64)
    got = od.bilinear(plane, ua, ub).numpy()
    np.testing.assert_allclose(got, al + be * ua.numpy()[:, None] + ga * ub.numpy()[:, None], rtol=0, atol=1e-12)
    # nodes, including the last row and column
    ii, jj = np.meshgrid(np.arange(ra), np.arange(rb))
    got = od.bilinear(plane, torch.as_tensor(xa[ii.ravel()]), torch.as_tensor(yb[jj.ravel()])).numpy()
    np.testing.assert_allclose(got, plane[jj.ravel(), ii.ravel()], rtol=0, atol=1e-12)


def test_normalized_coords_box_time_and_clamp():
    lo, hi = np.array([-1.0, -2.0, 2.0]), np.array([1.0, 2.0, 6.0])
    means = np.array([[-1.0, -2.0, 2.0], [1.0, 2.0, 6.0], [0.0, 0.0, 4.0], [5.0, -9.0, 4.5]])
    u = od.normalized_coords(means, 0.25, lo, hi).numpy()
    np.testing.assert_allclose(u[:3, :3], [[-1, -1, -1], [1, 1, 1], [0, 0, 0]], atol=0)
    np.testing.assert_allclose(u[3, :3], [1.0, -1.0, 0.25], atol=1e-15)
    assert np.all(u[:, 3] == -0.5)
    assert np.all(od.normalized_coords(means, 1.7, lo, hi).numpy()[:, 3] == 1.0)


def test_resolution_refines_space_not_time():
    assert [od.resolution(m, 0) for m in od.LEVELS] == [64, 128, 256, 512]
    assert [od.resolution(m, 3) for m in od.LEVELS] == [100, 100, 100, 100]


def _planes_const(C, levels=4, value=1.0, res=SMALL_RES):
    out = []
    for m in od.LEVELS[:levels]:
        r = [res[k] * m for k in range(3)] + [res[3]]
        out.append([np.full((r[b], r[a], C), value) for a, b in od.PLANE_PAIRS])
    return out


def test_hexplane_product_and_level_order():
    C = 4
    planes = _planes_const(C)
    consts = {}
    rng = np.random.default_rng(2)
    for li in range(4):
        for p in range(6):
            c = rng.uniform(0.5, 1.5)
            planes[li][p][:] = c
            consts[(li, p)] = c
    # one non-constant plane: level 2, pair (x, t), linear in x
    a, b = od.PLANE_PAIRS[2]
    rb, ra, _ = planes[2][2].shape
    xa = -1 + 2 * np.arange(ra) / (ra - 1)
    planes[2][2] = np.broadcast_to((0.3 + 0.2 * xa)[None, :, None], (rb, ra, C)).copy()
    lo, hi = np.array([-1.0, -1.0, 0.0]), np.array([1.0, 1.0, 4.0])
    means = rng.uniform([-1, -1, 0], [1, 1, 4], (20, 3))
    f = od.hexplane_features(means, 0.3, planes, lo, hi).numpy()
    assert f.shape == (20, 4 * C)
    ux = 2 * (means[:, 0] - lo[0]) / (hi[0] - lo[0]) - 1
    for li in range(4):
        prod = np.prod([consts[(li, p)] for p in range(6)])
        want = np.full(20, prod)
        if li == 2:
            want = want / consts[(2, 2)] * (0.3 + 0.2 * ux)
        np.testing.assert_allclose(f[:, li * C:(li + 1) * C], np.repeat(want[:, None], C, 1), rtol=1e-12)


def test_time_planes_at_one_make_features_time_independent():
    d = deform_inputs(3, 30, channels=4, width=16, feat_dim=8, base_res=SMALL_RES)
    for lvl in d["planes"]:
        for p, (a, b) in enumerate(od.PLANE_PAIRS):
            if b == 3:
                lvl[p][:] = 1.0
    f0 = od.hexplane_features(d["means"], 0.1, d["planes"], d["lo"], d["hi"]).numpy()
    f1 = od.hexplane_features(d["means"], 0.9, d["planes"], d["lo"], d["hi"]).numpy()
    np.testing.assert_allclose(f0, f1, rtol=1e-14, atol=0)   # the weights of a constant plane sum to 1
    # and they do depend on time otherwise
    d2 = deform_inputs(3, 30, channels=4, width=16, feat_dim=8, base_res=SMALL_RES)
    g0 = od.hexplane_features(d2["means"], 0.1, d2["planes"], d2["lo"], d2["hi"]).numpy()
    g1 = od.hexplane_features(d2["means"], 0.9, d2["planes"], d2["lo"], d2["hi"]).numpy()
    assert np.abs(g0 - g1).max() > 1e-3


def _lin(w, b):
    m = torch.nn.Linear(w.shape[1], w.shape[0], dtype=torch.float64)
    with torch.no_grad():
        m.weight.copy_(torch.as_tensor(w, dtype=torch.float64))
        m.bias.copy_(torch.as_tensor(b, dtype=torch.float64))
    return m


def test_mlp_matches_torch_modules():
    W = 16
    d = deform_inputs(4, 25, channels=4, width=W, feat_dim=12, base_res=SMALL_RES)
    L = d["layers"]
    f = torch.as_tensor(np.random.default_rng(5).normal(size=(25, 16)))
    mods = [_lin(*L["out"][0])]
    for layer in L["out"][1:]:
        mods += [torch.nn.ReLU(), _lin(*layer)]
    f_out = torch.nn.Sequential(*mods)
    r = od.deform_mlp(f, L)
    with torch.no_grad():
        h = f_out(f)
        torch.testing.assert_close(r["h"], h, rtol=1e-13, atol=1e-13)
        hs = []
        for g, dg in od.BRANCH_DIMS.items():
            (w1, b1), (w2, b2) = L["branch_" + g]
            feat = torch.nn.Sequential(torch.nn.ReLU(), _lin(w1, b1), torch.nn.ReLU(), _lin(w2, b2))
            head = torch.nn.Sequential(torch.nn.ReLU(), _lin(*L["head_" + g]))
            hg = feat(h)
            assert hg.shape[1] == W // 2
            torch.testing.assert_close(r["h_" + g], hg, rtol=1e-13, atol=1e-13)
            dgv = head(hg)
            assert dgv.shape[1] == dg
            torch.testing.assert_close(r["d_" + g], dgv, rtol=1e-13, atol=1e-13)
            hs.append(hg)
        sem = torch.nn.Sequential(_lin(*L["sem"][0]), torch.nn.ReLU(), _lin(*L["sem"][1]))
        torch.testing.assert_close(r["d_feat"], sem(torch.cat(hs, 1)), rtol=1e-13, atol=1e-13)


def test_zero_last_layers_give_the_canonical_gaussians():
    d = deform_inputs(6, 40, channels=4, width=16, feat_dim=8, base_res=SMALL_RES)
    L = d["layers"]
    for g in od.BRANCHES:
        w, b = L["head_" + g]
        L["head_" + g] = (np.zeros_like(w), np.zeros_like(b))
    w, b = L["sem"][1]
    L["sem"] = (L["sem"][0], (np.zeros_like(w), np.zeros_like(b)))
    params = dict(planes=d["planes"], lo=d["lo"], hi=d["hi"], layers=L)
    out = od.deform_gaussians(d["means"], d["quats"], d["log_scales"], d["logit_opacity"], d["feat"], 0.4, params)
    np.testing.assert_array_equal(out["means"], d["means"].astype(np.float64))
    np.testing.assert_array_equal(out["quats"], d["quats"].astype(np.float64))
    np.testing.assert_allclose(out["scales"], np.exp(d["log_scales"].astype(np.float64)), rtol=1e-15)
    np.testing.assert_allclose(out["opacity"], 1 / (1 + np.exp(-d["logit_opacity"].astype(np.float64))),
                               rtol=1e-15)
    np.testing.assert_array_equal(out["feat"], d["feat"].astype(np.float64))


def test_updates_enter_in_parameter_space():
    d = deform_inputs(7, 30, channels=4, width=16, feat_dim=8, base_res=SMALL_RES)
    params = dict(planes=d["planes"], lo=d["lo"], hi=d["hi"], layers=d["layers"])
    out = od.deform_gaussians(d["means"], d["quats"], d["log_scales"], d["logit_opacity"], d["feat"], 0.7, params)
    np.testing.assert_allclose(np.log(out["scales"]) - d["log_scales"], out["d_scale"], atol=1e-12)
    lg = np.log(out["opacity"] / (1 - out["opacity"]))
    np.testing.assert_allclose(lg - d["logit_opacity"], out["d_opacity"][:, 0], atol=1e-9)
    np.testing.assert_allclose(out["means"] - d["means"], out["d_mu"], atol=1e-12)
    np.testing.assert_allclose(out["quats"] - d["quats"], out["d_rot"], atol=1e-12)
    np.testing.assert_allclose(out["feat"] - d["feat"], out["d_feat"], atol=1e-12)
    assert np.abs(out["d_mu"]).max() > 1e-3 and np.abs(out["d_feat"]).max() > 1e-3


def test_each_plane_samples_its_coordinate_pair():
    """Plane p alone varies (affinely in its two coordinates), the others are
    1: level 0 of f is that affine function of the pair the HexPlane
    assigns to p (written out here, not taken from the oracle)."""
    pairs = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
    rng = np.random.default_rng(8)
    lo, hi = np.array([-1.0, -2.0, 1.0]), np.array([3.0, 2.0, 5.0])
    means = rng.uniform(lo, hi, (15, 3))
    t = 0.35
    u = np.concatenate([2 * (means - lo) / (hi - lo) - 1, np.full((15, 1), 2 * t - 1)], 1)
    for p, (a, b) in enumerate(pairs):
        planes = _planes_const(2, levels=1)
        rb, ra, _ = planes[0][p].shape
        res = [SMALL_RES[k] for k in range(4)]
        assert (ra, rb) == (res[a], res[b])
        xa = -1 + 2 * np.arange(ra) / (ra - 1)
        yb = -1 + 2 * np.arange(rb) / (rb - 1)
        planes[0][p] = np.broadcast_to((0.5 + 0.1 * xa[None, :] + 0.2 * yb[:, None])[:, :, None], (rb, ra, 2)).copy()
        f = od.hexplane_features(means, t, planes, lo, hi).numpy()
        want = 0.5 + 0.1 * u[:, a] + 0.2 * u[:, b]
        np.testing.assert_allclose(f[:, 0], want, rtol=1e-12, err_msg=str((p, a, b)))
