"""Pins for the oracle's gradients: central finite differences of the pure
float64 forward (samples whose discrete trace changes are skipped), and the
identity dL/df_i = sum_p w_i(p) when every feature pixel has upstream
gradient 1 (eq. 8 is linear in the features)."""
import numpy as np
import pytest

from oracle import render_backward, render_forward, fd_gradient, project
from tests.oracle_helpers import cam, gaussians, cfg

GROUPS = ["means", "scales", "quats", "opacity", "sh", "feat"]


def _scene(seed, n=25, w=24, h=24, d=3, L=2, scale=-2.2):
    rng = np.random.default_rng(seed)
    mu = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.5, 3.0, n)], 1)
    g = gaussians(mu, np.exp(rng.normal(scale, 0.3, (n, 3))), quats=rng.normal(size=(n, 4)),
                  opacity=rng.uniform(0.2, 0.95, n), feat=rng.normal(size=(n, d)), sh_degree=L)
    g["sh"][:] = rng.normal(0, 0.4, g["sh"].shape)
    g["sh"][:, 0, :] += 0.3
    c = cam(w, h, f=w * 1.0)
    d_rgb = rng.normal(size=(3, h, w))
    d_feat = rng.normal(size=(d, h, w))
    return {k: np.asarray(v, np.float64) for k, v in g.items()}, c, d_rgb, d_feat


def _check(g, c, cf, d_rgb, d_feat, per_group=12, rtol=1e-5):
    an = render_backward(**g, cam=c, cfg=cf, d_rgb=d_rgb, d_feat=d_feat, parity=False)
    rng = np.random.default_rng(0)
    total_valid = 0
    for name in GROUPS:
        size = g[name].size
        idx = rng.choice(size, size=min(per_group, size), replace=False)
        fd, valid = fd_gradient(g, name, list(idx), c, cf, d_rgb, d_feat)
        a = an[name].reshape(-1)[idx]
        total_valid += valid.sum()
        if valid.any():
            err = np.linalg.norm((fd - a)[valid]) / max(np.linalg.norm(a[valid]), 1e-12)
            assert err < rtol, (name, err)
    return total_valid


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    g, c, d_rgb, d_feat = _scene(seed)
    assert _check(g, c, cfg(tile=8, sh_degree=2, bg=(0.3, 0.2, 0.1)), d_rgb, d_feat) > 50


def test_gradients_through_clamps():
    # opaque, large Gaussians (alpha clamp at 0.99), colours near 0 (colour
    # clamp), and means beyond the Jacobian clamp
    g, c, d_rgb, d_feat = _scene(7, n=20, scale=-1.6)
    g["opacity"][:] = 0.999
    g["sh"][:5, 0, :] = -3.0
    g["means"][:4, 0] = 1.6 * g["means"][:4, 2]
    cf = cfg(tile=8, sh_degree=2)
    p = project(**g, cam=c, cfg=cf)
    assert bool(p["xclamped"][:4].all())
    assert _check(g, c, cf, d_rgb, d_feat) > 40


def test_depth_gradients_match_central_differences():
    # L = <d_depth, depth image> alone: the depth of each Gaussian moves its
    # weighted contribution (and, through J and (u, v), its footprint)
    g, c, d_rgb, d_feat = _scene(4)
    rng = np.random.default_rng(9)
    d_depth = rng.normal(size=(c.height, c.width))
    z_rgb, z_feat = np.zeros_like(d_rgb), np.zeros_like(d_feat)
    cf = cfg(tile=8, sh_degree=2)
    an = render_backward(**g, cam=c, cfg=cf, d_rgb=z_rgb, d_feat=z_feat, d_depth=d_depth, parity=False)
    nvalid = 0
    for name in ("means", "scales", "quats", "opacity"):
        size = g[name].size
        idx = list(rng.choice(size, size=min(16, size), replace=False))
        fd, valid = fd_gradient(g, name, idx, c, cf, z_rgb, z_feat, d_depth=d_depth)
        a = an[name].reshape(-1)[idx]
        nvalid += int(valid.sum())
        assert valid.sum() >= 4, name
        err = np.linalg.norm((fd - a)[valid]) / max(np.linalg.norm(a[valid]), 1e-12)
        assert err < 1e-5, (name, err)
    assert np.abs(an["means"][:, 2]).max() > 0 and np.abs(an["sh"]).max() == 0 and np.abs(an["feat"]).max() == 0
    # the screen-space depth gradient is sum_p w_i(p) d_depth(p)
    out = render_forward(**g, cam=c, cfg=cf, parity=False, keep_weights=True)
    ws = np.zeros(g["means"].shape[0])
    for t, (pi, pj, gi, w, incl) in out["weights"].items():
        np.add.at(ws, gi, (w * d_depth[pj, pi][:, None]).sum(0))
    np.testing.assert_allclose(an["depth2d"], ws, rtol=1e-12, atol=1e-14)


def test_feature_gradient_equals_weight_sum():
    g, c, d_rgb, d_feat = _scene(3, n=40)
    cf = cfg(tile=8, sh_degree=2)
    ones = np.ones_like(d_feat)
    an = render_backward(**g, cam=c, cfg=cf, d_rgb=np.zeros_like(d_rgb), d_feat=ones, parity=False)
    out = render_forward(**g, cam=c, cfg=cf, parity=False, keep_weights=True)
    wsum = np.zeros(g["means"].shape[0])
    for t, (pi, pj, gi, w, incl) in out["weights"].items():
        np.add.at(wsum, gi, w.sum(0))
    for k in range(g["feat"].shape[1]):
        np.testing.assert_allclose(an["feat"][:, k], wsum, rtol=1e-12, atol=1e-15)
