"""Pins for the oracle's projection: eq. (2) covariance, quaternion rotation,
the Jacobian of the pinhole map, closed forms of eq. (9), the 3-sigma box,
culling, and pose handling."""
import math

import numpy as np
import torch

from oracle.project import project, quat_to_rot, OracleConfig
from tests.oracle_helpers import cam, gaussians, cfg


def test_quaternion_rotation():
    rng = np.random.default_rng(0)
    q = torch.tensor(rng.normal(size=(100, 4)) * 3.0)
    R = quat_to_rot(q)
    I = torch.eye(3, dtype=R.dtype).expand_as(R)
    assert torch.allclose(R @ R.transpose(1, 2), I, atol=1e-14)
    assert torch.allclose(torch.linalg.det(R), torch.ones(100, dtype=R.dtype), atol=1e-14)
    assert torch.allclose(quat_to_rot(-q), R, atol=1e-15)
    assert torch.allclose(quat_to_rot(torch.tensor([[2.0, 0, 0, 0]], dtype=torch.float64))[0], I[0])
    th = 0.7   # rotation about z by th: (cos th/2, 0, 0, sin th/2)
    Rz = quat_to_rot(torch.tensor([[math.cos(th / 2), 0, 0, math.sin(th / 2)]], dtype=torch.float64))[0]
    expect = torch.tensor([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]],
                          dtype=torch.float64)
    assert torch.allclose(Rz, expect, atol=1e-15)


def _sigma3d(g):
    R = quat_to_rot(torch.tensor(g["quats"], dtype=torch.float64))
    S = torch.diag_embed(torch.tensor(g["scales"], dtype=torch.float64))
    return R @ S @ S @ R.transpose(1, 2)


def test_covariance_eigenvalues_are_squared_scales():
    rng = np.random.default_rng(1)
    g = gaussians(rng.normal(size=(20, 3)), np.abs(rng.normal(size=(20, 3))) + 0.1, quats=rng.normal(size=(20, 4)))
    Sig = _sigma3d(g)
    ev = torch.linalg.eigvalsh(Sig)
    expect = torch.sort(torch.tensor(g["scales"], dtype=torch.float64) ** 2, dim=1).values
    assert torch.allclose(ev, expect, rtol=1e-12, atol=1e-14)


def test_isotropic_on_axis_closed_form():
    # Sigma = s^2 I on the optical axis: Sigma' = (f s / z)^2 I + 0.3 I
    c = cam(64, 64, f=40.0)
    s, z = 0.05, 3.0
    g = gaussians([[0, 0, z]], [s, s, s], quats=[[0.3, -0.2, 0.9, 0.1]])
    p = project(**g, cam=c, cfg=cfg())
    s = float(np.float32(s))
    e = (40.0 * s / z) ** 2 + float(np.float32(0.3))
    np.testing.assert_allclose(p["cov2d"][0].numpy(), [e, 0.0, e], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(p["xy"][0].numpy(), [32.0, 32.0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(p["conic"][0].numpy(), [1 / e, 0, 1 / e], rtol=1e-13, atol=1e-15)


def test_isotropic_off_axis_closed_form():
    # Sigma = s^2 I anywhere: Sigma' = s^2 J J^T + 0.3 I, with
    # J = [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]]
    f, s = 50.0, 0.04
    c = cam(128, 96, f=f, cx=70.0, cy=40.0)
    x, y, z = 0.4, -0.3, 2.5
    g = gaussians([[x, y, z]], [s, s, s])
    p = project(**g, cam=c, cfg=cfg())
    x, y, z = (float(np.float32(v)) for v in (x, y, z))
    s = float(np.float32(s))
    a = s * s * ((f / z) ** 2 + (f * x / z ** 2) ** 2) + float(np.float32(0.3))
    b = s * s * (f * x / z ** 2) * (f * y / z ** 2)
    cc = s * s * ((f / z) ** 2 + (f * y / z ** 2) ** 2) + float(np.float32(0.3))
    np.testing.assert_allclose(p["cov2d"][0].numpy(), [a, b, cc], rtol=1e-12)
    np.testing.assert_allclose(p["xy"][0].numpy(), [f * x / z + 70.0, f * y / z + 40.0], rtol=1e-14)


def test_jacobian_matches_numeric_derivative_of_pinhole_map():
    # Sigma' - 0.3 I = T Sigma T^T with T = J W; J must be the derivative of
    # the pinhole map at the mean (unclamped case)
    rng = np.random.default_rng(2)
    fx = 60.0
    c = cam(200, 160, f=fx, cx=90.0, cy=70.0)
    ang = 0.3
    Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(0.2), -math.sin(0.2)], [0, math.sin(0.2), math.cos(0.2)]])
    Rc = (Rx @ Rz).astype(np.float32).astype(np.float64)
    tc = np.array([0.1, -0.2, 0.5], np.float32).astype(np.float64)
    c.world_to_cam = np.concatenate([Rc, tc[:, None]], 1)
    for _ in range(5):
        mu = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(2, 4)], np.float32)
        q = rng.normal(size=4).astype(np.float32)
        sc = (np.abs(rng.normal(size=3)) * 0.05 + 0.01).astype(np.float32)
        g = gaussians([mu], [sc], quats=[q])
        p = project(**g, cam=c, cfg=OracleConfig(tile_w=8, tile_h=8, sh_degree=0, jacobian_clamp=0.0))

        def pix(m):
            t = Rc @ m + tc
            return np.array([fx * t[0] / t[2] + 90.0, fx * t[1] / t[2] + 70.0])
        m0 = mu.astype(np.float64)
        Jn = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6
            e = np.zeros(3); e[k] = h
            Jn[:, k] = (pix(m0 + e) - pix(m0 - e)) / (2 * h)
        Sig = _sigma3d(g)[0].numpy()
        expect = Jn @ Sig @ Jn.T + 0.3 * np.eye(2)
        got = p["cov2d"][0].numpy()
        dil = float(np.float32(0.3))
        expect = Jn @ Sig @ Jn.T + dil * np.eye(2)
        np.testing.assert_allclose([got[0], got[1], got[2]], [expect[0, 0], expect[0, 1], expect[1, 1]],
                                   rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(p["xy"][0].numpy(), pix(m0), rtol=1e-13)


def test_jacobian_clamp():
    # beyond 1.3 x the half field of view, J is evaluated at the clamped ratio
    f = 32.0
    c = cam(32, 32, f=f)
    lim = 1.3 * 32 / (2 * f)                  # 0.65
    x, z, s = 3.0, 2.0, 0.05                  # x/z = 1.5 > lim
    g = gaussians([[x, 0.0, z]], [s, s, s])
    p = project(**g, cam=c, cfg=cfg())
    s = float(np.float32(s))
    j00, j02, j11 = f / z, -f * float(np.float32(lim)) / z, f / z
    a = s * s * (j00 ** 2 + j02 ** 2) + float(np.float32(0.3))
    np.testing.assert_allclose(p["cov2d"][0, 0].item(), a, rtol=1e-6)
    assert bool(p["xclamped"][0])


def test_box_is_tight_three_sigma_box():
    rng = np.random.default_rng(3)
    c = cam(48, 40, f=40.0)
    n = 40
    mu = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.5, 4, n)], 1)
    g = gaussians(mu, np.exp(rng.normal(-3, 0.5, (n, 3))), quats=rng.normal(size=(n, 4)))
    p = project(**g, cam=c, cfg=cfg())
    ii, jj = np.meshgrid(np.arange(48), np.arange(40), indexing="xy")
    for k in range(n):
        if not bool(p["valid"][k]):
            continue
        u, v = p["xy"][k].numpy()
        A, B, C = p["conic"][k].numpy()
        dx, dy = ii + 0.5 - u, jj + 0.5 - v
        qq = A * dx * dx + 2 * B * dx * dy + C * dy * dy
        i0, j0, i1, j1 = p["box"][k].numpy()
        inside = qq <= 9 * (1 - 1e-9)
        if inside.any():
            assert i0 <= ii[inside].min() and ii[inside].max() <= i1
            assert j0 <= jj[inside].min() and jj[inside].max() <= j1
        # tight: the box edges lie within 3 sigma along each axis
        rx = 3 * math.sqrt(p["cov2d"][k, 0].item())
        if bool(p["visible"][k]):
            for i in (i0, i1):
                assert abs(i + 0.5 - u) <= rx + 1e-9
            if i0 > 0:
                assert abs(i0 - 1 + 0.5 - u) > rx
            if i1 < 47:
                assert abs(i1 + 1 + 0.5 - u) > rx


def test_culling_and_nonfinite():
    c = cam(32, 32, f=32.0)
    g = gaussians([[0, 0, 0.1], [0, 0, 3.0], [np.nan, 0, 3.0], [0, 0, -2.0], [0, 0, 3.0], [30.0, 0, 3.0]],
                  [0.05, 0.05, 0.05], quats=[[1, 0, 0, 0]] * 4 + [[0, 0, 0, 0], [1, 0, 0, 0]])
    p = project(**g, cam=c, cfg=cfg())
    assert p["valid"].tolist() == [False, True, False, False, False, True]
    assert p["nonfinite"].tolist() == [False, False, True, False, True, False]
    assert p["visible"].tolist() == [False, True, False, False, False, False]   # last one is off-screen
    assert p["count"].tolist()[1] >= 1 and p["count"].tolist()[5] == 0


def test_pose_equals_transformed_scene():
    # rendering with pose (R, t) equals rendering the scene moved by (R, t)
    # with the identity pose (degree-0 colour is view independent)
    from oracle import render_forward
    rng = np.random.default_rng(4)
    ang = 0.25
    R = np.array([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0], [-math.sin(ang), 0, math.cos(ang)]])
    t = np.array([0.05, -0.1, 0.3])
    n = 30
    mu = np.stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.4, 0.4, n), rng.uniform(2, 3, n)], 1)
    q = rng.normal(size=(n, 4))
    g = gaussians(mu, np.exp(rng.normal(-2.8, 0.3, (n, 3))), quats=q, opacity=rng.uniform(0.3, 0.9, n),
                  colors=rng.uniform(0.1, 0.9, (n, 3)), feat=rng.normal(size=(n, 3)))
    # exact float64 inputs so that both renders see the same numbers
    c1 = cam(32, 32, f=30.0, pose=np.concatenate([R, t[:, None]], 1))
    c1.world_to_cam = np.concatenate([R, t[:, None]], 1)
    g64 = {k: np.asarray(v, np.float64) for k, v in g.items()}
    o1 = render_forward(**g64, cam=c1, cfg=cfg(), parity=False)
    mu2 = g64["means"] @ R.T + t
    # rotate the quaternions by R: q2 = qR * q
    from scipy.spatial.transform import Rotation
    qr = Rotation.from_matrix(R).as_quat()            # x, y, z, w
    qr = np.array([qr[3], qr[0], qr[1], qr[2]])
    def qmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b.T
        return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)
    g2 = dict(g64, means=mu2, quats=qmul(qr, g64["quats"]))
    o2 = render_forward(**g2, cam=cam(32, 32, f=30.0), cfg=cfg(), parity=False)
    np.testing.assert_allclose(o1["rgb"].numpy(), o2["rgb"].numpy(), atol=1e-9)
    np.testing.assert_allclose(o1["feat"].numpy(), o2["feat"].numpy(), atol=1e-9)


def test_view_dependent_colour_uses_camera_centre():
    # pose built from a chosen camera centre C: t = -R C.  A degree-1 SH with
    # only the Y_1^0 (z) coefficient set gives colour = sqrt(3/4pi) k dz + 1/2
    # with d = normalise(mu - C).
    ang = 0.4
    R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
    C = np.array([0.3, -0.2, -1.0])
    c = cam(32, 32, f=32.0, pose=np.concatenate([R, (-R @ C)[:, None]], 1))
    mu = np.array([[0.1, 0.2, 2.0], [-0.4, 0.1, 3.0]])
    g = gaussians(mu, [0.05, 0.05, 0.05], sh_degree=1)
    g["sh"][:, 2, :] = [0.5, -0.7, 0.9]
    g64 = {k: np.asarray(v, np.float64) for k, v in g.items()}
    p = project(**g64, cam=c, cfg=cfg(sh_degree=1))
    d = g64["means"] - C
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = g64["sh"][:1, 2, :]
    expect = np.maximum(0, math.sqrt(3 / (4 * math.pi)) * d[:, 2:3] * k + 0.5)
    np.testing.assert_allclose(p["rgb"].numpy(), expect, rtol=1e-12)
