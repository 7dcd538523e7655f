"""Small hand-built scenes for the oracle pins."""
import numpy as np

from oracle import OracleCamera, OracleConfig


def cam(w=32, h=32, f=32.0, cx=None, cy=None, pose=None, near=0.2):
    c = OracleCamera(w, h, f, f, w / 2 if cx is None else cx, h / 2 if cy is None else cy)
    if pose is not None:
        c.world_to_cam = np.asarray(pose, np.float64)
    c.near = near
    return c


def gaussians(means, scales, quats=None, opacity=None, colors=None, feat=None, sh_degree=0):
    """Build float32 inputs; ``colors`` are target degree-0 colours (the DC
    coefficient is chosen so that max(0, Y00 k + 1/2) = colour)."""
    means = np.atleast_2d(np.asarray(means, np.float32))
    n = means.shape[0]
    scales = np.broadcast_to(np.asarray(scales, np.float32), (n, 3)).copy()
    quats = (np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None
             else np.atleast_2d(np.asarray(quats, np.float32)))
    opacity = (np.full(n, 0.5, np.float32) if opacity is None
               else np.broadcast_to(np.asarray(opacity, np.float32), (n,)).copy())
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3), np.float32)
    if colors is not None:
        y00 = 0.5 / np.sqrt(np.pi)
        sh[:, 0, :] = (np.broadcast_to(np.asarray(colors, np.float64), (n, 3)) - 0.5) / y00
    feat = np.zeros((n, 2), np.float32) if feat is None else np.asarray(feat, np.float32)
    return dict(means=means, scales=scales, quats=quats, opacity=opacity, sh=sh, feat=feat)


def cfg(tile=8, sh_degree=0, **kw):
    return OracleConfig(tile_w=tile, tile_h=tile, sh_degree=sh_degree, **kw)
