"""Per-Gaussian projection in float64 (eqs. 2 and 9).

Test infrastructure only (see the package docstring).

For each Gaussian: camera-space centre t = W mu + t_c; rotation from the
normalised quaternion; Sigma = R diag(s^2) R^T (eq. 2); the affine
(Jacobian) approximation of the perspective map J at t and
Sigma' = J W Sigma W^T J^T (eq. 9) plus a small dilation of the diagonal;
the conic Sigma'^-1; the pixel position; a 3-sigma pixel box; and the view
dependent colour from SH coefficients.

Readings of points the paper leaves open (they are the same for the HIP
path, which is written independently):
* pixel (i, j) samples (i + 0.5, j + 0.5); u = fx (tx / tz) + cx;
* cull when tz <= near, when any of mean / scale / quaternion / opacity is
  not finite (these are counted), or when det Sigma' <= 0;
* J uses x~ = clamp(tx / tz, +-lim_x) with lim_x = k W / (2 fx), k = 1.3
  (0 disables the clamp); likewise for y;
* Sigma'_xx and Sigma'_yy gain +0.3 px^2 (dilation);
* box: i in [ceil(u - 3 sqrt(Sigma'_xx) - 1/2), floor(u + 3 sqrt(Sigma'_xx) - 1/2)]
  clipped to the image, likewise for j; a Gaussian whose box is empty emits
  nothing;
* colour = max(0, sum_k sh_k Y_k(dir) + 1/2), dir = normalise(mu - campos).

Every quantity that decides a sort key or a box (tz, u, v, Sigma'_xx,
Sigma'_yy) is evaluated as separate correctly rounded float64 operations in
the order written below, with no fused multiply-add, so that any other
implementation evaluating the same expressions in the same order obtains the
same bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np
import torch

from .sh import sh_basis

F64 = torch.float64


@dataclass
class OracleCamera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray = field(
        default_factory=lambda: np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], dtype=np.float64))
    near: float = 0.2

    @staticmethod
    def from_any(cam) -> "OracleCamera":
        # camera parameters cross the boundary as float32
        f32 = lambda v: float(np.float32(v))
        return OracleCamera(int(cam.width), int(cam.height), f32(cam.fx), f32(cam.fy), f32(cam.cx),
                            f32(cam.cy), np.asarray(cam.world_to_cam, np.float32).astype(np.float64),
                            f32(cam.near))


@dataclass
class OracleConfig:
    tile_w: int = 16
    tile_h: int = 16
    sh_degree: int = 3
    bg: tuple = (0.0, 0.0, 0.0)
    dilation: float = 0.3
    jacobian_clamp: float = 1.3

    def f32(self):
        """Scalar parameters cross the boundary as float32."""
        c = OracleConfig(**self.__dict__)
        c.bg = tuple(float(np.float32(b)) for b in self.bg)
        c.dilation = float(np.float32(self.dilation))
        c.jacobian_clamp = float(np.float32(self.jacobian_clamp))
        return c


def _t(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x if x.dtype == F64 else x.to(F64)
    return torch.as_tensor(np.asarray(x), dtype=F64)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the normalised quaternion (w, x, y, z), [N,3,3]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    n = torch.sqrt(((w * w + x * x) + y * y) + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    r = torch.stack([
        1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
        2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x),
        2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y),
    ], dim=-1)
    return r.reshape(-1, 3, 3)


def project(means, scales, quats, opacity, sh, cam, cfg: OracleConfig, sh_degree: int | None = None, feat=None):
    """Project Gaussians.  Inputs may be numpy arrays or float64 tensors (the
    latter keep autograd; ``feat`` is accepted and ignored).  Returns a dict of float64 tensors plus integer
    boxes / tile rectangles and masks."""
    cam = cam if isinstance(cam, OracleCamera) else OracleCamera.from_any(cam)
    cfg = cfg.f32()
    L = cfg.sh_degree if sh_degree is None else sh_degree
    mu, s, q, op, shc = _t(means), _t(scales), _t(quats), _t(opacity), _t(sh)
    n = mu.shape[0]
    Rc = torch.as_tensor(cam.world_to_cam[:, :3], dtype=F64)
    tc = torch.as_tensor(cam.world_to_cam[:, 3], dtype=F64)
    x, y, z = mu[:, 0], mu[:, 1], mu[:, 2]
    cam_t = [((Rc[i, 0] * x + Rc[i, 1] * y) + Rc[i, 2] * z) + tc[i] for i in range(3)]
    tx, ty, tz = cam_t

    finite = (torch.isfinite(mu).all(1) & torch.isfinite(s).all(1) & torch.isfinite(q).all(1)
              & torch.isfinite(op))
    qn2 = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
    finite = finite & (qn2.detach() > 0)
    in_front = tz.detach() > cam.near

    # guard the arithmetic of culled Gaussians so that no NaN reaches autograd
    ok = finite & in_front
    okf = ok.to(F64)
    safe_q = torch.where(ok[:, None], q, torch.tensor([1.0, 0, 0, 0], dtype=F64).expand_as(q))
    safe_s = torch.where(ok[:, None], s, torch.zeros_like(s))
    safe_tz = torch.where(ok, tz, torch.ones_like(tz))
    safe_tx = torch.where(ok, tx, torch.zeros_like(tx))
    safe_ty = torch.where(ok, ty, torch.zeros_like(ty))

    R = quat_to_rot(safe_q)
    M = R * safe_s[:, None, :]                       # M_ak = R_ak s_k
    Sig = [[(M[:, a, 0] * M[:, b, 0] + M[:, a, 1] * M[:, b, 1]) + M[:, a, 2] * M[:, b, 2]
            for b in range(3)] for a in range(3)]      # eq. (2)

    fx, fy = cam.fx, cam.fy
    xr = safe_tx / safe_tz
    yr = safe_ty / safe_tz
    if cfg.jacobian_clamp > 0:
        limx = (cfg.jacobian_clamp * cam.width) / (2.0 * fx)
        limy = (cfg.jacobian_clamp * cam.height) / (2.0 * fy)
        xc = torch.clamp(xr, -limx, limx)
        yc = torch.clamp(yr, -limy, limy)
        jclamped = (xr.detach().abs() > limx) | (yr.detach().abs() > limy)
    else:
        xc, yc = xr, yr
        jclamped = torch.zeros(n, dtype=torch.bool)
    j00 = fx / safe_tz
    j02 = (-fx * xc) / safe_tz
    j11 = fy / safe_tz
    j12 = (-fy * yc) / safe_tz
    # Tm = J W   (2x3)
    Tm0 = [j00 * Rc[0, k] + j02 * Rc[2, k] for k in range(3)]
    Tm1 = [j11 * Rc[1, k] + j12 * Rc[2, k] for k in range(3)]
    Tm = [Tm0, Tm1]
    # U = Tm Sigma ; Sigma' = U Tm^T   (eq. 9)
    U = [[(Tm[a][0] * Sig[0][b] + Tm[a][1] * Sig[1][b]) + Tm[a][2] * Sig[2][b] for b in range(3)]
         for a in range(2)]
    c2 = [[(U[a][0] * Tm[b][0] + U[a][1] * Tm[b][1]) + U[a][2] * Tm[b][2] for b in range(2)]
          for a in range(2)]
    ca = c2[0][0] + cfg.dilation
    cb = c2[0][1]
    cc = c2[1][1] + cfg.dilation
    det = ca * cc - cb * cb
    det_ok = torch.isfinite(det.detach()) & (det.detach() > 0)
    ok = ok & det_ok
    safe_det = torch.where(ok, det, torch.ones_like(det))
    conic = torch.stack([cc / safe_det, -cb / safe_det, ca / safe_det], dim=-1)

    u = fx * xr + cam.cx
    v = fy * yr + cam.cy

    # 3-sigma pixel box (decided on detached float64 values)
    with torch.no_grad():
        rx = 3.0 * torch.sqrt(torch.clamp(ca, min=0.0))
        ry = 3.0 * torch.sqrt(torch.clamp(cc, min=0.0))
        i0 = torch.ceil((u - rx) - 0.5)
        i1 = torch.floor((u + rx) - 0.5)
        j0 = torch.ceil((v - ry) - 0.5)
        j1 = torch.floor((v + ry) - 0.5)
        big = 1e9
        i0 = torch.clamp(torch.nan_to_num(i0, nan=big), -big, big).to(torch.int64).clamp(min=0)
        j0 = torch.clamp(torch.nan_to_num(j0, nan=big), -big, big).to(torch.int64).clamp(min=0)
        i1 = torch.clamp(torch.nan_to_num(i1, nan=-big), -big, big).to(torch.int64).clamp(max=cam.width - 1)
        j1 = torch.clamp(torch.nan_to_num(j1, nan=-big), -big, big).to(torch.int64).clamp(max=cam.height - 1)
        nonempty = (i0 <= i1) & (j0 <= j1)
        vis = ok & nonempty
        tw, th = cfg.tile_w, cfg.tile_h
        tx0 = torch.where(vis, i0 // tw, torch.zeros_like(i0))
        tx1 = torch.where(vis, i1 // tw, -torch.ones_like(i1))
        ty0 = torch.where(vis, j0 // th, torch.zeros_like(j0))
        ty1 = torch.where(vis, j1 // th, -torch.ones_like(j1))
        count = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
        count = torch.where(vis, count, torch.zeros_like(count))

    # view-dependent colour
    campos = [-((Rc[0, k] * tc[0] + Rc[1, k] * tc[1]) + Rc[2, k] * tc[2]) for k in range(3)]
    d = torch.stack([x - campos[0], y - campos[1], z - campos[2]], dim=-1)
    d = torch.where(ok[:, None], d, torch.tensor([0.0, 0.0, 1.0], dtype=F64).expand_as(d))
    dn = torch.sqrt(((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]))
    dirs = d / dn[:, None]
    kk = (L + 1) ** 2
    Y = sh_basis(dirs, L)                            # [N, K]
    shk = torch.where(ok[:, None, None], shc[:, :kk, :], torch.zeros_like(shc[:, :kk, :]))
    raw = (Y[:, :, None] * shk).sum(1) + 0.5        # [N, 3]
    rgb = torch.clamp(raw, min=0.0)

    return dict(
        n=n, tx=tx, ty=ty, tz=tz, u=u, v=v, xy=torch.stack([u, v], -1), cov2d=torch.stack([ca, cb, cc], -1),
        conic=conic, opacity=op, rgb=rgb, rgb_raw=raw, depth=tz,
        box=torch.stack([i0, j0, i1, j1], -1), rect=torch.stack([tx0, ty0, tx1, ty1], -1), count=count,
        visible=vis, valid=ok, nonfinite=~finite, xclamped=jclamped,
        okf=okf,
    )


def round_projected(p: dict, to=torch.float32) -> dict:
    """Round the projected record to float32 once (the precision boundary of
    the GPU path); gradients pass through the rounding unchanged.

    The rounding is added as a constant (detached) correction, so its
    derivative is exactly the identity: a plain dtype cast would also round
    the incoming gradient to float32 on the way back."""
    out = dict(p)
    for k in ("xy", "conic", "rgb", "depth", "opacity"):
        x = p[k]
        out[k] = x + (x.detach().to(to).to(F64) - x.detach())
    return out
