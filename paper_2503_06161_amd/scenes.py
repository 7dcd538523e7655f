"""Seeded synthetic scenes shaped like the paper's endoscopic workloads.

This module only draws random inputs; it holds none of the rasterizer's
arithmetic, so both the HIP path and the FP64 oracle can take their inputs
from it.  The activations that the paper leaves to the optimiser (scales are
stored in log space, opacities as logits) are applied here, because the
rasterizer consumes linear scales and opacities in (0, 1).

Five workloads are defined (sizes follow the paper: 640x512 frames (appendix
"Dataset Details", EndoVis18), 128 semantic channels (Sec. 3.2, "Semantic
Feature Extraction"), 30k-90k initial points and
about 1e5 Gaussians in a trained scene (hyper-parameter table)):

* ``small``   128x128, 2,000 Gaussians, SH degree 0, D=8, forward only.
* ``mid``     640x512, 100k Gaussians, SH degree 3, D=32, forward+backward.
* ``metric``  640x512, 300k Gaussians drawn like ``small``, SH degree 3,
              D=128, stored FP32 or BF16.
* ``batched`` 16 timestamps of one deforming scene (eq. 6 stand-in), pool of
              200k Gaussians, 50k-200k visible per frame, D=64 BF16.
* ``large``   1280x1024, 1M Gaussians, SH degree 3, D=128 BF16.

All draws use ``numpy.random.default_rng(seed)`` in float64 in a fixed order
(means, log-scales, quaternions, opacity logits, SH DC, SH rest, features,
upstream gradients) and are then cast to float32.  N(a, b) means mean a and
standard deviation b.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Camera", "Scene", "make_scene", "crop_camera", "bf16_round",
    "WORKLOADS", "batched_frames",
]


@dataclass
class Camera:
    """Pinhole camera; pixel (i, j) samples the point (i + 0.5, j + 0.5)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    # row-major 3x4 world-to-camera [R | t]; identity pose for every workload
    world_to_cam: np.ndarray = field(
        default_factory=lambda: np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], dtype=np.float32))
    near: float = 0.2


@dataclass
class Scene:
    name: str
    cam: Camera
    means: np.ndarray      # [N,3] f32
    scales: np.ndarray     # [N,3] f32, linear
    quats: np.ndarray      # [N,4] f32, (w,x,y,z), unnormalised
    opacity: np.ndarray    # [N]   f32 in (0,1)
    sh: np.ndarray         # [N,(L+1)^2,3] f32
    feat: np.ndarray       # [N,D] f32
    sh_degree: int
    d_rgb: np.ndarray | None = None    # [3,H,W] f32 upstream gradient
    d_feat: np.ndarray | None = None   # [D,H,W] f32 upstream gradient
    tile: tuple[int, int] = (16, 16)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def feat_dim(self) -> int:
        return int(self.feat.shape[1])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them widened back to float32.  NaN stays NaN."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _draw(rng, n, xy, zr, logs, sh_degree, feat_dim, dc=(0.5, 0.2), rest_std=0.05):
    means = np.empty((n, 3))
    means[:, 0] = rng.uniform(-xy, xy, n)
    means[:, 1] = rng.uniform(-xy, xy, n)
    means[:, 2] = rng.uniform(zr[0], zr[1], n)
    log_s = rng.normal(logs[0], logs[1], (n, 3))
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op_logit = rng.normal(0.0, 1.0, n)
    k = (sh_degree + 1) ** 2
    sh = np.zeros((n, k, 3))
    sh[:, 0, :] = rng.normal(dc[0], dc[1], (n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_std, (n, k - 1, 3))
    feat = rng.normal(0.0, 1.0, (n, feat_dim))
    return dict(means=means.astype(np.float32), scales=np.exp(log_s).astype(np.float32),
                quats=q.astype(np.float32), opacity=_sigmoid(op_logit).astype(np.float32),
                sh=sh.astype(np.float32), feat=feat.astype(np.float32))


# name -> (width, height, f, n, xy-range, z-range, log-scale N(mu,sd), sh degree, D, backward?)
WORKLOADS = {
    "small":   dict(w=128, h=128, f=102.4, n=2000, xy=1.0, z=(2.0, 6.0), logs=(-3.5, 0.4), sh=0, d=8, grads=False),
    "mid":     dict(w=640, h=512, f=512.0, n=100_000, xy=1.5, z=(1.0, 8.0), logs=(-4.0, 0.5), sh=3, d=32, grads=True),
    "metric":  dict(w=640, h=512, f=512.0, n=300_000, xy=1.0, z=(2.0, 6.0), logs=(-3.5, 0.4), sh=3, d=128, grads=True),
    "batched": dict(w=640, h=512, f=512.0, n=200_000, xy=1.5, z=(1.0, 8.0), logs=(-4.0, 0.5), sh=3, d=64, grads=True),
    "large":   dict(w=1280, h=1024, f=1024.0, n=1_000_000, xy=2.0, z=(0.5, 10.0), logs=(-4.5, 0.6), sh=3, d=128, grads=True),
}
_SEEDS = {"small": 1, "mid": 2, "metric": 3, "batched": 4, "large": 5}


def make_camera(width, height, f):
    return Camera(width=width, height=height, fx=float(f), fy=float(f), cx=width / 2.0, cy=height / 2.0)


def make_scene(name: str, seed: int | None = None, n: int | None = None, feat_dim: int | None = None,
               sh_degree: int | None = None, width: int | None = None, height: int | None = None,
               f: float | None = None, grads: bool | None = None) -> Scene:
    """Draw one named workload (overrides allow smaller variants of the same
    distributions for tests)."""
    w = dict(WORKLOADS[name])
    seed = _SEEDS[name] if seed is None else seed
    n = w["n"] if n is None else n
    d = w["d"] if feat_dim is None else feat_dim
    L = w["sh"] if sh_degree is None else sh_degree
    W = w["w"] if width is None else width
    H = w["h"] if height is None else height
    fl = w["f"] if f is None else f
    want_g = w["grads"] if grads is None else grads
    rng = np.random.default_rng(seed)
    arrs = _draw(rng, n, w["xy"], w["z"], w["logs"], L, d)
    cam = make_camera(W, H, fl)
    sc = Scene(name=name, cam=cam, sh_degree=L, **arrs)
    if want_g:
        sc.d_rgb = rng.normal(0.0, 1e-3, (3, H, W)).astype(np.float32)
        sc.d_feat = rng.normal(0.0, 1e-3, (d, H, W)).astype(np.float32)
    return sc


def crop_camera(cam: Camera, x0: int, y0: int, w: int, h: int) -> Camera:
    """Sub-window [x0, x0+w) x [y0, y0+h) of ``cam`` as a camera of its own:
    same focal length and pose, principal point shifted into the window."""
    return Camera(width=w, height=h, fx=cam.fx, fy=cam.fy, cx=cam.cx - x0, cy=cam.cy - y0,
                  world_to_cam=cam.world_to_cam.copy(), near=cam.near)


def batched_frames(seed: int = 4, n_frames: int = 16, pool: int = 200_000, base: int = 150_000,
                   n_min: int = 50_000, n_max: int = 200_000, feat_dim: int = 64, amp: float = 0.02):
    """Timestamps t_k = k / n_frames of one deforming scene.

    Frame k renders the first N_k Gaussians of a pool (the first ``base`` are
    the canonical scene), with N_k a seeded permutation of
    round(linspace(n_min, n_max, n_frames)); every mean is offset by
    amp * sin(2 pi t_k + phi) per axis with phi ~ U[0, 2 pi) per Gaussian and
    axis (a synthetic stand-in for the deformation network's output).
    Returns (pool scene, list of per-frame dicts with means and count)."""
    sc = make_scene("batched", seed=seed, n=pool, feat_dim=feat_dim)
    rng = np.random.default_rng(seed + 1000)
    phase = rng.uniform(0.0, 2 * np.pi, (pool, 3))
    counts = np.round(np.linspace(n_min, n_max, n_frames)).astype(np.int64)
    counts = counts[rng.permutation(n_frames)]
    frames = []
    for k in range(n_frames):
        t = k / n_frames
        nk = int(counts[k])
        m = sc.means[:nk].astype(np.float64) + amp * np.sin(2 * np.pi * t + phase[:nk])
        frames.append(dict(t=t, n=nk, means=m.astype(np.float32)))
    return sc, frames


def decoder_inputs(seed: int, feat_dim: int, height: int, width: int, channels: int = 256,
                   target_dtype: str = "f32"):
    """Inputs of the semantic decoder and feature loss (Sec. 3.3, eq. 10):
    a rendered feature map z [D,H,W] ~ N(0, 0.5), the 1x1-convolution weight
    W [C,D] ~ N(0, 1/D) (fan-in scaled) and bias b [C] ~ N(0, 0.1), and a
    stand-in for the segmentation model's feature map t [C,H,W] ~ N(0, 0.5),
    already at the render resolution (the model and its images are not
    available).  Drawn in that order in float64, cast to float32; with
    ``target_dtype="bf16"`` the target is rounded to bfloat16 (returned as
    float32 values that bfloat16 holds exactly)."""
    rng = np.random.default_rng(seed)
    z = rng.normal(0.0, 0.5, (feat_dim, height, width)).astype(np.float32)
    w = (rng.normal(0.0, 1.0, (channels, feat_dim)) / np.sqrt(feat_dim)).astype(np.float32)
    b = rng.normal(0.0, 0.1, channels).astype(np.float32)
    t = rng.normal(0.0, 0.5, (channels, height, width)).astype(np.float32)
    if target_dtype == "bf16":
        t = bf16_round(t)
    return z, w, b, t


DEFORM_PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def deform_inputs(seed: int, n: int, channels: int = 32, width: int = 64, feat_dim: int = 128,
                  base_res=(64, 64, 64, 100), levels=(1, 2, 4, 8), xy: float = 1.0, z=(2.0, 6.0),
                  logs=(-3.5, 0.4)):
    """Inputs of the FST deformation module (Sec. 3.2, eqs. 4-6) with
    synthetic weights (trained ones are not available):

    * canonical Gaussians in the optimiser's parameters: means uniform in
      [-xy, xy]^2 x z, log-scales ~ N(logs), quaternions normalised N(0, I4),
      opacity logits ~ N(0, 1), features [n, feat_dim] ~ N(0, 1);
    * the box [lo, hi] of the means;
    * HexPlane grids: for each level multiplier m and coordinate pair (a, b)
      of (x, y, z, t) in DEFORM_PAIRS order, a [res_b, res_a, channels]
      array (res = base_res[k] m for space, base_res[3] for time), space-only
      planes ~ U(0.1, 0.5), planes with time ~ U(0.5, 1.5);
    * affine layers (weight [out, in], bias [out]) ~ U(-1/sqrt(in),
      1/sqrt(in)): 'out' (4 channels -> width, then 7 x width -> width),
      'branch_<g>' (width -> width -> width/2), 'head_<g>' (width/2 -> d_g,
      d = 3, 4, 3, 1 for mu, rot, scale, opacity), 'sem' (2 width -> width
      -> feat_dim).
    Drawn in that order in float64 and cast to float32."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    means = np.empty((n, 3))
    means[:, 0] = rng.uniform(-xy, xy, n)
    means[:, 1] = rng.uniform(-xy, xy, n)
    means[:, 2] = rng.uniform(z[0], z[1], n)
    log_s = rng.normal(logs[0], logs[1], (n, 3))
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op_logit = rng.normal(0.0, 1.0, n)
    feat = rng.normal(0.0, 1.0, (n, feat_dim))
    lo = np.array([-xy, -xy, z[0]])
    hi = np.array([xy, xy, z[1]])
    planes = []
    for m in levels:
        res = [base_res[k] * m for k in range(3)] + [base_res[3]]
        lvl = []
        for a, b in DEFORM_PAIRS:
            lo_v, hi_v = (0.5, 1.5) if b == 3 else (0.1, 0.5)
            lvl.append(f32(rng.uniform(lo_v, hi_v, (res[b], res[a], channels))))
        planes.append(lvl)

    def affine(n_in, n_out):
        k = 1.0 / np.sqrt(n_in)
        return f32(rng.uniform(-k, k, (n_out, n_in))), f32(rng.uniform(-k, k, n_out))

    layers = {"out": [affine(4 * channels, width)] + [affine(width, width) for _ in range(7)]}
    for g, d in (("mu", 3), ("rot", 4), ("scale", 3), ("opacity", 1)):
        layers["branch_" + g] = (affine(width, width), affine(width, width // 2))
        layers["head_" + g] = affine(width // 2, d)
    layers["sem"] = (affine(2 * width, width), affine(width, feat_dim))
    return dict(means=f32(means), log_scales=f32(log_s), quats=f32(q), logit_opacity=f32(op_logit), feat=f32(feat),
                lo=f32(lo), hi=f32(hi), planes=planes, layers=layers, channels=channels, width=width,
                feat_dim=feat_dim, base_res=tuple(base_res), levels=tuple(levels))
