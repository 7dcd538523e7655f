"""Semantic decoder and feature loss in float64 (Sec. 3.3, eq. 10).

Test infrastructure only (see the package docstring).

The rendered feature map z (D channels per pixel) goes through a pointwise
(1x1) convolution to the C channels of the segmentation model's features,
z'(x) = W z(x) + b, and is compared with the target features by a per-pixel
L1 norm averaged over the H x W pixels:

    L_feat = (1 / HW) sum_x || z'(x) - t(x) ||_1

Readings (the paper does not fix them): the target map is given at the
render resolution H x W (the segmentation model's coarser map resized by the
caller), and the L1 subgradient at a zero residual is 0.  With r = z' - t and
s = sign(r) / HW the gradients are

    dL/dz(x) = W^T s(x),   dL/dW = sum_x s(x) z(x)^T,   dL/db = sum_x s(x).

A residual near 0 decides a sign: ``sign_from`` lets the caller supply the
sign of chosen entries (taken by the implementation under test in its own
precision); every other sign is the float64 one.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def decoder_l1(feat, weight, bias, target, sign_from=None, amb_rel=0.0):
    """feat [D, H, W], weight [C, D], bias [C], target [C, H, W] (any float
    arrays).  Returns float64 numpy arrays: loss (scalar), decoded [C, H, W],
    d_feat [D, H, W], d_weight [C, D], d_bias [C], and ``ambiguous`` [C, H, W]:
    residuals within amb_rel * (|b| + sum_k |W_ck z_k| + |t|) of zero.
    ``sign_from`` (optional (mask, signs)) overrides the sign where mask is
    set."""
    z = torch.as_tensor(np.asarray(feat), dtype=F64)
    D, H, W_ = z.shape
    Wt = torch.as_tensor(np.asarray(weight), dtype=F64)
    b = torch.as_tensor(np.asarray(bias), dtype=F64)
    t = torch.as_tensor(np.asarray(target), dtype=F64)
    C = Wt.shape[0]
    P = H * W_
    zf = z.reshape(D, P)
    dec = Wt @ zf + b[:, None]                       # the pointwise convolution
    r = dec - t.reshape(C, P)
    loss = r.abs().sum() / P                         # eq. (10)
    sg = torch.sign(r)
    scale = b.abs()[:, None] + Wt.abs() @ zf.abs() + t.reshape(C, P).abs()
    amb = r.abs() <= amb_rel * scale
    if sign_from is not None:
        mask, signs = sign_from
        mask = torch.as_tensor(np.asarray(mask)).reshape(C, P)
        signs = torch.as_tensor(np.asarray(signs), dtype=F64).reshape(C, P)
        sg = torch.where(mask, signs, sg)
        loss = (sg * r).sum() / P                    # |r| with the chosen signs
    s = sg / P
    return dict(loss=float(loss), decoded=dec.reshape(C, H, W_).numpy(),
                d_feat=(Wt.T @ s).reshape(D, H, W_).numpy(), d_weight=(s @ zf.T).numpy(),
                d_bias=s.sum(1).numpy(), ambiguous=amb.reshape(C, H, W_).numpy())
