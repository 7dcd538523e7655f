"""Real spherical harmonics up to any degree, from their definition.

Test infrastructure only (see the package docstring).

The paper stores view-dependent colour as SH coefficients per Gaussian
(Sec. 3.1, parameter list after eq. 2) without fixing a basis.  The reading
used here: the real, orthonormal basis without the Condon-Shortley phase,

    Y_l^m  = sqrt(2) K_l^m  dP_l^m(z) Re((x + i y)^m)     for m > 0
    Y_l^0  =         K_l^0  P_l(z)
    Y_l^-m = sqrt(2) K_l^m  dP_l^m(z) Im((x + i y)^m)     for m > 0

with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and dP_l^m the m-th
derivative of the Legendre polynomial P_l (so that
(1-z^2)^(m/2) dP_l^m(z) cos(m phi) = dP_l^m(z) Re((x+iy)^m) on the unit
sphere).  Coefficient index l^2 + l + m for m = -l..l.
"""
from __future__ import annotations

import math
import numpy as np
import torch


def sh_coeff_count(degree: int) -> int:
    return (degree + 1) ** 2


def _legendre_coeffs(l: int) -> np.ndarray:
    """Power-series coefficients of P_l via Bonnet's recurrence
    (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1}."""
    p_prev = np.zeros(l + 1)
    p_prev[0] = 1.0
    if l == 0:
        return p_prev
    p = np.zeros(l + 1)
    p[1] = 1.0
    for n in range(1, l):
        nxt = np.zeros(l + 1)
        nxt[1:] += (2 * n + 1) * p[:-1]
        nxt -= n * p_prev
        nxt /= n + 1
        p_prev, p = p, nxt
    return p


def _poly_eval(coeffs: np.ndarray, z: torch.Tensor) -> torch.Tensor:
    out = torch.zeros_like(z)
    for c in coeffs[::-1]:
        out = out * z + float(c)
    return out


def sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Evaluate the basis at unit vectors ``dirs`` [..., 3] (float64).

    Returns [..., (degree+1)^2].  Differentiable (used by the autograd
    backward of the colour)."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    out = []
    # powers of (x + i y) as (re, im)
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    for l in range(degree + 1):
        pl = _legendre_coeffs(l)
        row = [None] * (2 * l + 1)
        for m in range(0, l + 1):
            dp = np.polynomial.polynomial.polyder(pl, m) if m > 0 else pl
            k = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            pz = _poly_eval(np.atleast_1d(dp), z)
            if m == 0:
                row[l] = k * pz
            else:
                row[l + m] = math.sqrt(2.0) * k * pz * re[m]
                row[l - m] = math.sqrt(2.0) * k * pz * im[m]
        out.extend(row)
    return torch.stack(out, dim=-1)
