"""Pins for the oracle's SH basis (colour model of Sec. 3.1): orthonormality
on the sphere, the addition theorem, and the textbook Cartesian forms of the
real harmonics (no Condon-Shortley phase)."""
import math

import numpy as np
import torch

from oracle.sh import sh_basis


def _sphere_quadrature(nz=24, nphi=48):
    # Gauss-Legendre in z = cos(theta) times the trapezoid rule in phi: exact
    # for polynomials of degree < 2 nz in z and trigonometric degree < nphi.
    z, wz = np.polynomial.legendre.leggauss(nz)
    phi = np.arange(nphi) * 2 * np.pi / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    W = np.outer(wz, np.full(nphi, 2 * np.pi / nphi))
    r = np.sqrt(1 - Z ** 2)
    dirs = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    return torch.tensor(dirs), torch.tensor(W.reshape(-1))


def test_orthonormal_on_sphere():
    dirs, w = _sphere_quadrature()
    Y = sh_basis(dirs, 3)
    G = (Y * w[:, None]).T @ Y
    assert torch.allclose(G, torch.eye(16, dtype=G.dtype), atol=1e-12)


def test_addition_theorem():
    # sum_m Y_l^m(a) Y_l^m(b) = (2l+1)/(4 pi) P_l(a.b): fixes normalisation and
    # rotation invariance independently of the sign convention
    rng = np.random.default_rng(0)
    a = rng.normal(size=(50, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(50, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = sh_basis(torch.tensor(a), 3), sh_basis(torch.tensor(b), 3)
    c = (a * b).sum(1)
    P = [np.ones_like(c), c, 0.5 * (3 * c ** 2 - 1), 0.5 * (5 * c ** 3 - 3 * c)]
    for l in range(4):
        s = (Ya[:, l * l:(l + 1) ** 2] * Yb[:, l * l:(l + 1) ** 2]).sum(1).numpy()
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi) * P[l], atol=1e-13)


def test_textbook_cartesian_forms():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    x, y, z = d.T
    pi = math.pi
    expect = [
        np.full_like(x, 0.5 / math.sqrt(pi)),
        math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x,
        0.5 * math.sqrt(15 / pi) * x * y, 0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (3 * z * z - 1), 0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y), 0.5 * math.sqrt(105 / pi) * x * y * z,
        0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1), 0.25 * math.sqrt(7 / pi) * z * (5 * z * z - 3),
        0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1), 0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
        0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    ]
    Y = sh_basis(torch.tensor(d), 3).numpy()
    np.testing.assert_allclose(Y, np.stack(expect, 1), atol=1e-14)
