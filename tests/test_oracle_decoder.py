"""Pins for the oracle's decoder and feature loss (Sec. 3.3, eq. 10): central
finite differences of the loss for every parameter group, the identity
decoder (closed form), a perfect fit (zero loss and zero subgradient),
positive homogeneity, invariance under pixel permutation and under tiling
the image (mean over pixels), and the sign override of near-zero residuals."""
import numpy as np
import pytest

from oracle import decoder_l1


def _case(seed, D=5, C=7, H=3, W=4):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(D, H, W)), rng.normal(size=(C, D)) / np.sqrt(D), rng.normal(size=C) * 0.1,
            rng.normal(size=(C, H, W)))


def _loss(z, Wt, b, t):
    return decoder_l1(z, Wt, b, t)["loss"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradients_match_central_differences(seed):
    z, Wt, b, t = _case(seed)
    out = decoder_l1(z, Wt, b, t)
    h = 1e-6
    for name, arr, grad in (("feat", z, out["d_feat"]), ("weight", Wt, out["d_weight"]), ("bias", b, out["d_bias"])):
        flat = arr.reshape(-1)
        for i in range(flat.size):
            x0 = flat[i]
            flat[i] = x0 + h
            lp = _loss(z, Wt, b, t)
            flat[i] = x0 - h
            lm = _loss(z, Wt, b, t)
            flat[i] = x0
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad.reshape(-1)[i]) < 1e-7 * max(1.0, abs(fd)), (name, i, fd, grad.reshape(-1)[i])


def test_identity_decoder_closed_form():
    rng = np.random.default_rng(4)
    z = rng.normal(size=(6, 4, 5))
    out = decoder_l1(z, np.eye(6), np.zeros(6), np.zeros((6, 4, 5)))
    assert abs(out["loss"] - np.abs(z).sum() / 20) < 1e-14
    np.testing.assert_array_equal(out["d_feat"], np.sign(z) / 20)
    np.testing.assert_allclose(out["decoded"], z, rtol=0, atol=0)


def test_perfect_fit_has_zero_loss_and_subgradient():
    z, Wt, b, _ = _case(5)
    t = np.einsum("cd,dhw->chw", Wt, z) + b[:, None, None]
    out = decoder_l1(z, Wt, b, t)
    assert out["loss"] < 1e-14
    # residuals are zero up to rounding: the ones exactly zero give 0
    r = out["decoded"] - t
    assert np.all(out["d_bias"][np.all(r == 0, axis=(1, 2))] == 0)


def test_positive_homogeneity_and_pixel_mean():
    z, Wt, b, t = _case(6)
    base = decoder_l1(z, Wt, b, t)["loss"]
    assert abs(decoder_l1(z, 2.5 * Wt, 2.5 * b, 2.5 * t)["loss"] - 2.5 * base) < 1e-12
    # the image tiled twice along each axis: same mean over pixels
    z4, t4 = np.tile(z, (1, 2, 2)), np.tile(t, (1, 2, 2))
    assert abs(decoder_l1(z4, Wt, b, t4)["loss"] - base) < 1e-12
    # a permutation of the pixels: same loss, permuted feature gradient
    perm = np.random.default_rng(7).permutation(z.shape[1] * z.shape[2])
    zp = z.reshape(z.shape[0], -1)[:, perm].reshape(z.shape)
    tp = t.reshape(t.shape[0], -1)[:, perm].reshape(t.shape)
    o1, o2 = decoder_l1(z, Wt, b, t), decoder_l1(zp, Wt, b, tp)
    assert abs(o1["loss"] - o2["loss"]) < 1e-12
    np.testing.assert_allclose(o2["d_feat"].reshape(z.shape[0], -1), o1["d_feat"].reshape(z.shape[0], -1)[:, perm],
                               atol=1e-15)
    np.testing.assert_allclose(o2["d_weight"], o1["d_weight"], atol=1e-14)


def test_near_zero_residuals_are_flagged_and_their_sign_can_be_chosen():
    z, Wt, b, t = _case(8, D=3, C=2, H=2, W=2)
    dec = np.einsum("cd,dhw->chw", Wt, z) + b[:, None, None]
    t = t.copy()
    t[1, 0, 1] = dec[1, 0, 1] + 1e-12          # a residual of -1e-12
    out = decoder_l1(z, Wt, b, t, amb_rel=1e-9)
    assert out["ambiguous"][1, 0, 1] and out["ambiguous"].sum() == 1
    mask = out["ambiguous"]
    flip = decoder_l1(z, Wt, b, t, sign_from=(mask, np.ones_like(t)), amb_rel=1e-9)
    # the residual's sign goes from -1 to +1: every gradient moves by 2/HW times its factor
    P = 4
    np.testing.assert_allclose(flip["d_bias"] - out["d_bias"], [0.0, 2.0 / P], atol=1e-15)
    np.testing.assert_allclose(flip["d_weight"][1] - out["d_weight"][1], 2.0 / P * z[:, 0, 1], atol=1e-15)
    np.testing.assert_allclose(flip["d_feat"][:, 0, 1] - out["d_feat"][:, 0, 1], 2.0 / P * Wt[1], atol=1e-15)
    assert abs(flip["loss"] - out["loss"]) < 1e-11
