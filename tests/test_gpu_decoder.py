"""Semantic decoder + L1 feature loss (Sec. 3.3, eq. 10) on the GPU against
the FP64 oracle, through the C ABI: the decoded map element by element, the
loss, and every gradient, for D = 32 / 64 / 128, float32 and bfloat16
targets, pixel counts that end in a ragged 32-pixel block, single-pixel and
block-sized maps, exactly zero residuals, the 640x512 D=128 frame, and the
host-side errors.

Error budget (float32 operands split into two bf16 parts, x = hi + lo + e
with |e| <= 2^-18 |x|; products keep hi*hi, hi*lo, lo*hi; sums in float32):
each product is within about 3 * 2^-18 ~ 1.1e-5 of exact, so

* decoded:  |err| <= 2e-5 (|b| + sum_k |W_ck z_k|)
* d_feat:   |err| <= 2e-5 sum_c |W_ck| / P          (signs exact)
* d_weight: |err| <= 2e-5 sum_x |z_k(x)| / P (+ the float32 sum over pixels)
* d_bias:   counts are exact; only the final scaling rounds.

A residual within 3e-5 of that scale of zero decides a sign in float32 on the
GPU: the oracle takes the GPU's sign for exactly those entries (the sign of
the GPU's decoded value minus the target, which is the sign of the float32
difference the kernel forms)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import decoder_inputs

pytestmark = pytest.mark.gpu

AMB_REL = 3e-5


def _run(z, w, b, t, target_dtype):
    dev = "cuda"
    tt = torch.from_numpy(t).to(dev)
    if target_dtype == "bf16":
        tt = tt.to(torch.bfloat16)
    out = rast.decoder_l1(torch.from_numpy(z).to(dev), torch.from_numpy(w).to(dev), torch.from_numpy(b).to(dev),
                          tt.contiguous(), d_feat=True, decoded=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def _compare(z, w, b, t, g, dec_tol=2e-5, dw_tol=2e-5):
    z64, w64, b64, t64 = (a.astype(np.float64) for a in (z, w, b, t))
    D, H, W = z.shape
    P = H * W
    scale = np.abs(b64)[:, None, None] + (np.abs(w64) @ np.abs(z64).reshape(D, P)).reshape(-1, H, W)
    first = oracle.decoder_l1(z64, w64, b64, t64, amb_rel=AMB_REL)
    err = np.abs(g["decoded"] - first["decoded"])
    bad = err > dec_tol * scale
    assert not bad.any(), ("decoded", np.argwhere(bad)[:5], err[bad][:5])
    gpu_sign = np.sign(g["decoded"] - t64)
    ref = oracle.decoder_l1(z64, w64, b64, t64, sign_from=(first["ambiguous"], gpu_sign))
    # loss: |r| summed in float32 over C P terms
    lscale = (scale + np.abs(t64)).sum() / P
    assert abs(g["loss"][0] - ref["loss"]) <= dec_tol * lscale + 1e-6 * ref["loss"], (g["loss"][0], ref["loss"])
    tol_f = 2e-5 * np.abs(w64).sum(0)[:, None, None] / P + 1e-12
    e = np.abs(g["d_feat"] - ref["d_feat"])
    assert (e <= tol_f).all(), ("d_feat", np.argwhere(e > tol_f)[:5], e.max())
    tol_w = dw_tol * np.abs(z64).reshape(D, -1).sum(1)[None, :] / P + 1e-12
    e = np.abs(g["d_weight"] - ref["d_weight"])
    assert (e <= tol_w).all(), ("d_weight", np.argwhere(e > tol_w)[:5], e.max())
    # d_bias: exact counts of the chosen signs, scaled by 1/P in float32
    signs = np.where(first["ambiguous"], gpu_sign, np.sign(first["decoded"] - t64))
    count = (signs != 0).reshape(256, -1).sum(1)
    e = np.abs(g["d_bias"] - ref["d_bias"])
    assert (e <= 1e-6 * (count + 1) / P).all(), ("d_bias", e.max())
    return first["ambiguous"].sum()


@pytest.mark.parametrize("target_dtype", ["f32", "bf16"])
@pytest.mark.parametrize("D", [32, 64, 128])
def test_decoder_matches_oracle(D, target_dtype):
    print(f"decoder D={D} target={target_dtype} 29x37", flush=True)
    z, w, b, t = decoder_inputs(10 + D, D, 29, 37, target_dtype=target_dtype)
    g = _run(z, w, b, t, target_dtype)
    _compare(z, w, b, t, g)


@pytest.mark.parametrize("hw", [(1, 1), (1, 32), (1, 33), (3, 11), (8, 64)])
def test_decoder_small_and_block_edges(hw):
    print(f"decoder edges {hw}", flush=True)
    z, w, b, t = decoder_inputs(3, 32, hw[0], hw[1])
    _compare(z, w, b, t, _run(z, w, b, t, "f32"))


def test_decoder_exact_zero_residuals():
    """Dyadic inputs make every product and sum exact in float32 and in the
    bf16 parts, so the decode is exact; the target equals the decode on a
    third of the entries, whose sign (and subgradient) must be 0."""
    print("decoder exact zero residuals", flush=True)
    rng = np.random.default_rng(7)
    D, H, W = 64, 13, 21
    z = (rng.integers(-16, 17, (D, H, W)) / 8).astype(np.float32)
    w = (rng.integers(-16, 17, (256, D)) / 16).astype(np.float32)
    b = (rng.integers(-32, 33, 256) / 32).astype(np.float32)
    exact = oracle.decoder_l1(z, w, b, np.zeros((256, H, W)))["decoded"]
    t = (rng.integers(-64, 65, (256, H, W)) / 8).astype(np.float64)
    pick = rng.random((256, H, W)) < 1 / 3
    t[pick] = exact[pick]
    t = t.astype(np.float32)
    assert np.array_equal(t[pick].astype(np.float64), exact[pick])
    g = _run(z, w, b, t, "f32")
    np.testing.assert_array_equal(g["decoded"], exact)
    ref = oracle.decoder_l1(z, w, b, t)
    assert (np.sign(ref["decoded"] - t)[pick] == 0).all()
    # the oracle sums terms already divided by P in float64: exact zeros come
    # out as ~1e-17 there, hence the absolute floor
    np.testing.assert_allclose(g["d_bias"], ref["d_bias"], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(g["d_feat"], ref["d_feat"], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(g["d_weight"], ref["d_weight"], rtol=1e-6, atol=1e-14)
    assert abs(g["loss"][0] - ref["loss"]) <= 1e-6 * ref["loss"]


def test_decoder_full_frame():
    """640x512, D = 128, bfloat16 target: the whole map against the oracle."""
    print("decoder 640x512 D=128 bf16 target", flush=True)
    z, w, b, t = decoder_inputs(21, 128, 512, 640, target_dtype="bf16")
    g = _run(z, w, b, t, "bf16")
    n_amb = _compare(z, w, b, t, g, dw_tol=1e-4)
    # |r| ~ N(0, ~0.8) puts about 1e-4 of the entries inside the 3e-5 window
    assert n_amb < 1e-3 * t.size


def test_decoder_loss_autograd_scales_by_upstream():
    print("decoder autograd", flush=True)
    z, w, b, t = decoder_inputs(5, 32, 16, 24)
    dev = "cuda"
    zt = torch.from_numpy(z).to(dev).requires_grad_()
    wt = torch.from_numpy(w).to(dev).requires_grad_()
    bt = torch.from_numpy(b).to(dev).requires_grad_()
    tt = torch.from_numpy(t).to(dev)
    loss = rast.decoder_loss(zt, wt, bt, tt)
    (3.0 * loss).backward()
    direct = rast.decoder_l1(zt.detach(), wt.detach(), bt.detach(), tt)
    torch.cuda.synchronize()
    assert torch.equal(loss.detach(), direct["loss"][0])
    torch.testing.assert_close(zt.grad, 3.0 * direct["d_feat"], rtol=0, atol=0)
    torch.testing.assert_close(wt.grad, 3.0 * direct["d_weight"], rtol=0, atol=0)
    torch.testing.assert_close(bt.grad, 3.0 * direct["d_bias"], rtol=0, atol=0)


def test_decoder_host_errors():
    print("decoder host errors", flush=True)
    dev = "cuda"
    z = torch.zeros(16, 4, 4, device=dev)
    with pytest.raises(rast.RasterError) as e:
        rast.decoder_l1(z, torch.zeros(256, 16, device=dev), torch.zeros(256, device=dev),
                        torch.zeros(256, 4, 4, device=dev))
    assert e.value.status == rast.FE_ERR_UNSUPPORTED
    z = torch.zeros(32, 4, 4, device=dev)
    ws = torch.empty(256, dtype=torch.uint8, device=dev)
    with pytest.raises(rast.RasterError) as e:
        rast.decoder_l1(z, torch.zeros(256, 32, device=dev), torch.zeros(256, device=dev),
                        torch.zeros(256, 4, 4, device=dev), workspace=ws)
    assert e.value.status == rast.FE_ERR_WORKSPACE_TOO_SMALL
