"""Autotuner: every candidate renders the same image, and the choice is
cached and reused."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast, autotune
from paper_2503_06161_amd.scenes import make_scene, crop_camera
from tests import gpu_util as U


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


def test_candidates_agree_and_choice_is_cached(tmp_path, monkeypatch):
    print("[case] autotune window of mid", flush=True)
    monkeypatch.setenv("FE4DGS_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    sc = make_scene("mid")
    cam = crop_camera(sc.cam, 250, 200, 96, 64)
    d = U.to_device(sc, "bf16")
    st = rast.Settings(sh_degree=3, feat_dim=32, sh_dtype="bf16", feat_dtype="bf16")
    ref = None
    cands = autotune.candidates_for(st, cam, sc.n)
    # both thread counts are offered where the two-per-pixel kernels exist
    assert (8, 8, rast.FE_VARIANT_MFMA, 64) in cands and (8, 8, rast.FE_VARIANT_MFMA, 128) in cands
    assert (16, 16, rast.FE_VARIANT_MFMA, 256) in cands and (16, 16, rast.FE_VARIANT_MFMA, 0) in cands
    assert (16, 16, rast.FE_VARIANT_MFMA, 512) in cands          # D = 32 through the 128-channel kernel
    assert (16, 16, rast.FE_VARIANT_VALU, 512) not in cands and (16, 16, rast.FE_VARIANT_VALU, 256) in cands
    for tw, th, v, tpt in cands:
        s2 = rast.Settings(**{**st.__dict__, "tile_w": tw, "tile_h": th, "variant": v, "threads_per_tile": tpt})
        f = rast.render_forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"], cam, s2)
        if ref is None:
            ref = f
        # the transmittance chain is bit-identical in every form (n_contrib is a
        # position in the tile's list, so it depends on the tile shape); the
        # wave-specialized forward sums colour and features on the matrix cores
        # (each product exact, float32 sums in the hardware's order), so those
        # agree with the vector-ALU sums to rounding
        assert torch.equal(f.final_T, ref.final_T)
        torch.testing.assert_close(f.rgb, ref.rgb, rtol=0, atol=2e-6)
        torch.testing.assert_close(f.feat, ref.feat, rtol=0, atol=2e-6)
    g_rgb = torch.zeros(3, 64, 96, device="cuda")
    g_feat = torch.full((32, 64, 96), 1e-3, device="cuda")
    best = autotune.autotune(d, cam, st, g_rgb, g_feat, verbose=True)
    assert (best.tile_w, best.tile_h) in autotune.TILE_SHAPES
    again = autotune.autotune(d, cam, st, g_rgb, g_feat, candidates=[(8, 8, rast.FE_VARIANT_VALU, 64)])
    assert ((again.tile_w, again.tile_h, again.variant, again.threads_per_tile)
            == (best.tile_w, best.tile_h, best.variant, best.threads_per_tile))
