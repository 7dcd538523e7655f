"""Whole frames at the workload sizes, in the launch configuration the
benchmark times (16x16 tiles, matrix-core variant), against the FP64 oracle:

* the 640x512, 300k-Gaussian, D=128 BF16 frame of the headline metric:
  projected record, every sort key, every pixel, all six gradient groups and
  the screen-space sums, and the backward's row count;
* the 640x512, 100k-Gaussian, D=32 FP32 frame, the same checks;
* the 1280x1024, 1M-Gaussian, D=128 BF16 frame with the sort buffer sized for
  8 tile overlaps per Gaussian: no overflow, every key bit-exact, images on
  sampled tiles, and gradients with the upstream gradient restricted to those
  tiles (every other tile then contributes exactly zero, so the whole-frame
  backward must equal the oracle's backward over the sampled tiles)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import make_scene
from tests import gpu_util as U


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


def _tile_walks(n_contrib, tw, th):
    H, W = n_contrib.shape
    ty, tx = -(-H // th), -(-W // tw)
    x = np.zeros((ty * th, tx * tw), np.int64)
    x[:H, :W] = n_contrib
    return x.reshape(ty, th, tx, tw).max(axis=(1, 3)).reshape(-1)


def _whole_frame(sc, dtype):
    st = U.settings_for(sc, dtype=dtype, variant=rast.FE_VARIANT_MFMA)
    fwd, d = U.gpu_forward(sc, st)
    gs = U.read_state(fwd, sc.n, st, sc.cam)
    orc = U.oracle_forward(sc, st)
    nv = U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    stats = U.compare_images(fwd, orc, sc, st)
    say("visible", nv, "keys", orc["lists"].k, stats)
    # the backward's partial rows: one per (tile, list position) walked, the
    # walk of a tile being its largest n_contrib (compared with the oracle above)
    walks = _tile_walks(fwd.n_contrib.cpu().numpy(), st.tile_w, st.tile_h)
    assert fwd.report["rows_needed"] == int(walks.sum())
    d_depth = U.depth_grad(sc.cam.height, sc.cam.width, 1)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(sc.d_rgb).cuda(), torch.from_numpy(sc.d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sc, st, sc.d_rgb, sc.d_feat, d_depth=d_depth)
    U.check_grads(U.screen_grads(gr, sc.n), ob, keys=U.SCREEN_KEYS)
    U.check_grads(gr, ob)


def test_metric_whole_frame_bf16():
    say("whole metric frame: 640x512, 300k Gaussians, D=128, BF16, 16x16 tiles")
    _whole_frame(make_scene("metric"), "bf16")


def test_mid_whole_frame_f32():
    say("whole mid frame: 640x512, 100k Gaussians, D=32, SH 3, FP32")
    _whole_frame(make_scene("mid"), "f32")


def test_large_frame_capacity_8n_sampled_tiles():
    say("large frame: 1280x1024, 1M Gaussians, D=128, BF16, key capacity 8N")
    sc = make_scene("large")
    st = U.settings_for(sc, dtype="bf16", variant=rast.FE_VARIANT_MFMA, key_capacity=8 * sc.n)
    fwd, d = U.gpu_forward(sc, st)
    assert fwd.report["status"] == 0 and fwd.report["keys_needed"] <= 8 * sc.n
    gs = U.read_state(fwd, sc.n, st, sc.cam)
    tiles_x, tiles_y = -(-sc.cam.width // 16), -(-sc.cam.height // 16)
    rng = np.random.default_rng(55)
    sample = sorted(rng.choice(tiles_x * tiles_y, size=24, replace=False).tolist())
    orc = U.oracle_forward(sc, st, tiles=sample)
    nv = U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    stats = U.compare_images(fwd, orc, sc, st, tiles=sample)
    say("visible", nv, "keys", orc["lists"].k, "sampled tiles", stats)
    # upstream gradients only inside the sampled tiles
    mask = np.zeros((sc.cam.height, sc.cam.width), np.float32)
    for t in sample:
        x0, y0 = (t % tiles_x) * 16, (t // tiles_x) * 16
        mask[y0:y0 + 16, x0:x0 + 16] = 1.0
    d_rgb = (sc.d_rgb * mask).astype(np.float32)
    d_feat = (sc.d_feat * mask).astype(np.float32)
    d_depth = (U.depth_grad(sc.cam.height, sc.cam.width, 2) * mask).astype(np.float32)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sc, st, d_rgb, d_feat, tiles=sample, d_depth=d_depth)
    U.check_grads(gr, ob)
