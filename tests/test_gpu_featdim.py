"""Feature widths outside the headline D=128: a single channel, odd widths
(the leftover-channel paths of the row reduction), widths of the paper's
feature-dimension ablation (16 ... 256), and widths above 128 that are not a
multiple of 4, in both variants and both storage forms, forward and
backward, against the FP64 oracle."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import make_scene, crop_camera
from tests import gpu_util as U


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


_METRIC = {}


def _metric_scene(D):
    if D not in _METRIC:
        _METRIC.clear()
        _METRIC[D] = make_scene("metric", feat_dim=D, grads=False)
    import copy
    return copy.copy(_METRIC[D])


def _fwd_bwd(sc, st, cam, seed):
    fwd, d = U.gpu_forward(sc, st, cam=cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    orc = U.oracle_forward(sc, st, cam=cam)
    U.compare_keys(gs, orc)
    say("fwd", U.compare_images(fwd, orc, sc, st))
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    d_rgb = rng.normal(0, 1, (3, H, W)).astype(np.float32)
    d_feat = rng.normal(0, 1, (sc.feat_dim, H, W)).astype(np.float32)
    d_depth = U.depth_grad(H, W, seed, std=1.0)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sc, st, d_rgb, d_feat, cam=cam, d_depth=d_depth)
    U.check_grads(U.screen_grads(gr, sc.n), ob, keys=U.SCREEN_KEYS)
    U.check_grads(gr, ob)


@pytest.mark.parametrize("variant", [rast.FE_VARIANT_VALU, rast.FE_VARIANT_MFMA])
@pytest.mark.parametrize("D", [1, 3, 5, 16, 250, 256])
def test_small_scene_feature_widths(D, variant):
    say("small 96x80 n=600 D", D, "variant", variant)
    sc = make_scene("small", seed=30 + D, n=600, feat_dim=D)
    cam = crop_camera(sc.cam, 16, 24, 96, 80)
    sc.cam = cam
    dtype = "bf16" if D in (3, 250) else "f32"
    st = U.settings_for(sc, dtype=dtype, variant=variant)
    _fwd_bwd(sc, st, cam, seed=D)


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8)])
@pytest.mark.parametrize("D,dtype", [(5, "bf16"), (64, "f32"), (130, "bf16"), (256, "bf16"), (256, "f32")])
def test_metric_window_feature_widths(D, dtype, tile):
    # 48x40 window of the 640x512, 300k-Gaussian workload with D channels
    say("metric window 48x40 D", D, dtype, "tile", tile)
    sc = _metric_scene(D)
    cam = crop_camera(sc.cam, 300, 236, 48, 40)
    sc.cam = cam
    st = U.settings_for(sc, tile=tile, dtype=dtype, variant=rast.FE_VARIANT_MFMA)
    _fwd_bwd(sc, st, cam, seed=100 + D)
