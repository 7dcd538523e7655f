"""HIP path vs the FP64 oracle, through the C ABI, on seeded workloads:
projected record, sort keys (bit-exact), images (normwise 1e-5 with
near-threshold acceptance), gradients (normwise 1e-4), both storage forms,
several tile shapes, ragged image sizes, and the edge cases."""
import sys

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


def _subset_scene(sc, cam):
    """Same Gaussians, another camera (a window of the original)."""
    import copy
    s2 = copy.copy(sc)
    s2.cam = cam
    return s2


VARIANTS = [rast.FE_VARIANT_VALU, rast.FE_VARIANT_MFMA]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8)])
def test_small_forward_keys_and_images(tile, variant):
    say("small 128x128 n=2000 D=8 tile", tile, "variant", variant)
    sc = make_scene("small")
    st = U.settings_for(sc, tile=tile, variant=variant)
    fwd, _ = U.gpu_forward(sc, st)
    gs = U.read_state(fwd, sc.n, st, sc.cam)
    orc = U.oracle_forward(sc, st)
    nv = U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    stats = U.compare_images(fwd, orc, sc, st)
    say("visible", nv, "keys", orc["lists"].k, stats)


@pytest.mark.parametrize("variant", VARIANTS)
def test_gpu_images_independent_of_tile_shape(variant):
    say("small: tile-shape invariance, variant", variant)
    sc = make_scene("small")
    outs = [U.gpu_forward(sc, U.settings_for(sc, tile=t, variant=variant))[0]
            for t in ((16, 16), (8, 8), (32, 8), (8, 16))]
    for o in outs[1:]:
        assert torch.equal(o.rgb, outs[0].rgb)
        assert torch.equal(o.final_T, outs[0].final_T)
        if variant == rast.FE_VARIANT_VALU:
            assert torch.equal(o.feat, outs[0].feat)
        else:
            # the matrix cores sum each 16-Gaussian batch in their own order: equal to rounding
            torch.testing.assert_close(o.feat, outs[0].feat, rtol=0, atol=2e-6)


def test_forward_is_deterministic():
    say("mid: forward twice")
    sc = make_scene("mid")
    st = U.settings_for(sc)
    a, d = U.gpu_forward(sc, st)
    r1, f1 = a.rgb.clone(), a.feat.clone()
    b, _ = U.gpu_forward(sc, st, dev_in=d)
    assert torch.equal(r1, b.rgb) and torch.equal(f1, b.feat)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_mid_window_forward_backward(dtype, variant):
    # ragged 100x76 window of the 640x512 mid workload: 7x5 tiles, partial edges
    say("mid window 100x76 D=32 SH3", dtype, "variant", variant)
    sc = make_scene("mid")
    cam = crop_camera(sc.cam, 250, 200, 100, 76)
    sw = _subset_scene(sc, cam)
    st = U.settings_for(sc, dtype=dtype, variant=variant)
    fwd, d = U.gpu_forward(sw, st, cam=cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    orc = U.oracle_forward(sw, st, cam=cam)
    U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    stats = U.compare_images(fwd, orc, sw, st)
    say("fwd", stats)
    rng = np.random.default_rng(11)
    d_rgb = rng.normal(0, 1e-3, (3, 76, 100)).astype(np.float32)
    d_feat = rng.normal(0, 1e-3, (32, 76, 100)).astype(np.float32)
    d_depth = U.depth_grad(76, 100, 11)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sw, st, d_rgb, d_feat, cam=cam, d_depth=d_depth)
    U.check_grads(U.screen_grads(gr, sc.n), ob, keys=U.SCREEN_KEYS)
    U.check_grads(gr, ob)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_metric_window_d128(dtype, variant):
    # 64x48 window of the 640x512, 300k-Gaussian, D=128 workload
    say("metric window 64x48 D=128", dtype, "variant", variant)
    sc = make_scene("metric")
    cam = crop_camera(sc.cam, 290, 230, 64, 48)
    sw = _subset_scene(sc, cam)
    st = U.settings_for(sc, dtype=dtype, variant=variant)
    fwd, d = U.gpu_forward(sw, st, cam=cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    orc = U.oracle_forward(sw, st, cam=cam)
    U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    say("fwd", U.compare_images(fwd, orc, sw, st))
    rng = np.random.default_rng(12)
    d_rgb = rng.normal(0, 1e-3, (3, 48, 64)).astype(np.float32)
    d_feat = rng.normal(0, 1e-3, (128, 48, 64)).astype(np.float32)
    d_depth = U.depth_grad(48, 64, 12)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sw, st, d_rgb, d_feat, cam=cam, d_depth=d_depth)
    U.check_grads(U.screen_grads(gr, sc.n), ob, keys=U.SCREEN_KEYS)
    U.check_grads(gr, ob)


@pytest.mark.parametrize("tile,threads", [((16, 16), 256), ((16, 16), 512), ((16, 8), 128), ((16, 8), 256),
                                          ((8, 8), 64), ((8, 8), 128)])
def test_threads_per_tile(tile, threads):
    # one thread per pixel (single-role kernels) or two (wave-specialized),
    # 56x40 window of the metric workload, D = 128 BF16, against the oracle
    say("metric window 56x40 D=128 bf16 tile", tile, "threads per tile", threads)
    sc = make_scene("metric")
    cam = crop_camera(sc.cam, 292, 232, 56, 40)
    sw = _subset_scene(sc, cam)
    st = U.settings_for(sc, tile=tile, dtype="bf16", variant=rast.FE_VARIANT_MFMA, threads_per_tile=threads)
    fwd, d = U.gpu_forward(sw, st, cam=cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    orc = U.oracle_forward(sw, st, cam=cam)
    U.compare_keys(gs, orc)
    say("fwd", U.compare_images(fwd, orc, sw, st))
    rng = np.random.default_rng(13)
    d_rgb = rng.normal(0, 1, (3, 40, 56)).astype(np.float32)
    d_feat = rng.normal(0, 1, (128, 40, 56)).astype(np.float32)
    d_depth = U.depth_grad(40, 56, 13)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sw, st, d_rgb, d_feat, cam=cam, d_depth=d_depth)
    U.check_grads(U.screen_grads(gr, sc.n), ob, keys=U.SCREEN_KEYS)
    U.check_grads(gr, ob)

