"""Edge cases of the HIP path through the C ABI: empty and culled inputs,
non-finite parameters, key and row capacity overflow (reported, never
silently truncated), images smaller than a tile, a single tile, and ragged
sizes; each is compared with the FP64 oracle."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import make_scene, crop_camera, Camera
from tests import gpu_util as U


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


def _small(n=300, seed=7, **kw):
    return make_scene("small", seed=seed, n=n, **kw)


VARIANTS = [rast.FE_VARIANT_VALU, rast.FE_VARIANT_MFMA]


@pytest.mark.parametrize("variant", VARIANTS)
def test_zero_gaussians_renders_background(variant):
    say("n=0", variant)
    sc = _small(n=0)
    st = U.settings_for(sc, variant=variant, bg=(0.25, 0.5, 0.75))
    fwd, d = U.gpu_forward(sc, st)
    assert torch.allclose(fwd.rgb[0], torch.full_like(fwd.rgb[0], 0.25))
    assert torch.allclose(fwd.rgb[2], torch.full_like(fwd.rgb[2], 0.75))
    assert float(fwd.feat.abs().max()) == 0.0 and float(fwd.final_T.min()) == 1.0
    assert fwd.report["keys_needed"] == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_all_culled_and_nonfinite_counted(variant):
    say("culled + non-finite", variant)
    sc = _small(n=200)
    sc.means[:, 2] = -1.0                # all behind the camera
    sc.means[:10, 0] = np.nan            # ten non-finite
    sc.quats[10:15] = 0.0                # five zero quaternions
    st = U.settings_for(sc, variant=variant)
    fwd, d = U.gpu_forward(sc, st)
    assert fwd.report["n_culled_nonfinite"] == 15
    assert fwd.report["n_visible"] == 0 and fwd.report["keys_needed"] == 0
    assert float(fwd.final_T.min()) == 1.0
    g = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                             torch.ones(3, sc.cam.height, sc.cam.width, device="cuda"),
                             torch.ones(sc.feat_dim, sc.cam.height, sc.cam.width, device="cuda"), st)
    for k in ("means", "scales", "quats", "opacity", "sh", "feat"):
        assert float(g[k].abs().max()) == 0.0, k


@pytest.mark.parametrize("variant", VARIANTS)
def test_key_overflow_is_reported_not_truncated(variant):
    say("key overflow", variant)
    sc = _small(n=500)
    st = U.settings_for(sc, variant=variant, key_capacity=100)
    with pytest.raises(rast.RasterError) as e:
        U.gpu_forward(sc, st)
    assert e.value.status == rast.FE_ERR_KEY_OVERFLOW
    # automatic capacity grows and renders the right image
    st2 = U.settings_for(sc, variant=variant)
    fwd, _ = U.gpu_forward(sc, st2)
    orc = U.oracle_forward(sc, st2)
    U.compare_images(fwd, orc, sc, st2)


def test_row_overflow_is_reported():
    say("row overflow")
    sc = _small(n=500, grads=True)
    st = U.settings_for(sc, variant=rast.FE_VARIANT_MFMA, row_capacity=3)
    fwd, d = U.gpu_forward(sc, st)
    args = (d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"])
    rng = np.random.default_rng(8)
    d_rgb = rng.normal(0, 1, (3, 128, 128)).astype(np.float32)
    d_feat = rng.normal(0, 1, (sc.feat_dim, 128, 128)).astype(np.float32)
    gd_rgb, gd_feat = torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda()
    with pytest.raises(rast.RasterError) as e:
        rast.render_backward(fwd, *args, gd_rgb, gd_feat, st)
    assert e.value.status == rast.FE_ERR_ROW_OVERFLOW
    rep = rast.read_report(fwd.state)
    assert rep["backward_status"] == rast.FE_ERR_ROW_OVERFLOW and rep["rows_needed"] > 3
    # a second backward of the same forward state with enough rows clears the
    # status and returns the oracle's gradients
    st.row_capacity = None
    gr = rast.render_backward(fwd, *args, gd_rgb, gd_feat, st)
    rep = rast.read_report(fwd.state)
    assert rep["status"] == 0 and rep["backward_status"] == 0
    ob = U.oracle_backward(sc, st, d_rgb, d_feat)
    U.check_grads(gr, ob)


@pytest.mark.parametrize("cap_extra", [0, 1, 3])
def test_tiny_key_capacity_with_dirty_scratch(cap_extra):
    # key_capacity 1..4 (the frame's exact need plus a little) and a scratch
    # buffer filled with 0xFF: the backward must clear every row index it reads
    say("tiny key capacity, dirty scratch, cap_extra", cap_extra)
    sc = make_scene("small", seed=21, n=1, grads=True)
    sc.means[0] = (0.0, 0.0, 4.0)
    sc.scales[0] = (0.06, 0.035, 0.045)          # anisotropic and rotated: every group has a gradient
    sc.quats[0] = (0.9, 0.2, -0.3, 0.25)
    cam = crop_camera(sc.cam, 56, 56, 16, 16)        # one tile, the Gaussian in the middle
    sc.cam = cam
    st = U.settings_for(sc, variant=rast.FE_VARIANT_MFMA)
    fwd, d = U.gpu_forward(sc, st, cam=cam)
    need = int(fwd.report["keys_needed"])
    assert need == 1
    st.key_capacity = need + cap_extra
    fwd, d = U.gpu_forward(sc, st, cam=cam, dev_in=d)
    rng = np.random.default_rng(9)
    d_rgb = rng.normal(0, 1, (3, 16, 16)).astype(np.float32)
    d_feat = rng.normal(0, 1, (sc.feat_dim, 16, 16)).astype(np.float32)
    cfg = rast.fe_config.from_buffer_copy(fwd.cfg)
    nbytes = rast.load_library().fe_backward_scratch_bytes(rast.C.byref(cfg), rast.C.byref(fwd.cam), sc.n)
    scratch = torch.full((nbytes,), 255, dtype=torch.uint8, device="cuda")
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st, scratch=scratch)
    torch.cuda.synchronize()
    ob = U.oracle_backward(sc, st, d_rgb, d_feat, cam=cam)
    U.check_grads(gr, ob)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("wh", [(5, 3), (16, 16), (21, 9), (70, 33), (200, 8)])
def test_ragged_and_tiny_images(wh, variant):
    # images smaller than one tile, exactly one tile, ragged tails, and a
    # strip one tile high (the backward's tile order then skips its Z order)
    w, h = wh
    say("image", wh, "variant", variant)
    sc = _small(n=400, seed=11, grads=True)
    cam = crop_camera(sc.cam, 64 - w // 2, 64 - h // 2, w, h)
    sc.cam = cam
    st = U.settings_for(sc, variant=variant)
    fwd, d = U.gpu_forward(sc, st, cam=cam)
    orc = U.oracle_forward(sc, st, cam=cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    U.compare_keys(gs, orc)
    U.compare_images(fwd, orc, sc, st)
    rng = np.random.default_rng(3)
    d_rgb = rng.normal(0, 1, (3, h, w)).astype(np.float32)
    d_feat = rng.normal(0, 1, (sc.feat_dim, h, w)).astype(np.float32)
    d_depth = U.depth_grad(h, w, 3, std=1.0)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(d_rgb).cuda(), torch.from_numpy(d_feat).cuda(), st,
                              d_depth=torch.from_numpy(d_depth).cuda())
    torch.cuda.synchronize()
    ob = U.oracle_backward(sc, st, d_rgb, d_feat, cam=cam, d_depth=d_depth)
    U.check_grads(gr, ob)


def test_invalid_arguments_return_status():
    say("invalid arguments")
    sc = _small(n=10)
    st = U.settings_for(sc, tile=(16, 5))
    with pytest.raises(rast.RasterError) as e:
        U.gpu_forward(sc, st)
    assert e.value.status == rast.FE_ERR_UNSUPPORTED
    d = U.to_device(sc)
    bad_sh = torch.zeros(sc.n * 3 + 1, device="cuda")[1:].view(sc.n, 1, 3)   # misaligned start
    st2 = U.settings_for(sc)
    with pytest.raises(rast.RasterError) as e:
        rast.render_forward(d["means"], d["scales"], d["quats"], d["opacity"], bad_sh, d["feat"], sc.cam, st2)
    assert e.value.status == rast.FE_ERR_INVALID_ARG
