"""fe_render_backward_noalloc (scratch in the library's per-GPU array)
against fe_render_backward (caller scratch) through the C ABI: two calls in
a row, the second with a smaller input; results must be bit-identical (the
same kernels on the same inputs).  An oversized request is refused before
anything runs."""
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


def _empty_grads(n, K, D):
    return dict(means=torch.full((n, 3), 7.0, device="cuda"), scales=torch.full((n, 3), 7.0, device="cuda"),
                quats=torch.full((n, 4), 7.0, device="cuda"), opacity=torch.full((n,), 7.0, device="cuda"),
                sh=torch.full((n, K, 3), 7.0, device="cuda"), feat=torch.full((n, D), 7.0, device="cuda"))


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_noalloc_backward_equals_backward_twice_second_smaller(dtype):
    sc = make_scene("metric")
    cases = [(crop_camera(sc.cam, 200, 150, 240, 200), sc.n), (crop_camera(sc.cam, 330, 260, 72, 40), 120_000)]
    for k, (cam, n) in enumerate(cases):
        say("noalloc call", k, dtype, "window", cam.width, "x", cam.height, "n", n)
        s2 = make_scene("metric", n=n) if n != sc.n else sc
        s2.cam = cam
        st = U.settings_for(s2, dtype=dtype, variant=rast.FE_VARIANT_MFMA)
        fwd, d = U.gpu_forward(s2, st, cam=cam)
        rng = np.random.default_rng(40 + k)
        d_rgb = torch.from_numpy(rng.normal(0, 1, (3, cam.height, cam.width)).astype(np.float32)).cuda()
        d_feat = torch.from_numpy(rng.normal(0, 1, (128, cam.height, cam.width)).astype(np.float32)).cuda()
        d_depth = torch.from_numpy(rng.normal(0, 1, (cam.height, cam.width)).astype(np.float32)).cuda()
        args = (d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"])
        ref = rast.render_backward(fwd, *args, d_rgb, d_feat, st, d_depth=d_depth)
        K = (s2.sh_degree + 1) ** 2
        got = rast.render_backward_noalloc(fwd, *args, d_rgb, d_feat, st, _empty_grads(n, K, 128), d_depth=d_depth)
        torch.cuda.synchronize()
        for name in U.GRAD_KEYS:
            assert torch.equal(got[name], ref[name]), (k, name)
        if k == 1:
            ob = U.oracle_backward(s2, st, d_rgb.cpu().numpy(), d_feat.cpu().numpy(), cam=cam,
                                   d_depth=d_depth.cpu().numpy())
            U.check_grads(got, ob)


def test_noalloc_refuses_an_oversized_frame():
    say("noalloc: scratch beyond the limit is refused")
    sc = make_scene("metric")
    st = U.settings_for(sc, dtype="bf16", variant=rast.FE_VARIANT_MFMA)
    cam = crop_camera(sc.cam, 300, 240, 32, 32)
    sc.cam = cam
    fwd, d = U.gpu_forward(sc, st, cam=cam)
    st.row_capacity = 2_000_000       # 2M rows of 160 floats: far beyond the array
    args = (d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"])
    z = torch.zeros(3, 32, 32, device="cuda"), torch.zeros(128, 32, 32, device="cuda")
    with pytest.raises(rast.RasterError) as e:
        rast.render_backward_noalloc(fwd, *args, *z, st, _empty_grads(sc.n, 16, 128))
    assert e.value.status == rast.FE_ERR_WORKSPACE_TOO_SMALL
