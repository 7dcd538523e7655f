"""torch.autograd.Function wiring, and the GPU gradients against FP64 central
finite differences of the oracle on the 64-Gaussian 32x32 window of the
640x512, 300k-Gaussian, D=128 workload (both storage forms); the loss takes
the colour, feature and depth images."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import make_scene, crop_camera, bf16_round
import oracle
from tests import gpu_util as U


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


def _window_scene():
    """The 32x32 window [304,336)x[240,272) of the metric camera and the first
    64 Gaussians (by index) whose 3-sigma box meets it."""
    sc = make_scene("metric")
    cam = crop_camera(sc.cam, 304, 240, 32, 32)
    p = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, sc.sh, cam,
                       oracle.OracleConfig(tile_w=16, tile_h=16, sh_degree=3))
    idx = np.nonzero(p["visible"].numpy())[0][:64]
    sub = make_scene("metric", n=1, grads=False)
    for k in ("means", "scales", "quats", "opacity", "sh", "feat"):
        setattr(sub, k, np.ascontiguousarray(getattr(sc, k)[idx]))
    sub.cam = cam
    rng = np.random.default_rng(21)
    sub.d_rgb = rng.normal(0, 1, (3, 32, 32)).astype(np.float32)
    sub.d_feat = rng.normal(0, 1, (128, 32, 32)).astype(np.float32)
    sub.d_depth = rng.normal(0, 1, (32, 32)).astype(np.float32)
    return sub


def test_autograd_function_matches_c_abi():
    say("autograd wiring")
    sc = _window_scene()
    st = U.settings_for(sc, dtype="bf16")
    d = U.to_device(sc, "bf16")
    leaves = {k: d[k].clone().requires_grad_(True) for k in ("means", "scales", "quats", "opacity")}
    sh = d["sh"].clone().requires_grad_(True)
    ft = d["feat"].clone().requires_grad_(True)
    rgb, feat, depth, T, n = rast.rasterize(leaves["means"], leaves["scales"], leaves["quats"], leaves["opacity"],
                                            sh, ft, sc.cam, st)
    assert not T.requires_grad and not n.requires_grad and depth.requires_grad
    g_rgb, g_feat = torch.from_numpy(sc.d_rgb).cuda(), torch.from_numpy(sc.d_feat).cuda()
    g_depth = torch.from_numpy(sc.d_depth).cuda()
    ((rgb * g_rgb).sum() + (feat * g_feat).sum() + (depth * g_depth).sum()).backward()
    fwd = rast.render_forward(d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"], sc.cam, st)
    ref = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                               g_rgb, g_feat, st, d_depth=g_depth)
    for k in ("means", "scales", "quats", "opacity"):
        torch.testing.assert_close(leaves[k].grad, ref[k], rtol=1e-5, atol=1e-7)
    assert sh.grad.dtype == torch.bfloat16 and ft.grad.dtype == torch.bfloat16
    torch.testing.assert_close(ft.grad.float(), ref["feat"].bfloat16().float())


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_gradients_vs_fp64_finite_differences(dtype):
    say("FD window 64 Gaussians 32x32 D=128", dtype)
    sc = _window_scene()
    st = U.settings_for(sc, dtype=dtype)
    fwd, d = U.gpu_forward(sc, st, cam=sc.cam)
    gr = rast.render_backward(fwd, d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"],
                              torch.from_numpy(sc.d_rgb).cuda(), torch.from_numpy(sc.d_feat).cuda(), st,
                              d_depth=torch.from_numpy(sc.d_depth).cuda())
    torch.cuda.synchronize()
    inp = U.stored_inputs(sc, dtype)
    params = {k: np.asarray(v, np.float64) for k, v in inp.items()}
    cfg = U.oracle_cfg(sc, st)
    rng = np.random.default_rng(0)
    nvalid = 0
    for name in ("means", "scales", "quats", "opacity", "sh", "feat"):
        flat = params[name].reshape(-1)
        idx = list(rng.choice(flat.size, size=min(24, flat.size), replace=False))
        fd, valid = oracle.fd_gradient(params, name, idx, sc.cam, cfg, sc.d_rgb, sc.d_feat, d_depth=sc.d_depth)
        g = gr[name].cpu().numpy().reshape(-1)[idx]
        nvalid += int(valid.sum())
        # every group needs enough samples whose discrete trace is unchanged at x +- h
        assert valid.sum() >= 4, (name, int(valid.sum()))
        err = np.linalg.norm((g - fd)[valid]) / max(np.linalg.norm(fd[valid]), 1e-30)
        say(name, "valid", int(valid.sum()), "normwise", err)
        assert err < 1e-4, (name, err)
    assert nvalid >= 48
