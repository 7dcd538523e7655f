"""FST deformation module (Sec. 3.2, eqs. 4-6) on the GPU against the FP64
oracle, through the C ABI: G_t (means, quaternions, scales, opacity,
features) for HexPlane widths 32 and 64 at the paper's grid sizes, a ragged
last workgroup, single-Gaussian and empty inputs, Gaussians outside the box,
t at both ends of [0, 1], bf16 feature output, and the host-side errors.

Error budget: the HexPlane runs in float32 from float64 weights (relative
error ~1e-6 of f); every affine layer multiplies two-part bf16 splits of
activations and weights (each product within ~3 * 2^-18 ~ 1.1e-5 of exact)
and sums in float32; 11 layers sit between f and the deepest output.  The
bound applied is |gpu - oracle| <= 2e-4 * max|update| per output group
(the update is the MLP's output for that group; the inputs pass through
exactly), plus the float32 rounding of the result itself."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import deform_inputs

pytestmark = pytest.mark.gpu

REL = 2e-4
_NETS = {}


def _inputs(C, n, seed=11):
    key = (C, n, seed)
    if key not in _NETS:
        d = deform_inputs(seed, n, channels=C)
        net = rast.DeformNet(d["planes"], d["layers"], d["lo"], d["hi"], C, 64, 128)
        _NETS.clear()
        _NETS[key] = (d, net)
    return _NETS[key]


def _run(d, net, t, n=None, out_feat_dtype="f32"):
    n = d["means"].shape[0] if n is None else n
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a[:n])).cuda()
    out = rast.deform_forward(net, T(d["means"]), T(d["quats"]), T(d["log_scales"]), T(d["logit_opacity"]),
                              T(d["feat"]), t, out_feat_dtype=out_feat_dtype)
    torch.cuda.synchronize()
    return {k: v.float().cpu().numpy().astype(np.float64) for k, v in out.items()}


def _oracle(d, t, n=None):
    n = d["means"].shape[0] if n is None else n
    params = dict(planes=d["planes"], lo=d["lo"], hi=d["hi"], layers=d["layers"])
    return oracle.deform_gaussians(d["means"][:n], d["quats"][:n], d["log_scales"][:n], d["logit_opacity"][:n],
                                   d["feat"][:n], t, params)


def _check(g, o, feat_rel=0.0):
    f32 = np.finfo(np.float32).eps
    pairs = (("means", "d_mu"), ("quats", "d_rot"), ("feat", "d_feat"))
    for k, dk in pairs:
        tol = REL * np.abs(o[dk]).max() + f32 * np.abs(o[k]) + feat_rel * np.abs(o[k])
        err = np.abs(g[k] - o[k])
        assert (err <= tol).all(), (k, err.max(), np.argwhere(err > tol)[:4])
    # scales = exp(log s + ds): relative error of the update carried through exp
    tol = (REL * np.abs(o["d_scale"]).max() + 4 * f32) * o["scales"]
    err = np.abs(g["scales"] - o["scales"])
    assert (err <= tol).all(), ("scales", err.max())
    op = o["opacity"]
    tol = (REL * np.abs(o["d_opacity"]).max() + 4 * f32) * op * (1 - op) + f32 * op
    err = np.abs(g["opacity"] - op)
    assert (err <= tol).all(), ("opacity", err.max())


@pytest.mark.parametrize("C", [32, 64])
def test_deform_matches_oracle(C):
    print(f"deform C={C} n=1000", flush=True)
    d, net = _inputs(C, 1000)
    for t in (0.0, 0.37, 1.0):
        _check(_run(d, net, t), _oracle(d, t))


def test_deform_edges_and_outside_box():
    print("deform edges", flush=True)
    d, net = _inputs(32, 1000)
    d = dict(d)
    means = d["means"].copy()
    means[:7] = [[-3.0, 0.0, 4.0], [3.0, 0.5, 4.0], [0.0, -2.0, 1.0], [0.2, 2.0, 7.0], [5.0, 5.0, 9.0],
                 [-5.0, -5.0, 0.0], [1.0, 1.0, 6.0]]
    d["means"] = means
    for n in (1, 63, 64, 65):
        _check(_run(d, net, 0.5, n=n), _oracle(d, 0.5, n=n))
    empty = _run(d, net, 0.5, n=0)
    assert all(v.size == 0 for v in empty.values())


def test_deform_bf16_features():
    print("deform bf16 feature output", flush=True)
    d, net = _inputs(32, 1000)
    g = _run(d, net, 0.25, out_feat_dtype="bf16")
    # bf16 rounding of the result: half an ulp, 2^-9 relative
    _check(g, _oracle(d, 0.25), feat_rel=2.0 ** -8)


def test_deform_host_errors():
    print("deform host errors", flush=True)
    d, net = _inputs(32, 1000)
    bad = rast.fe_deform_net.from_buffer_copy(net.net)
    bad.width = 32
    lib = rast.load_library()
    assert lib.fe_deform_workspace_bytes(rast.C.byref(bad)) == 0
    io = rast.fe_deform_io()
    io.n = 1
    st = lib.fe_deform_forward(rast.C.byref(bad), rast.C.byref(io), rast.C.c_void_p(net.workspace.data_ptr()),
                               net.workspace.numel(), None)
    assert st == rast.FE_ERR_UNSUPPORTED
    st = lib.fe_deform_forward(rast.C.byref(net.net), rast.C.byref(io), rast.C.c_void_p(net.workspace.data_ptr()),
                               16, None)
    assert st == rast.FE_ERR_WORKSPACE_TOO_SMALL
    box = rast.fe_deform_net.from_buffer_copy(net.net)
    box.hi[0] = box.lo[0]
    st = lib.fe_deform_forward(rast.C.byref(box), rast.C.byref(io), rast.C.c_void_p(net.workspace.data_ptr()),
                               net.workspace.numel(), None)
    assert st == rast.FE_ERR_INVALID_ARG
