"""The C-ABI library loads and exports every symbol the header declares;
host-only entry points (validation, state layout) behave as documented.
No compute call is made (these run without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fe4dgs_rast.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fe_render_forward", "fe_render_backward", "fe_state_bytes", "fe_read_report",
                 "fe_batch_plan_create", "fe_batch_launch", "fe_validate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2503_06161_amd import rast
    lib = rast.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", rast.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fe_[a-z0-9_]+)", out))
    assert set(_declared()) <= exported
    assert set(rast.EXPORTS) == set(_declared())


def _cfg(**kw):
    from paper_2503_06161_amd import rast
    st = rast.Settings(sh_degree=kw.pop("sh_degree", 3), feat_dim=kw.pop("feat_dim", 32))
    for k, v in kw.items():
        setattr(st, k, v)
    return st


def _cam(w=640, h=512):
    from paper_2503_06161_amd.scenes import make_camera
    return make_camera(w, h, 512.0)


def test_validate_and_state_layout():
    from paper_2503_06161_amd import rast
    lib = rast.load_library()
    cam = rast.camera_c(_cam())
    ok = _cfg().to_c(1 << 20)
    assert lib.fe_validate(C.byref(ok), C.byref(cam), 1000) == rast.FE_OK
    bad = [
        (dict(feat_dim=300), rast.FE_ERR_UNSUPPORTED), (dict(feat_dim=0), rast.FE_ERR_INVALID_ARG),
        (dict(sh_degree=4), rast.FE_ERR_UNSUPPORTED), (dict(tile_w=12), rast.FE_ERR_UNSUPPORTED),
        (dict(tile_w=16, tile_h=5), rast.FE_ERR_UNSUPPORTED),
    ]
    for kw, code in bad:
        c = _cfg(**kw).to_c(1 << 20)
        assert lib.fe_validate(C.byref(c), C.byref(cam), 1000) == code, kw
    assert lib.fe_validate(C.byref(ok), C.byref(cam), -1) == rast.FE_ERR_INVALID_ARG
    big = rast.camera_c(_cam(40000, 10))
    assert lib.fe_validate(C.byref(ok), C.byref(big), 10) == rast.FE_ERR_UNSUPPORTED
    assert lib.fe_state_bytes(C.byref(_cfg(feat_dim=999).to_c(10)), C.byref(cam), 10) == 0
    lay = rast.state_layout(_cam(), _cfg(), 300_000, 4_800_000)
    for k, v in lay.items():
        if k != "total":
            assert v % 256 == 0 and v < lay["total"], k
    assert lay["total"] >= 300_000 * 48 + 4_800_000 * 16
    assert lib.fe_backward_scratch_bytes(C.byref(ok), C.byref(cam), 1000) >= 1000 * 36


def test_forward_rejects_bad_arguments_before_any_gpu_work():
    from paper_2503_06161_amd import rast
    lib = rast.load_library()
    cam = rast.camera_c(_cam())
    cfg = _cfg().to_c(1 << 16)
    g = rast.fe_gaussians()
    g.n = 10                     # pointers left NULL
    im = rast.fe_images()
    st = lib.fe_render_forward(C.byref(cfg), C.byref(cam), C.byref(g), C.byref(im), None, 0, None)
    assert st == rast.FE_ERR_INVALID_ARG
    assert lib.fe_render_forward(None, C.byref(cam), C.byref(g), C.byref(im), None, 0, None) == rast.FE_ERR_INVALID_ARG
    # a state buffer that is not 256-byte aligned is refused before anything
    # is launched (the pointers are never dereferenced on this path)
    fake = 1 << 20
    g = rast.fe_gaussians(10, fake, fake, fake, fake, fake, fake)
    im = rast.fe_images(fake, fake, fake, fake)
    big = lib.fe_state_bytes(C.byref(cfg), C.byref(cam), 10) + 512
    assert lib.fe_render_forward(C.byref(cfg), C.byref(cam), C.byref(g), C.byref(im),
                                 C.c_void_p(fake + 16), big, None) == rast.FE_ERR_INVALID_ARG
    assert lib.fe_render_forward(C.byref(cfg), C.byref(cam), C.byref(g), C.byref(im),
                                 C.c_void_p(fake), 16, None) == rast.FE_ERR_WORKSPACE_TOO_SMALL
    rep = rast.fe_report()
    assert lib.fe_read_report(None, 0, C.byref(rep), None) == rast.FE_ERR_INVALID_ARG
    assert lib.fe_status_string(rast.FE_ERR_KEY_OVERFLOW) == b"sort key capacity exceeded"


def test_threads_per_tile_choices():
    """threads_per_tile: 0, one per pixel, or two per pixel where the
    wave-specialized kernels exist in both directions (host-only checks)."""
    from paper_2503_06161_amd import rast
    lib = rast.load_library()
    cam = rast.camera_c(_cam())

    def v(**kw):
        return lib.fe_validate(C.byref(_cfg(**kw).to_c(1 << 20)), C.byref(cam), 1000)

    bf = dict(sh_dtype="bf16", feat_dtype="bf16", variant=rast.FE_VARIANT_MFMA)
    assert v(feat_dim=128, threads_per_tile=0, **bf) == rast.FE_OK
    assert v(feat_dim=128, threads_per_tile=256, **bf) == rast.FE_OK
    assert v(feat_dim=128, threads_per_tile=512, **bf) == rast.FE_OK
    assert v(feat_dim=64, tile_w=16, tile_h=8, threads_per_tile=256, **bf) == rast.FE_OK
    assert v(feat_dim=32, threads_per_tile=512, **bf) == rast.FE_OK   # narrow features: the 128-channel kernel
    assert v(feat_dim=200, threads_per_tile=512, **bf) == rast.FE_ERR_UNSUPPORTED     # D > 128
    assert v(feat_dim=128, threads_per_tile=512, variant=rast.FE_VARIANT_MFMA) == rast.FE_ERR_UNSUPPORTED  # FP32
    assert v(feat_dim=128, threads_per_tile=512, sh_dtype="bf16", feat_dtype="bf16",
             variant=rast.FE_VARIANT_VALU) == rast.FE_ERR_UNSUPPORTED
    assert v(feat_dim=128, threads_per_tile=100, **bf) == rast.FE_ERR_UNSUPPORTED
