"""Tile binning and the per-tile depth sort of the HIP path against the
oracle's lists (tile, then float32 depth bits, then Gaussian index):
a list longer than one workgroup sorts in LDS (sorted chunks merged through
global memory), depths that tie (ordered by index), and more tiles than the
per-workgroup LDS counters cover (one global atomic per pair)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from paper_2503_06161_amd import rast
from paper_2503_06161_amd.scenes import make_scene, crop_camera
from oracle.project import project
from oracle.raster import bin_gaussians
from tests import gpu_util as U


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rast.load_library()


def _oracle_lists(sc, st, cam):
    inp = U.stored_inputs(sc, st.feat_dtype)
    inp.pop("feat")
    cfg = U.oracle_cfg(sc, st)
    p = project(**inp, cam=cam, cfg=cfg)
    return dict(proj=p, lists=bin_gaussians(p, cam, cfg))


def _check(sc, st, cam):
    fwd, _ = U.gpu_forward(sc, st, cam=cam)
    orc = _oracle_lists(sc, st, cam)
    gs = U.read_state(fwd, sc.n, st, cam)
    U.compare_projection(gs, orc, sc.n)
    U.compare_keys(gs, orc)
    return orc["lists"]


@pytest.mark.parametrize("variant", [rast.FE_VARIANT_VALU, rast.FE_VARIANT_MFMA])
def test_one_tile_longer_than_an_lds_sort(variant):
    # 24000 Gaussians squeezed onto one 16x16 tile, on three depth planes:
    # three sorted chunks and two merge rounds, with ties inside every chunk
    say("one tile, 24000 keys, variant", variant)
    sc = make_scene("small", seed=21, n=24000)
    sc.means[:, :2] *= 0.08
    sc.means[:, 2] = np.array([3.0, 3.5, 4.0], np.float32)[np.arange(sc.n) % 3]
    cam = crop_camera(sc.cam, 56, 56, 16, 16)
    st = U.settings_for(sc, variant=variant)
    L = _check(sc, st, cam)
    assert L.k > 16384


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_equal_depths_are_ordered_by_index(tile):
    say("all depths equal, tile", tile)
    sc = make_scene("small", seed=22, n=6000)
    sc.means[:, 2] = 4.0
    cam = crop_camera(sc.cam, 40, 40, 48, 48)
    st = U.settings_for(sc, tile=tile)
    L = _check(sc, st, cam)
    assert L.k > 1000 and len(np.unique(L.depth_bits)) == 1


def test_more_tiles_than_the_lds_counters():
    # 1040 x 1040 in 8x8 tiles: 16900 tiles, above the LDS binning limit
    say("16900 tiles")
    sc = make_scene("small", seed=23, n=3000, width=1040, height=1040, f=832.0)
    st = U.settings_for(sc, tile=(8, 8))
    L = _check(sc, st, sc.cam)
    assert L.ranges.shape[0] == 16900 and L.k > 100000
