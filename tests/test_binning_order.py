"""The key order the HIP binning relies on, checked on the CPU against the
oracle's lists: a pair's emit position is its Gaussian's first position (the
exclusive prefix of the pair counts in index order) plus the tile's
row-major place in the Gaussian's tile rectangle; sorting each tile's keys
(float32 depth bits << 32 | emit position) must give the order of the
oracle's sort by (tile, depth bits, index), ties in depth included."""
import numpy as np
import pytest

from paper_2503_06161_amd.scenes import make_scene, crop_camera
from oracle.project import project, OracleConfig
from oracle.raster import bin_gaussians


def _lists_by_emit_keys(p, cam, tw, th):
    rect = p["rect"].numpy()
    count = p["count"].numpy().astype(np.int64)
    dbits = p["depth"].numpy().astype(np.float32).view(np.uint32).astype(np.uint64)
    tiles_x = -(-cam.width // tw)
    tiles_y = -(-cam.height // th)
    eoff = np.concatenate([[0], np.cumsum(count)[:-1]])
    tile_keys = [[] for _ in range(tiles_x * tiles_y)]
    gofe = np.zeros(int(count.sum()), np.int64)
    for g in np.nonzero(count > 0)[0]:
        tx0, ty0, tx1, ty1 = rect[g]
        e = int(eoff[g])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                tile_keys[ty * tiles_x + tx].append((int(dbits[g]) << 32) | e)
                gofe[e] = g
                e += 1
    gidx, tile_of = [], []
    for t, keys in enumerate(tile_keys):
        for k in sorted(keys):
            gidx.append(gofe[k & 0xFFFFFFFF])
            tile_of.append(t)
    return np.asarray(tile_of, np.int64), np.asarray(gidx, np.int64)


@pytest.mark.parametrize("flat", [False, True])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_emit_position_keys_give_the_depth_then_index_order(flat, tile):
    sc = make_scene("small", seed=31, n=1500)
    if flat:
        sc.means[:, 2] = np.float32(4.0)     # every depth equal: order by index alone
    cam = crop_camera(sc.cam, 20, 24, 80, 72)
    cfg = OracleConfig(tile_w=tile[0], tile_h=tile[1], sh_degree=sc.sh_degree)
    p = project(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=sc.sh,
                cam=cam, cfg=cfg)
    L = bin_gaussians(p, cam, cfg)
    assert L.k > 1000
    if flat:
        assert len(np.unique(L.depth_bits)) == 1
    tile_of, gidx = _lists_by_emit_keys(p, cam, *tile)
    np.testing.assert_array_equal(tile_of, L.tile_of)
    np.testing.assert_array_equal(gidx, L.gidx)
