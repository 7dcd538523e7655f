"""Tile-shape / threads-per-tile / kernel-variant selection by timing.

Every candidate renders the same image (the 3-sigma box rule makes the
result independent of the tile shape; the kernels differ only in how the
work is spread over threads), so the choice only changes speed.  Threads per
tile is one per pixel or, where the wave-specialized matrix-core kernels
exist, two per pixel.
Candidates are timed with HIP events on the current stream (forward, or
forward + backward), the fastest is kept, and results are cached in a JSON
file keyed by device, image size, feature width, storage dtypes and a
Gaussian-count bucket.  ``FE4DGS_AUTOTUNE_CACHE`` overrides the cache path.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import rast

TILE_SHAPES = [(16, 16), (32, 8), (16, 8), (8, 16), (8, 8)]
VARIANTS = [rast.FE_VARIANT_MFMA, rast.FE_VARIANT_VALU]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fe4dgs_autotune.json")


def _cache_path():
    return os.environ.get("FE4DGS_AUTOTUNE_CACHE", DEFAULT_CACHE)


def cache_key(cam, st: rast.Settings, n: int, backward: bool) -> str:
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    bucket = 2 ** int(math.log2(max(n, 1)))
    return (f"{dev}|{int(cam.width)}x{int(cam.height)}|D{st.feat_dim}|L{st.sh_degree}|{st.sh_dtype}/{st.feat_dtype}"
            f"|n~{bucket}|{'fwdbwd' if backward else 'fwd'}")


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c):
    path = _cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def candidates_for(st: rast.Settings, cam, n: int, shapes=None, variants=None):
    """(tile_w, tile_h, variant, threads_per_tile) combinations the library
    accepts for these settings (checked with the host-only fe_validate).
    threads_per_tile 0 lets each direction take the two-per-pixel kernel
    where it exists (which can differ between forward and backward)."""
    import ctypes as C
    lib = rast.load_library()
    cam_c = rast.camera_c(cam)
    out = []
    for tw, th in shapes or TILE_SHAPES:
        for v in variants or VARIANTS:
            # one thread per pixel, the library's choice per direction (0), two per pixel
            for tpt in (tw * th, 0, 2 * tw * th):
                if v == rast.FE_VARIANT_VALU and tpt != tw * th:
                    continue                      # one kernel form only
                s2 = rast.Settings(**{**st.__dict__, "tile_w": tw, "tile_h": th, "variant": v, "threads_per_tile": tpt})
                if lib.fe_validate(C.byref(s2.to_c(1 << 20)), C.byref(cam_c), n) == rast.FE_OK:
                    out.append((tw, th, v, tpt))
    return out


def _pick(st, c):
    flags = (st.flags & ~rast.FE_FLAG_BATCH_PER_FRAME) | c.get("batch_flags", 0)
    return rast.Settings(**{**st.__dict__, "tile_w": c["tile_w"], "tile_h": c["tile_h"], "variant": c["variant"],
                            "threads_per_tile": c.get("threads_per_tile", 0), "flags": flags})


def time_candidate(g: dict, cam, st: rast.Settings, d_rgb=None, d_feat=None, reps: int = 5) -> float:
    """Median milliseconds of one forward (+ backward when upstream gradients
    are given) for the settings ``st``."""
    args = (g["means"], g["scales"], g["quats"], g["opacity"], g["sh"], g["feat"])
    fwd = rast.render_forward(*args, cam, st, check=True)
    st2 = rast.Settings(**{**st.__dict__, "key_capacity": fwd.cfg.key_capacity,
                           "row_capacity": max(int(fwd.report["rows_needed"]), 1)})
    out = dict(rgb=fwd.rgb, feat=fwd.feat, final_T=fwd.final_T, n_contrib=fwd.n_contrib)
    grads, scratch = None, None
    times = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f = rast.render_forward(*args, cam, st2, check=False, state=fwd.state, out=out)
        if d_rgb is not None:
            grads = rast.render_backward(f, *args, d_rgb, d_feat, st2, grads=grads, scratch=scratch, check=False)
            scratch = grads["_scratch"]
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def autotune(g: dict, cam, st: rast.Settings, d_rgb=None, d_feat=None, candidates=None, use_cache=True,
             verbose=False) -> rast.Settings:
    """Return a copy of ``st`` with the fastest tile shape, variant and
    threads per tile."""
    n = int(g["means"].shape[0])
    key = cache_key(cam, st, n, d_rgb is not None)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return _pick(st, cache[key])
    cands = candidates or candidates_for(st, cam, n)
    results = []
    for tw, th, v, tpt in cands:
        s2 = rast.Settings(**{**st.__dict__, "tile_w": tw, "tile_h": th, "variant": v, "threads_per_tile": tpt})
        ms = time_candidate(g, cam, s2, d_rgb, d_feat)
        results.append((ms, tw, th, v, tpt))
        if verbose:
            print(f"autotune {tw}x{th} variant {v} threads {tpt}: {ms:.3f} ms", flush=True)
    ms, tw, th, v, tpt = min(results)
    best = dict(tile_w=tw, tile_h=th, variant=v, threads_per_tile=tpt)
    if use_cache:
        cache[key] = dict(best, ms=ms, all=[dict(tile_w=a, tile_h=b, variant=c, threads_per_tile=t, ms=m)
                                            for m, a, b, c, t in results])
        _store_cache(cache)
    return _pick(st, best)


def autotune_batch(frames, cams, st: rast.Settings, d_rgb=None, d_feat=None, candidates=None, use_cache=True,
                   reps: int = 5, verbose=False) -> rast.Settings:
    """Tile shape and variant for a batch of frames, chosen by timing whole
    graph replays of the batch (the multi-frame compositing path included).
    ``frames``/``cams``/``d_rgb``/``d_feat`` are as for ``BatchRenderer``."""
    from .batch import BatchRenderer
    mode = rast.FE_MODE_FORWARD_BACKWARD if d_rgb is not None else rast.FE_MODE_FORWARD
    n = max(int(f["means"].shape[0]) for f in frames)
    key = cache_key(cams[0], st, n, d_rgb is not None) + f"|batch{len(frames)}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return _pick(st, cache[key])
    # each candidate twice: persistent multi-frame compositing, and every
    # frame's own kernels on parallel graph branches
    cands = candidates or [c + (fl,) for c in candidates_for(st, cams[0], n)
                           for fl in (0, rast.FE_FLAG_BATCH_PER_FRAME)]
    results = []
    for tw, th, v, tpt, fl in cands:
        s2 = rast.Settings(**{**st.__dict__, "tile_w": tw, "tile_h": th, "variant": v, "threads_per_tile": tpt,
                              "flags": (st.flags & ~rast.FE_FLAG_BATCH_PER_FRAME) | fl})
        br = BatchRenderer(frames, cams, s2, mode, d_rgb, d_feat)
        br.launch()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            br.launch()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        br.close()
        times.sort()
        ms = times[len(times) // 2]
        results.append((ms, tw, th, v, tpt, fl))
        if verbose:
            print(f"autotune batch {tw}x{th} variant {v} threads {tpt} flags {fl}: {ms:.3f} ms", flush=True)
    ms, tw, th, v, tpt, fl = min(results)
    best = dict(tile_w=tw, tile_h=th, variant=v, threads_per_tile=tpt, batch_flags=fl)
    if use_cache:
        cache[key] = dict(best, ms=ms, all=[dict(tile_w=a, tile_h=b, variant=c, threads_per_tile=t, batch_flags=f,
                                                 ms=m) for m, a, b, c, t, f in results])
        _store_cache(cache)
    return _pick(st, best)
