#!/usr/bin/env python3
"""Forward+backward throughput of the feature-distilled Gaussian rasterizer
on one MI355X.

Workload: one 640x512 camera, 300,000 Gaussians, SH degree 3, 128 semantic
channels, 16x16 tiles (the paper's frame size and feature width), seeded
synthetic scene.  A step is one forward render plus its backward pass for
one frame, through the C ABI on one HIP stream, with every input already in
HBM.  Both storage forms are timed: SH and features in BF16 (the reported
value) and plain FP32, and their speedup is reported beside it.

Prints one JSON line.  Stage durations come from HIP events that the library
records on the stream around each stage during the timed steps.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "metric"


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-tiles", type=int, default=0,
                    help="tiles blended by the CPU oracle (0: every tile, i.e. one whole frame)")
    ap.add_argument("--forms", default="bf16,f32")
    ap.add_argument("--variant", default="mfma", choices=["mfma", "valu"],
                    help="compositing kernels: matrix cores (default) or vector ALU")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-timestamp graph form")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM counters)")
    return ap.parse_args()


def _device_inputs(sc, form):
    import numpy as np
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    lo = torch.bfloat16 if form == "bf16" else torch.float32
    return dict(means=t(sc.means), scales=t(sc.scales), quats=t(sc.quats), opacity=t(sc.opacity),
                sh=t(sc.sh).to(lo).contiguous(), feat=t(sc.feat).to(lo).contiguous()), t(sc.d_rgb), t(sc.d_feat)


def _processed_pairs(n_contrib, tile_w, tile_h):
    """(tile, list position) pairs a compositing launch walks: per tile, the
    largest n_contrib of its pixels."""
    import torch
    H, W = n_contrib.shape
    th, tw = -(-H // tile_h), -(-W // tile_w)
    x = torch.zeros(th * tile_h, tw * tile_w, dtype=torch.int32, device=n_contrib.device)
    x[:H, :W] = n_contrib
    m = x.reshape(th, tile_h, tw, tile_w).amax(dim=(1, 3))
    return int(m.sum().item())


def _algorithmic_bytes(stage, n, k, pairs, H, W, D, L, eb):
    """Bytes a stage must move once (inputs read once, outputs written once)."""
    K3 = 3 * (L + 1) ** 2
    rec = 8 + 16 + 16 + 8                       # xy, conic+opacity, colour, pixel box
    if stage == "composite":
        return pairs * (rec + D * eb) + H * W * ((D + 3) * 4 + 8)
    if stage == "composite_bwd":
        return H * W * ((D + 3) * 4 + 8) + pairs * (rec + D * eb) + pairs * (D + 9) * 4
    if stage == "project":
        return n * (12 + 12 + 16 + 4 + K3 * eb) + n * (rec + 8)
    if stage == "project_bwd":
        return n * (12 + 12 + 16 + K3 * eb + 36) + n * (12 + 12 + 16 + 4 + K3 * 4)
    if stage == "sort":
        # per Gaussian: tile count, pixel box, depth key; per key: placed and read
        # (8 + 8), sorted Gaussian id and emit position written (8), emit-order
        # Gaussian id written and gathered (4 + 4)
        return n * 16 + k * 32
    return 0


def run_form(sc, form, steps, warmup, variant="mfma"):
    import torch
    from paper_2503_06161_amd import rast
    d, d_rgb, d_feat = _device_inputs(sc, form)
    st = rast.Settings(sh_degree=sc.sh_degree, feat_dim=sc.feat_dim, tile_w=16, tile_h=16,
                       sh_dtype=form, feat_dtype=form,
                       variant=rast.FE_VARIANT_VALU if variant == "valu" else rast.FE_VARIANT_MFMA)
    args = (d["means"], d["scales"], d["quats"], d["opacity"], d["sh"], d["feat"])
    fwd = rast.render_forward(*args, sc.cam, st, check=True)      # sizes the key buffers
    rep = fwd.report
    st.key_capacity = fwd.cfg.key_capacity
    st.row_capacity = max(int(rep["rows_needed"]), 1)
    out = dict(rgb=fwd.rgb, feat=fwd.feat, final_T=fwd.final_T, n_contrib=fwd.n_contrib)
    grads = None
    scratch = None

    def step(events=None):
        nonlocal fwd, grads, scratch
        st.stage_events = events
        f = rast.render_forward(*args, sc.cam, st, check=False, state=fwd.state, out=out)
        g = rast.render_backward(f, *args, d_rgb, d_feat, st, grads=grads, scratch=scratch, check=False)
        fwd, grads, scratch = f, g, g["_scratch"]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ns = len(rast.STAGES)

    def make_events(stages):
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * ns)] for _ in range(steps)]
        for row in evs:
            for e in row:
                e.record()   # creates the HIP event on this device
        torch.cuda.synchronize()
        handles = [(C.c_void_p * (2 * ns))(*[e.cuda_event if (k // 2) in stages else None
                                              for k, e in enumerate(row)]) for row in evs]
        return evs, handles

    def stage_times(evs, stages):
        out = {}
        for s_i, name in enumerate(rast.STAGES):
            if s_i not in stages:
                continue
            vals = []
            for row in evs:
                try:
                    vals.append(row[2 * s_i].elapsed_time(row[2 * s_i + 1]))
                except RuntimeError:
                    pass
            if vals and max(vals) > 0:
                out[name] = sum(vals) / len(vals)
        return out

    # 1. per-stage breakdown (untimed pass): events recorded by the library on
    #    the call's stream around every stage
    every = set(range(ns))
    evs, handles = make_events(every)
    for i in range(steps):
        step(handles[i])
    torch.cuda.synchronize()
    stage_ms = stage_times(evs, every)
    dominant = max(stage_ms, key=stage_ms.get)
    # 2. timed region: exactly `steps` steps, events only around the dominant stage
    dom = {rast.STAGES.index(dominant)}
    evs, handles = make_events(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(handles[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st.stage_events = None
    stage_ms.update(stage_times(evs, dom))
    pairs = _processed_pairs(fwd.n_contrib, 16, 16)
    rep2 = rast.read_report(fwd.state)
    return dict(ms_per_step=1e3 * (t1 - t0) / steps, fps=steps / (t1 - t0), stage_ms=stage_ms, pairs=pairs,
                keys=int(rep2["keys_needed"]), report=rep, eb=2 if form == "bf16" else 4)


def run_batched(steps, warmup):
    """16 timestamps of one deforming scene (50k-200k Gaussians per frame,
    D=64 BF16, 640x512), forward+backward of all frames as one graph replay."""
    import numpy as np
    import torch
    from paper_2503_06161_amd import rast
    from paper_2503_06161_amd.batch import BatchRenderer
    from paper_2503_06161_amd.scenes import batched_frames
    sc, fr = batched_frames()
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    frames, cams = [], []
    for f in fr:
        n = f["n"]
        frames.append(dict(means=t(f["means"]), scales=t(sc.scales[:n]), quats=t(sc.quats[:n]),
                           opacity=t(sc.opacity[:n]), sh=t(sc.sh[:n]).bfloat16().contiguous(),
                           feat=t(sc.feat[:n]).bfloat16().contiguous()))
        cams.append(sc.cam)
    rng = np.random.default_rng(44)
    H, W = sc.cam.height, sc.cam.width
    d_rgb = [t(rng.normal(0, 1e-3, (3, H, W)).astype(np.float32)) for _ in fr]
    d_feat = [t(rng.normal(0, 1e-3, (64, H, W)).astype(np.float32)) for _ in fr]
    st = rast.Settings(sh_degree=3, feat_dim=64, sh_dtype="bf16", feat_dtype="bf16")
    # tile shape and variant from the batch autotuner (untimed; whole replays)
    from paper_2503_06161_amd import autotune
    st = autotune.autotune_batch(frames, cams, st, d_rgb, d_feat)
    br = BatchRenderer(frames, cams, st, rast.FE_MODE_FORWARD_BACKWARD, d_rgb, d_feat)
    for _ in range(warmup):
        br.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        br.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bad = [k for k in range(len(fr)) if br.report(k)["status"] != 0]
    br.close()
    ms = 1e3 * (t1 - t0) / steps
    return dict(frames=len(fr), gaussians_per_frame=[f["n"] for f in fr], ms_per_replay=round(ms, 4),
                frames_per_s=round(len(fr) * 1e3 / ms, 2), status_errors=bad,
                tile=f"{st.tile_w}x{st.tile_h}", variant="valu" if st.variant == rast.FE_VARIANT_VALU else "mfma")


def cpu_baseline(sc, sample_tiles):
    """The float64 oracle, as it is, forward + backward on the same frame:
    projection, binning and projection backward of all Gaussians, and the
    blending forward+backward of every tile (or of `sample_tiles` evenly spaced
    tiles, with the frame time extrapolated to all tiles)."""
    import numpy as np
    import torch
    import oracle
    from paper_2503_06161_amd.scenes import bf16_round
    inp = dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacity=sc.opacity, sh=bf16_round(sc.sh),
               feat=bf16_round(sc.feat))
    cfg = oracle.OracleConfig(tile_w=16, tile_h=16, sh_degree=sc.sh_degree)
    ntiles = -(-sc.cam.width // 16) * -(-sc.cam.height // 16)
    oracle.render_backward(**inp, cam=sc.cam, cfg=cfg, d_rgb=sc.d_rgb, d_feat=sc.d_feat, tiles=[0])   # warm-up
    if sample_tiles <= 0 or sample_tiles >= ntiles:
        t0 = time.perf_counter()
        oracle.render_backward(**inp, cam=sc.cam, cfg=cfg, d_rgb=sc.d_rgb, d_feat=sc.d_feat)
        per_frame = time.perf_counter() - t0
        what = f"one whole frame ({per_frame:.1f} s of CPU work)"
    else:
        sample = list(np.linspace(0, ntiles - 1, sample_tiles).astype(int))
        t0 = time.perf_counter()
        oracle.render_backward(**inp, cam=sc.cam, cfg=cfg, d_rgb=sc.d_rgb, d_feat=sc.d_feat, tiles=[])
        t1 = time.perf_counter()
        oracle.render_backward(**inp, cam=sc.cam, cfg=cfg, d_rgb=sc.d_rgb, d_feat=sc.d_feat, tiles=sample)
        t2 = time.perf_counter()
        per_tile = max((t2 - t1) - (t1 - t0), 0.0) / len(sample)
        per_frame = (t1 - t0) + per_tile * ntiles
        what = (f"projection, binning and projection backward of all {sc.n} Gaussians plus {len(sample)} of "
                f"{ntiles} tiles blended forward+backward ({t2 - t0:.1f} s of CPU work), extrapolated to all tiles")
    return dict(value=1.0 / per_frame, unit="frames/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"float64 oracle fwd+bwd of the {sc.cam.width}x{sc.cam.height}, {sc.n}-Gaussian, "
                       f"D={sc.feat_dim} frame: {what}")


def _kernel_source_hash():
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2503_06161_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:12]


def _traffic(stage):
    """HBM traffic from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{stage}_metric_pmc.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != _kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(frames shard across GPUs as independent renders, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_06161_amd.scenes import make_scene
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sc = make_scene(WORKLOAD)
    res = {}
    for form in args.forms.split(","):
        res[form] = run_form(sc, form, args.steps, args.warmup, args.variant)
    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    main_form = "bf16" if "bf16" in res else next(iter(res))
    r = res[main_form]
    H, W, D, L = sc.cam.height, sc.cam.width, sc.feat_dim, sc.sh_degree
    stage, ms = max(r["stage_ms"].items(), key=lambda kv: kv[1])
    by = _algorithmic_bytes(stage, sc.n, r["keys"], r["pairs"], H, W, D, L, r["eb"])
    achieved = by / (ms * 1e-3) / 1e9
    line = {
        "metric": "fwd+bwd frames/s at 640x512, 300k Gaussians, D=128; BF16 vs FP32 speedup",
        "value": round(r["fps"], 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 storage, f32 compute" if main_form == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": "640x512 camera (f=512), 300k Gaussians, SH degree 3, D=128 features, "
                               "16x16 tiles, one frame forward+backward", "form": main_form,
                   "gaussians": sc.n, "width": W, "height": H, "feat_dim": D, "sh_degree": L,
                   "keys": r["keys"], "processed_tile_pairs": r["pairs"], "variant": args.variant},
        "forms": {f: {"frames_per_s": round(v["fps"], 2), "ms_per_step": round(v["ms_per_step"], 4),
                      "stage_ms": {k: round(x, 4) for k, x in v["stage_ms"].items()}} for f, v in res.items()},
        "roofline": {"kernel": stage, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": _traffic(stage), "algorithmic_bytes": by},
    }
    if "bf16" in res and "f32" in res:
        line["bf16_speedup_vs_f32"] = round(res["f32"]["ms_per_step"] / res["bf16"]["ms_per_step"], 4)
    if not args.no_batched:
        try:
            line["batched_16_timestamps"] = run_batched(max(3, args.steps // 2), 2)
        except Exception as e:  # reported, never hides the main measurement
            line["batched_16_timestamps"] = {"error": repr(e)[:200]}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_sample_tiles)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
