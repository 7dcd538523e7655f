"""Summaries of rocprofv3 output for the kernels of this library.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats`` and
``--pmc`` runs, ``--output-format csv``) and prints short Markdown or JSON
summaries: per-kernel average duration, and per-kernel counter values
averaged over dispatches.  HBM traffic counters are scaled by the same
counters read on a plain device copy of known size (``bench.py
--calibrate-copy`` issues one 256 MiB copy), so that FETCH_SIZE / WRITE_SIZE
become bytes.

  python -m paper_2503_06161_amd.profiling trace <dir> [--match REGEX]
  python -m paper_2503_06161_amd.profiling pmc <dir> [<dir> ...] [--match REGEX] [--json KERNEL]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

COPY_BYTES = 256 << 20      # bench.py --calibrate-copy
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# the sources each frame stage's kernels are built from, and the kernels
STAGE_SOURCES = {
    "composite": ("fe_composite_mfma.hip", "fe_common.h"),
    "composite_bwd": ("fe_backward_mfma.hip", "fe_common.h"),
    "project": ("fe_project.hip", "fe_common.h"),
    "project_bwd": ("fe_project.hip", "fe_common.h"),
    "sort": ("fe_sort.hip", "fe_common.h"),
    "reduce": ("fe_backward_mfma.hip", "fe_common.h"),
}
STAGE_KERNELS = {
    "composite": r"^composite_fwd",
    "composite_bwd": r"^composite_bwd",
    "project": r"^project_fwd",
    "project_bwd": r"^project_bwd",
    "sort": r"^(bin_count|bin_offsets|bin_place|tile_sort|zero_u32)",
    "reduce": r"^(reduce_rows|backward_prep)",
}


def kernel_source_hash(stage: str) -> str:
    """Hash of the sources of one stage's kernels: a traffic record taken on
    other sources is stale."""
    h = hashlib.sha1()
    for f in STAGE_SOURCES[stage]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def _csv_rows(root: str, suffix: str):
    rows = []
    for path in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _short(name: str) -> str:
    name = re.sub(r"^void ", "", name.strip())
    if name.endswith(")"):                            # drop the argument list (the last balanced group)
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(name[i], 0)
            if depth == 0:
                name = name[:i]
                break
    name = name.replace("fe::(anonymous namespace)::", "").replace("fe::", "")
    return name.replace("unsigned short", "bf16")


def kernel_times(root: str):
    """{kernel: (dispatches, average us, grid, block, lds, vgpr, agpr, scratch)} from the kernel trace."""
    acc = defaultdict(list)
    info = {}
    for r in _csv_rows(root, "kernel_trace.csv"):
        k = _short(r["Kernel_Name"])
        acc[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        info[k] = (r.get("Grid_Size", ""), r.get("Workgroup_Size", ""), r.get("LDS_Block_Size", ""),
                   r.get("VGPR_Count", ""), r.get("Accum_VGPR_Count", ""), r.get("Scratch_Size", ""))
    return {k: (len(v), sum(v) / len(v)) + info[k] for k, v in acc.items()}


def counters(roots):
    """{kernel: {counter: average value per dispatch}} over one or more --pmc runs."""
    acc = defaultdict(lambda: defaultdict(list))
    for root in roots:
        for r in _csv_rows(root, "counter_collection.csv"):
            acc[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def copy_scale(roots):
    """Bytes per FETCH_SIZE / WRITE_SIZE unit, from the calibration copy: the
    copy dispatch with the largest count in each run is the 256 MiB
    device-to-device copy of ``bench.py --calibrate-copy``."""
    best = {}
    for root in roots:
        for r in _csv_rows(root, "counter_collection.csv"):
            if re.search(r"copy|elementwise", r["Kernel_Name"], re.I) and r["Counter_Name"] in ("FETCH_SIZE", "WRITE_SIZE"):
                v = float(r["Counter_Value"])
                best[r["Counter_Name"]] = max(best.get(r["Counter_Name"], 0.0), v)
    f = COPY_BYTES / best["FETCH_SIZE"] if best.get("FETCH_SIZE") else None
    w = COPY_BYTES / best["WRITE_SIZE"] if best.get("WRITE_SIZE") else None
    return f, w


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--match", default=".")
    p = sub.add_parser("pmc")
    p.add_argument("dirs", nargs="+")
    p.add_argument("--match", default=".")
    p.add_argument("--json", default=None, help="print the traffic record of the first kernel matching this regex")
    tr = sub.add_parser("traffic", help="per-stage HBM bytes per launch (FETCH_SIZE run, WRITE_SIZE run)")
    tr.add_argument("fetch_dir")
    tr.add_argument("write_dir")
    tr.add_argument("--command", default="", help="the rocprofv3 command the runs came from")
    a = ap.parse_args(argv)
    if a.cmd == "traffic":
        cnt = counters([a.fetch_dir, a.write_dir])
        fs, ws = copy_scale([a.fetch_dir, a.write_dir])
        if not (fs and ws):
            print("no calibration copy in these runs", file=sys.stderr)
            return 1
        stages = {}
        for st, rx in STAGE_KERNELS.items():
            ks = [k for k in cnt if re.search(rx, k)]
            if not ks:
                continue
            rd = sum(cnt[k].get("FETCH_SIZE", 0.0) for k in ks) * fs
            wr = sum(cnt[k].get("WRITE_SIZE", 0.0) for k in ks) * ws
            stages[st] = {"kernels": sorted(ks), "source_files": list(STAGE_SOURCES[st]),
                          "source_hash": kernel_source_hash(st), "read_bytes": round(rd), "write_bytes": round(wr),
                          "bytes_per_launch": round(rd + wr)}
        print(json.dumps({"workload": "640x512, 300k Gaussians, SH 3, D=128, BF16 storage, MFMA kernels, 16x16 tiles",
                          "fetch_scale": fs, "write_scale": ws, "command": a.command, "stages": stages}, indent=1))
        return 0
    if a.cmd == "trace":
        kt = kernel_times(a.dir)
        print("| kernel | dispatches | avg µs | grid | block | LDS B | VGPR | AGPR | scratch |")
        print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
        for k, (n, us, grid, blk, lds, vg, ag, scr) in sorted(kt.items(), key=lambda kv: -kv[1][1] * kv[1][0]):
            if re.search(a.match, k):
                print(f"| `{k}` | {n} | {us:.2f} | {grid} | {blk} | {lds} | {vg} | {ag} | {scr} |")
        return 0
    cnt = counters(a.dirs)
    fs, ws = copy_scale(a.dirs)
    if a.json:
        for k, d in cnt.items():
            if re.search(a.json, k):
                rd = d.get("FETCH_SIZE", 0.0) * (fs or 0.0)
                wr = d.get("WRITE_SIZE", 0.0) * (ws or 0.0)
                print(json.dumps({"kernel": k, "read_bytes": round(rd), "write_bytes": round(wr),
                                  "bytes_per_launch": round(rd + wr), "fetch_scale": fs, "write_scale": ws}))
                return 0
        return 1
    names = sorted({c for d in cnt.values() for c in d})
    print(f"copy calibration: bytes per FETCH_SIZE unit = {fs:.1f}, per WRITE_SIZE unit = {ws:.1f}"
          if fs and ws else "no calibration copy in these runs")
    print()
    print("| kernel | " + " | ".join(names) + " |")
    print("|---|" + "---:|" * len(names))
    for k, d in sorted(cnt.items()):
        if re.search(a.match, k):
            print(f"| `{k}` | " + " | ".join(f"{d[c]:.4g}" if c in d else "" for c in names) + " |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
