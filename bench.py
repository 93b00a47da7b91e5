#!/usr/bin/env python3
"""Throughput of the batched per-ROI GLCM path on one MI355X.

One step = the whole path over one batch of images already resident in HBM:
ROI discovery and per-ROI statistics, fixed-bin-number binning, co-occurrence
counting over the offsets, and the 30 GLCM features per direction plus their
mean, replayed as one HIP graph (nyx_plan_execute).  The metric is ROI-voxels
per second (sum of ROI voxel counts / step time), reported next to the same
step with one accumulation launch per ROI (nyx_plan_execute_per_roi), the
per-phase kernel times measured with HIP events, and the CPU oracle timed on
a bounded sample of the same workload.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, offs, seconds: float) -> dict:
    """The oracle, as it stands, on whole images of the workload until about
    `seconds` of wall time; all host threads."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    off = np.array(offs, np.int32)
    vox, t0, n_img = 0, time.perf_counter(), 0
    for k in range(w.n_images):
        st, _ = oracle.extract(w.intensity[k], w.labels[k], w.n_bins, off, n_threads=threads)
        vox += int(st["count"].sum())
        n_img += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": vox / dt, "unit": "ROI-voxels/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_img} of {w.n_images} images ({vox} ROI voxels), FP64 oracle, {dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3_batch")
    ap.add_argument("--per-roi-steps", type=int, default=1)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU; multi-GPU runs are not part of this build (use --gpus 1)",
              file=sys.stderr)
        return 2

    import torch

    import synth
    from paper_2603_12016_amd import nyx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    w = synth.make(args.workload)
    log(f"generated {args.workload} in {time.perf_counter() - t0:.1f} s")
    imgs = []
    for k in range(w.n_images):
        imgs.append((torch.from_numpy(w.intensity[k].view(np.int16)).to(dev),
                     torch.from_numpy(w.labels[k].view(np.int32)).to(dev)))
    torch.cuda.synchronize()
    offs = nyx.nyx_offsets_default(w.dims, 1)
    K = len(offs)
    prec = nyx.NYX_FP64 if w.precision == "fp64" else nyx.NYX_FP32
    ctx = nyx.nyx_create(0)
    t0 = time.perf_counter()
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, prec, autotune=not args.no_autotune)
    plan_s = time.perf_counter() - t0
    log(f"plan in {plan_s:.2f} s: {nyx.nyx_plan_describe(plan)}")
    n_rois = plan.n_rois
    roi_vox = int(np.count_nonzero(w.labels))
    img_vox = int(w.labels.size)
    table = nyx.new_table(plan, K, prec)

    for _ in range(args.warmup):
        nyx.nyx_plan_execute(plan, table)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    log(f"warmup done ({args.warmup} steps)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nyx.nyx_plan_execute(plan, table)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nyx.nyx_plan_check(plan)
    ms = dt * 1e3 / args.steps
    value = roi_vox / (dt / args.steps)
    log(f"batched: {ms:.3f} ms/step, {value / 1e9:.2f} G ROI-voxels/s")

    # phase times of the same step, eager, with HIP events between phases
    prof = {p: 0.0 for p in nyx.PHASES}
    for _ in range(args.profile_steps):
        r = nyx.nyx_plan_profile(plan, table)
        for p in prof:
            prof[p] += r[p] / args.profile_steps
    log("phases (ms): " + ", ".join(f"{p}={v:.4f}" for p, v in prof.items()))

    # one launch per ROI
    dt_roi, same = None, None
    if args.per_roi_steps > 0:
        t2 = nyx.new_table(plan, K, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.per_roi_steps):
            nyx.nyx_plan_execute_per_roi(plan, t2)
        torch.cuda.synchronize()
        dt_roi = (time.perf_counter() - t0) / args.per_roi_steps
        nyx.nyx_plan_check(plan)
        same = bool(torch.allclose(table, t2, rtol=1e-5, atol=1e-6, equal_nan=True))
        log(f"per-ROI launches: {dt_roi * 1e3:.1f} ms/step, tables agree: {same}")

    # algorithmic bytes: scan reads 4 B label + 2 B intensity
    # per image voxel; the accumulate/feature kernel reads 4 B label + 2 B
    # intensity per ROI voxel and writes the feature rows.
    out_bytes = n_rois * (K + 1) * 30 * (8 if prec == nyx.NYX_FP64 else 4)
    alg = {"scan": img_vox * 6.0, "batch": roi_vox * 6.0 + out_bytes}
    dom = max(("scan", "batch"), key=lambda p: prof[p])
    achieved = alg[dom] / (prof[dom] * 1e-3) / 1e9
    step_alg = img_vox * 4.0 + roi_vox * 2.0 + out_bytes

    rec = {
        "metric": "ROI-voxels/s for GLCM+features, batched vs per-ROI launch; % HBM peak",
        "value": value,
        "unit": "ROI-voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 counts, f32 features" if prec == nyx.NYX_FP32 else "u32 counts, f64 features",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": w.description, "images": w.n_images,
                   "image_voxels": img_vox, "roi_voxels": roi_vox, "rois": n_rois, "n_bins": w.n_bins,
                   "offsets": K, "plan": nyx.nyx_plan_describe(plan)},
        "per_roi_launch": None if dt_roi is None else {"value": roi_vox / dt_roi, "ms_per_step": dt_roi * 1e3,
                                                       "steps": args.per_roi_steps, "tables_agree": same},
        "speedup_vs_per_roi": None if dt_roi is None else dt_roi * 1e3 / ms,
        "step_hbm_frac_alg": step_alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "phases_ms": prof,
        "roofline": {"kernel": "k_batch" if dom == "batch" else "k_scan", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "plan_seconds": plan_s,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(w, offs, args.cpu_seconds)
        log(f"cpu baseline: {rec['cpu_baseline']['value'] / 1e6:.2f} M ROI-voxels/s")
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
