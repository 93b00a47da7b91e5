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
COPY_BYTES = 1 << 30    # the copy kernel's size (read and written once per rep)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SYMBOLS = {"k_batch": "nyx::k_batch<", "k_scan": "nyx::k_scan(", "k_band": "nyx::k_band("}
COPY_SYMBOL = "k_copy("


def source_digest() -> str:
    """Digest of the HIP sources: a stored traffic measurement is used only
    while the kernels it was taken on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_12016_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_path(kernel: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from two rocprofv3 counter runs
    (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the
    same counter reads for a copy kernel of known size in the same process;
    None if absent or taken on other sources."""
    try:
        with open(traffic_path(kernel, workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    return t["fetch_kib"] * 1024.0 * t["fetch_scale"] + t["write_kib"] * 1024.0 * t["write_scale"]


def summarize_pmc(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int, command: str) -> None:
    """Writes profiles/<kernel>_<workload>_traffic.txt (JSON) for every kernel in
    KERNEL_SYMBOLS from the counter CSVs of a FETCH_SIZE and a WRITE_SIZE run
    of this script (which runs the copy kernel on copy_bytes once per rep)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                for k, sym in list(KERNEL_SYMBOLS.items()) + [("copy", COPY_SYMBOL)]:
                    if sym in r["Kernel_Name"]:
                        vals.setdefault(k, []).append(float(r["Counter_Value"]))
        return {k: statistics.median(v) for k, v in vals.items()}
    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    fs = copy_bytes / (fetch["copy"] * 1024.0)
    ws = copy_bytes / (write["copy"] * 1024.0)
    for k in KERNEL_SYMBOLS:
        if k not in fetch or k not in write:
            continue
        rec = {"kernel": k, "workload": workload, "source_digest": source_digest(),
               "fetch_kib": fetch[k], "write_kib": write[k], "fetch_scale": fs, "write_scale": ws,
               "copy_kernel": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                               "fetch_kib": fetch["copy"], "write_kib": write["copy"]},
               "bytes_per_launch": fetch[k] * 1024.0 * fs + write[k] * 1024.0 * ws,
               "command": command}
        with open(traffic_path(k, workload), "w") as f:
            json.dump(rec, f, indent=1)
        log(f"{k}: {rec['bytes_per_launch'] / 1e9:.3f} GB per launch -> {traffic_path(k, workload)}")


def summarize_trace(stats_csv: str, workload: str, command: str, top: int = 14) -> None:
    """Writes profiles/<kernel>_<workload>.md for the dominant kernels from a
    rocprofv3 --kernel-trace --stats kernel_stats.csv of this script."""
    import csv
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel trace: {workload}", "", "Command (from the repository root on the GPU host):", "",
             f"    {command}", "", f"Sources: `paper_2603_12016_amd/csrc` digest {source_digest()}.", "",
             "| kernel | calls | total us | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e3:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    # named for the dominant kernel of KERNEL_SYMBOLS (largest total time)
    tot = {k: sum(float(r["TotalDurationNs"]) for r in rows if sym in r["Name"]) for k, sym in KERNEL_SYMBOLS.items()}
    k = max(tot, key=tot.get)
    if tot[k] > 0:
        path = os.path.join(ROOT, "profiles", f"{k}_{workload}.md")
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        log(f"wrote {path}")


def summarize_sq(sq_csv: str, workload: str, command: str, roi_vox: int) -> None:
    """Writes profiles/<kernel>_<workload>_counters.md from a rocprofv3 --pmc
    run of this script with the SQ counters below: the median per dispatch of
    every counter for each kernel in KERNEL_SYMBOLS, and what follows from
    them (SQ_BUSY_CYCLES is summed over the 32 shader engines, the LDS
    conflict counters over the 256 CUs; a wave64 VALU instruction occupies its
    SIMD for 4 cycles)."""
    import csv
    import statistics
    vals = {}
    with open(sq_csv) as f:
        for r in csv.DictReader(f):
            for k, sym in KERNEL_SYMBOLS.items():
                if sym in r["Kernel_Name"]:
                    vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    med = {k: {c: statistics.median(v) for c, v in cs.items()} for k, cs in vals.items()}
    names = sorted({c for cs in med.values() for c in cs})
    ks = [k for k in KERNEL_SYMBOLS if k in med]
    lines = [f"# rocprofv3 SQ counters: {workload}", "", "Command (from the repository root on the GPU host):", "",
             f"    {command}", "", f"Sources: `paper_2603_12016_amd/csrc` digest {source_digest()}.", "",
             "Median per dispatch.", "", "| counter | " + " | ".join(ks) + " |", "|---" * (len(ks) + 1) + "|"]
    for c in names:
        lines.append(f"| {c} | " + " | ".join(f"{med[k].get(c, float('nan')):.4g}" for k in ks) + " |")
    lines += ["", "| derived | " + " | ".join(ks) + " |", "|---" * (len(ks) + 1) + "|"]
    rows = {"kernel cycles (SQ_BUSY_CYCLES / 32)": [], "VALU busy (4 x ACTIVE_INST_VALU / (1024 SIMDs x cycles))": [],
            "LDS bank-conflict cycles per CU / kernel cycles": [], "LDS address-conflict cycles per CU / kernel cycles": [],
            "SALU / VALU instructions": [], "VALU wave-instructions per ROI voxel": []}
    for k in ks:
        m = med[k]
        cyc = m.get("SQ_BUSY_CYCLES", float("nan")) / 32.0
        rows["kernel cycles (SQ_BUSY_CYCLES / 32)"].append(f"{cyc:.4g}")
        rows["VALU busy (4 x ACTIVE_INST_VALU / (1024 SIMDs x cycles))"].append(
            f"{4.0 * m.get('SQ_ACTIVE_INST_VALU', float('nan')) / (1024.0 * cyc):.2f}")
        rows["LDS bank-conflict cycles per CU / kernel cycles"].append(
            f"{m.get('SQ_LDS_BANK_CONFLICT', float('nan')) / 256.0 / cyc:.2f}")
        rows["LDS address-conflict cycles per CU / kernel cycles"].append(
            f"{m.get('SQ_LDS_ADDR_CONFLICT', float('nan')) / 256.0 / cyc:.2f}")
        rows["SALU / VALU instructions"].append(f"{m.get('SQ_INSTS_SALU', 0.0) / max(m.get('SQ_INSTS_VALU', 1.0), 1.0):.2f}")
        rows["VALU wave-instructions per ROI voxel"].append(f"{m.get('SQ_INSTS_VALU', float('nan')) / roi_vox:.2f}")
    for n, v in rows.items():
        lines.append(f"| {n} | " + " | ".join(v) + " |")
    # named for the dominant kernel (most busy cycles)
    dom = max(ks, key=lambda k: med[k].get("SQ_BUSY_CYCLES", 0.0)) if ks else None
    path = os.path.join(ROOT, "profiles", f"{dom}_{workload}_counters.md") if ks else None
    if path:
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        log(f"wrote {path}")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(w, offs, seconds: float, threads: int) -> tuple:
    """The oracle, as it stands, on whole images of the workload until about
    `seconds` of wall time."""
    import oracle
    off = np.array(offs, np.int32)
    vox, t0, n_img = 0, time.perf_counter(), 0
    for k in range(w.n_images):
        st, _ = oracle.extract(w.intensity[k], w.labels[k], w.n_bins, off, n_threads=threads)
        vox += int(st["count"].sum())
        n_img += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return vox / dt, n_img, vox, dt


def cpu_baseline(w, offs, seconds: float) -> dict:
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rate, n_img, vox, dt = oracle_rate(w, offs, seconds, threads)
    rate1, n1, vox1, dt1 = oracle_rate(w, offs, seconds / 3.0, 1)
    return {"value": rate, "unit": "ROI-voxels/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_img} of {w.n_images} images ({vox} ROI voxels), FP64 oracle, {dt:.1f} s",
            "single_thread": {"value": rate1, "sample": f"{n1} images ({vox1} ROI voxels), {dt1:.1f} s"},
            "cpu_model": cpu_model()}


def oracle_parity(w, offs, table: np.ndarray, n_images: int, prec: int) -> dict:
    """Largest error of the benched feature table against the FP64 oracle over
    every ROI of the first n_images images, under the precision contract's
    measure: |gpu - oracle| / max(|oracle|, M_f), M_f = 1 for CORR, the
    information measures and the entropies (bits), the cluster-shade magnitude
    sum |i + j - mu_x - mu_y|^3 p for cluster shade, 0 otherwise; NaN must
    match NaN."""
    import oracle
    names = oracle.feature_names()
    unit = [n in ("CORR", "INFOMEAS1", "INFOMEAS2", "JE", "ENTROPY", "DIFENTRO", "SUMENT") for n in names]
    shade = names.index("CLUSHADE")
    off = np.array(offs, np.int32)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    row, worst, where, rois = 0, 0.0, None, 0
    n_images = min(n_images, w.n_images)
    for k in range(n_images):
        _, want, mag = oracle.extract(w.intensity[k], w.labels[k], w.n_bins, off, n_threads=threads,
                                      want_shade_magnitude=True)
        got = table[row:row + len(want)].astype(np.float64)
        row += len(want)
        rois += len(want)
        M = np.zeros_like(want)
        M[:, :, np.array(unit)] = 1.0
        mv = np.where(np.isnan(mag), 0.0, mag)
        M[:, :-1, shade] = mv
        cnt = np.maximum((~np.isnan(mag)).sum(axis=1), 1)
        M[:, -1, shade] = mv.sum(axis=1) / cnt
        with np.errstate(divide="ignore", invalid="ignore"):
            err = np.abs(got - want) / np.maximum(np.abs(want), M)
        err = np.where(np.isnan(got) & np.isnan(want), 0.0, err)
        err = np.where(np.isnan(got) != np.isnan(want), np.inf, err)
        err = np.where(got == want, 0.0, err)
        if err.size and float(err.max()) > worst:
            i = np.unravel_index(int(np.argmax(err)), err.shape)
            worst, where = float(err[i]), f"image {k} row {int(i[0])} block {int(i[1])} {names[i[2]]}"
    tol = 1e-12 if prec == 1 else 1e-5
    return {"images": n_images, "rois": rois, "max_error": worst, "at": where, "tolerance": tol,
            "pass": bool(worst <= tol)}


def split_band_voxels(plan, w) -> int:
    """Voxels of the ROIs the plan sends through the band kernel (0 unless the
    description reports any)."""
    from paper_2603_12016_amd import nyx
    fields = dict(kv.split("=", 1) for kv in nyx.nyx_plan_describe(plan).split() if "=" in kv)
    return int(fields.get("band_voxels", 0))


def same_label_pairs(lab, off) -> int:
    """Voxel pairs (v, v + off) inside one ROI (equal nonzero labels); lab is
    a (nz, ny, nx) device tensor."""
    def cut(d, n):
        return (slice(0, max(n - d, 0)), slice(d, n)) if d >= 0 else (slice(-d, n), slice(0, max(n + d, 0)))
    (za, zb), (ya, yb), (xa, xb) = (cut(d, n) for d, n in zip(off, lab.shape))
    a, b = lab[za, ya, xa], lab[zb, yb, xb]
    return int(((a == b) & (a != 0)).sum().item())


# Nested offset sets for the cost grid: each adds offsets to the previous one
# (2D: 0, then 90, then 45 and 135 degrees at distance 1, then the four at 2).
GRID_OFFSETS = ([(0, 0, 1)], [(0, 0, 1), (0, -1, 0)], [(0, 0, 1), (0, -1, 0), (0, -1, 1), (0, -1, -1)],
                [(0, 0, 1), (0, -1, 0), (0, -1, 1), (0, -1, -1), (0, 0, 2), (0, -2, 0), (0, -2, 2), (0, -2, -2)])
GRID_BINS = (8, 16, 32, 64, 128, 256)


def cost_grid(args) -> int:
    """Soft-feature cost grid (Methods, "Feature Control and Tunability",
    Eqs. 2-5): the whole step's time t(p) over an ordered grid of the two GLCM
    hyperparameters, the bin count and a nested set of offsets, on one
    synthetic workload; a soft feature's time never decreases along either
    axis.  Default plans (no autotuning), so that only p changes."""
    import torch
    import synth
    from paper_2603_12016_amd import nyx
    w = synth.make(args.workload)
    dev = torch.device("cuda:0")
    imgs = [(torch.from_numpy(w.intensity[k].view(np.int16)).to(dev),
             torch.from_numpy(w.labels[k].view(np.int32)).to(dev)) for k in range(w.n_images)]
    if w.dims != 2:
        print("the cost grid uses 2D workloads", file=sys.stderr)
        return 2
    ctx = nyx.nyx_create(0)
    grid = []
    for ng in GRID_BINS:
        row = []
        for offs in GRID_OFFSETS:
            plan = nyx.nyx_plan_create(ctx, imgs, ng, offs, nyx.NYX_FP32)
            table = nyx.new_table(plan, len(offs), nyx.NYX_FP32)
            for _ in range(args.warmup):
                nyx.nyx_plan_execute(plan, table)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                nyx.nyx_plan_execute(plan, table)
            torch.cuda.synchronize()
            nyx.nyx_plan_check(plan)
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            row.append(ms)
            log(f"n_bins={ng} offsets={len(offs)}: {ms:.3f} ms ({nyx.nyx_plan_describe(plan).split()[0]})")
            del plan, table
        grid.append(row)
    tol = 0.03   # timing noise allowed before a decrease counts
    down_bins = [(GRID_BINS[i], len(GRID_OFFSETS[j])) for j in range(len(GRID_OFFSETS))
                 for i in range(1, len(GRID_BINS)) if grid[i][j] < grid[i - 1][j] * (1 - tol)]
    down_offs = [(GRID_BINS[i], len(GRID_OFFSETS[j])) for i in range(len(GRID_BINS))
                 for j in range(1, len(GRID_OFFSETS)) if grid[i][j] < grid[i][j - 1] * (1 - tol)]
    print(json.dumps({"metric": "GLCM step time over (n_bins, nested offset sets)", "unit": "ms per step",
                      "workload": args.workload, "roi_voxels": int(np.count_nonzero(w.labels)),
                      "n_bins": list(GRID_BINS), "offsets": [len(o) for o in GRID_OFFSETS],
                      "offset_sets": GRID_OFFSETS, "ms": grid,
                      "decreases_along_bins": down_bins, "decreases_along_offsets": down_offs,
                      "noise_tolerance": tol}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3_batch")
    ap.add_argument("--per-roi-steps", type=int, default=3)
    ap.add_argument("--per-roi-warmup", type=int, default=3)
    ap.add_argument("--parity-images", type=int, default=2,
                    help="images of the benched table compared with the FP64 oracle (untimed)")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--aggregate", choices=("per-offset", "merged"), default="per-offset",
                    help="features per offset and their mean (default), or of the summed matrix")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/*_traffic.txt from rocprofv3 counter CSVs of this script and exit")
    ap.add_argument("--summarize-trace", metavar="STATS_CSV",
                    help="write profiles/<kernel>_<workload>.md from a rocprofv3 kernel_stats.csv and exit")
    ap.add_argument("--summarize-sq", metavar="SQ_CSV",
                    help="write profiles/<kernel>_<workload>_counters.md from a rocprofv3 SQ counter CSV and exit")
    ap.add_argument("--pmc-command", default="", help="the command the profile CSVs came from (recorded)")
    ap.add_argument("--cost-grid", action="store_true",
                    help="time the step over a grid of bin counts x nested offset sets and check that the "
                         "time is monotone along both axes (prints one JSON line)")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload, args.pmc_command)
        return 0
    if args.summarize_sq:
        import synth
        summarize_sq(args.summarize_sq, args.workload, args.pmc_command,
                     int(np.count_nonzero(synth.make(args.workload).labels)))
        return 0
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, COPY_BYTES, args.pmc_command)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU: the path runs on one GPU and several GPUs are not supported (use --gpus 1)",
              file=sys.stderr)
        return 2

    import torch
    if args.cost_grid:
        return cost_grid(args)

    import synth
    from paper_2603_12016_amd import nyx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    w = synth.make(args.workload)
    log(f"generated {args.workload} in {time.perf_counter() - t0:.1f} s")
    # inputs to HBM from pinned host memory, timed apart from the step
    host = [(torch.from_numpy(w.intensity[k].view(np.int16)).pin_memory(),
             torch.from_numpy(w.labels[k].view(np.int32)).pin_memory()) for k in range(w.n_images)]
    imgs = [(torch.empty_like(i, device=dev), torch.empty_like(l, device=dev)) for i, l in host]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (di, dl), (hi, hl) in zip(imgs, host):
        di.copy_(hi, non_blocking=True)
        dl.copy_(hl, non_blocking=True)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    in_bytes = sum(i.numel() * 2 + l.numel() * 4 for i, l in host)
    del host
    log(f"inputs to device: {in_bytes / 1e9:.2f} GB in {h2d_s * 1e3:.1f} ms")
    offs = nyx.nyx_offsets_default(w.dims, 1)
    K = len(offs)
    prec = nyx.NYX_FP64 if w.precision == "fp64" else nyx.NYX_FP32
    ctx = nyx.nyx_create(0)
    t0 = time.perf_counter()
    agg = nyx.NYX_AGG_MERGED if args.aggregate == "merged" else nyx.NYX_AGG_PER_OFFSET
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, prec, autotune=not args.no_autotune, aggregate=agg)
    plan_s = time.perf_counter() - t0
    log(f"plan in {plan_s:.2f} s: {nyx.nyx_plan_describe(plan)}")
    n_rois = plan.n_rois
    roi_vox = int(np.count_nonzero(w.labels))
    img_vox = int(w.labels.size)
    table = nyx.new_table(plan, K, prec, aggregate=agg)

    for _ in range(args.warmup):
        nyx.nyx_plan_execute(plan, table)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    log(f"warmup done ({args.warmup} steps)")
    # events between replays, on the stream the graph is launched on
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        nyx.nyx_plan_execute(plan, table)
        evs[k + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nyx.nyx_plan_check(plan)
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    ms = dt * 1e3 / args.steps
    value = roi_vox / (dt / args.steps)
    log(f"batched: {ms:.3f} ms/step (median {np.median(step_ms):.3f}, min {min(step_ms):.3f}), "
        f"{value / 1e9:.2f} G ROI-voxels/s")

    # phase times of the same step, eager, with HIP events between phases
    prof = {p: 0.0 for p in nyx.PHASES}
    for _ in range(args.profile_steps):
        r = nyx.nyx_plan_profile(plan, table)
        for p in prof:
            prof[p] += r[p] / args.profile_steps
    log("phases (ms): " + ", ".join(f"{p}={v:.4f}" for p, v in prof.items()))

    # the benched table against the oracle on whole images (untimed)
    parity = None
    if args.parity_images > 0 and agg == nyx.NYX_AGG_PER_OFFSET:
        parity = oracle_parity(w, offs, table.cpu().numpy(), args.parity_images, prec)
        log(f"parity vs oracle: {parity}")

    # one launch per ROI
    dt_roi, same = None, None
    if args.per_roi_steps > 0:
        t2 = nyx.new_table(plan, K, prec, aggregate=agg)
        for _ in range(args.per_roi_warmup):
            nyx.nyx_plan_execute_per_roi(plan, t2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.per_roi_steps):
            nyx.nyx_plan_execute_per_roi(plan, t2)
        torch.cuda.synchronize()
        dt_roi = (time.perf_counter() - t0) / args.per_roi_steps
        nyx.nyx_plan_check(plan)
        same = bool(torch.allclose(table, t2, rtol=1e-5, atol=1e-6, equal_nan=True))
        log(f"per-ROI launches: {dt_roi * 1e3:.1f} ms/step ({args.per_roi_warmup} warm-up, "
            f"{args.per_roi_steps} timed), tables agree: {same}")

    # algorithmic bytes: the scan reads 4 B label + 2 B intensity per image
    # voxel; each accumulate/feature kernel reads 4 B label + 2 B intensity per
    # voxel of the ROIs it owns and writes their feature rows.
    row_bytes = nyx.table_blocks(K, agg) * 30 * (8 if prec == nyx.NYX_FP64 else 4)
    out_bytes = n_rois * row_bytes
    # the band kernel reads the voxels of the split ROIs whose triangle exceeds LDS
    band_vox = split_band_voxels(plan, w)
    alg = {"scan": img_vox * 6.0,
           "batch": (roi_vox - band_vox) * 6.0 + n_rois * row_bytes,
           "band": band_vox * 6.0}
    kernel_names = {"scan": "k_scan", "batch": "k_batch", "band": "k_band"}
    dom = max(("scan", "batch", "band"), key=lambda p: prof[p])
    achieved = alg[dom] / (prof[dom] * 1e-3) / 1e9
    step_alg = img_vox * 4.0 + roi_vox * 2.0 + out_bytes

    # same-ROI neighbour pairs = LDS atomics of the accumulation
    pairs = sum(same_label_pairs(lab, o) for _, lab in imgs for o in offs)
    machine = {}
    try:
        from paper_2603_12016_amd import micro
        machine = {"copy_GBps": micro.copy_bandwidth(COPY_BYTES)["GBps"], "read_GBps": micro.read_bandwidth()["GBps"],
                   "lds_atomics_per_s": micro.lds_atomic_rate()["per_second"]}
        log("machine: " + ", ".join(f"{k}={v:.4g}" for k, v in machine.items()))
    except (ImportError, OSError, RuntimeError) as e:
        log(f"machine ceilings not measured: {e}")

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
                   "offsets": K, "aggregate": args.aggregate, "plan": nyx.nyx_plan_describe(plan)},
        "per_roi_launch": None if dt_roi is None else {"value": roi_vox / dt_roi, "ms_per_step": dt_roi * 1e3,
                                                       "steps": args.per_roi_steps, "tables_agree": same},
        "speedup_vs_per_roi": None if dt_roi is None else dt_roi * 1e3 / ms,
        "step_hbm_frac_alg": step_alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "ms_median": float(np.median(step_ms)),
        "ms_min": float(min(step_ms)),
        "phases_ms": prof,
        "inputs_h2d": {"bytes": in_bytes, "seconds": h2d_s, "GBps": in_bytes / h2d_s / 1e9,
                       "value_incl_h2d": roi_vox / (h2d_s + dt / args.steps)},
        "lds_atomics": {"pairs_per_step": pairs,
                        "achieved_per_s": pairs / (sum(prof[p] for p in ("batch", "band", "split")) * 1e-3)},
        "machine": machine,
        "roofline": {"kernel": kernel_names[dom], "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic(kernel_names[dom], args.workload) if agg == nyx.NYX_AGG_PER_OFFSET
                     else None,
                     "alg_bytes": alg[dom], "ms": prof[dom]},
        "plan_seconds": plan_s,
        "parity_vs_oracle": parity,
    }
    if not args.no_cpu_baseline and agg == nyx.NYX_AGG_MERGED:
        log("cpu baseline skipped: the oracle's timed extraction is the per-offset one")
    elif not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(w, offs, args.cpu_seconds)
        log(f"cpu baseline: {rec['cpu_baseline']['value'] / 1e6:.2f} M ROI-voxels/s")
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
