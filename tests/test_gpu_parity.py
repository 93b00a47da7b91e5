"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Counts, ROI tables and bin images must match bit for bit; features must meet
the precision contract (1e-12 for the FP64 table, 1e-5 for the FP32 table,
error measure in gpu_util).
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

from gpu_util import (NAMES, device_images, feature_errors, oracle_rois, record, scales,
                      scales_from_magnitudes, worst)

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_FP64 = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2603_12016_amd import nyx
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    return nyx, nyx.nyx_create(0), dev


@pytest.fixture(scope="module")
def workloads(synth_mod):
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = synth_mod.make(name)
        return cache[name]
    return get


def _offsets(nyx, w):
    return nyx.nyx_offsets_default(w.dims, 1)


def _oracle_table(oracle, w, offs, rows=None):
    """Oracle table for all ROIs (or a subset of global rows)."""
    off = np.array(offs, np.int32)
    out, Ps = [], []
    ro = oracle_rois(oracle, w)
    sel = range(len(ro)) if rows is None else rows
    for g in sel:
        k, r, st = ro[g]
        P = oracle.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                            st["bbox"][r], w.n_bins, off)
        out.append(oracle.features_roi(P))
        Ps.append(P)
    return np.array(out), Ps


def _check_scaled(got, want, M, tol, tag):
    """got, want: (n, blocks, 30); M: (n, blocks, 30) error floors."""
    assert got.shape == want.shape, (got.shape, want.shape)
    if len(want) == 0:
        return
    errs = feature_errors(got, want, M)
    record(tag, errs, got, want, len(want), tol)
    e, name, idx = worst(errs)
    say(f"  {tag}: {len(want)} ROIs, max error {e:.3e} ({name} at {idx})")
    assert e <= tol, (tag, name, idx, got[idx[0], idx[1]], want[idx[0], idx[1]])


def _check_features(got, want, Ps, tol, tag):
    assert got.shape == want.shape, (got.shape, want.shape)
    if len(Ps) == 0:
        return
    _check_scaled(got, want, np.stack([scales(P) for P in Ps]), tol, tag)


# ------------------------------------------------------------------ C1
def test_c1_fp64_extract_batch(env, workloads, oracle_mod):
    nyx, ctx, dev = env
    w = workloads("c1_tiny")
    say("case c1_tiny extract_batch fp64")
    offs = _offsets(nyx, w)
    rois, table = nyx.nyx_extract_batch(ctx, device_images(w, dev), w.n_bins, offs, nyx.NYX_FP64)
    import torch
    torch.cuda.synchronize()
    want, Ps = _oracle_table(oracle_mod, w, offs)
    _check_features(table.cpu().numpy(), want, Ps, TOL_FP64, "c1 fp64")
    assert rois.n_rois == 1


# ------------------------------------------------------------------ ROI table / bins
SMALL = ["c2_small", "c3_small", "c4_small", "c5_small"]


@pytest.mark.parametrize("name", SMALL + ["c1_tiny"])
def test_roi_table_and_bins_exact(env, workloads, oracle_mod, name):
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} bin_rois")
    rois, bins = nyx.nyx_bin_rois(ctx, device_images(w, dev), w.n_bins, want_bins=True)
    n = rois.n_rois
    ro = oracle_rois(oracle_mod, w)
    assert n == len(ro)
    lab = rois.label.cpu().numpy()[:n].view(np.uint32)
    img = rois.image.cpu().numpy()[:n]
    cnt = rois.n_vox.cpu().numpy()[:n]
    vmin = rois.vmin.cpu().numpy()[:n].view(np.uint16)
    vmax = rois.vmax.cpu().numpy()[:n].view(np.uint16)
    bbox = rois.bbox.cpu().numpy()[:n]
    for g, (k, r, st) in enumerate(ro):
        assert img[g] == k and lab[g] == st["label"][r] and cnt[g] == st["count"][r]
        assert vmin[g] == st["vmin"][r] and vmax[g] == st["vmax"][r]
        assert np.array_equal(bbox[g], st["bbox"][r])
    got_bins = bins.cpu().numpy().view(np.uint16)
    off = 0
    for k in range(w.n_images):
        want = oracle_mod.bin_image(w.intensity[k], w.labels[k], w.n_bins)
        sz = want.size
        assert np.array_equal(got_bins[off:off + sz].reshape(want.shape), want), f"image {k}"
        off += sz


# ------------------------------------------------------------------ counts
def _dense_from_coo(g, n_rois, K, ng):
    keys = g.keys.cpu().numpy().view(np.uint64)
    cnt = g.counts.cpu().numpy().view(np.uint64)
    assert np.all(keys[1:] > keys[:-1]), "COO keys not strictly sorted"
    U = np.zeros((n_rois, K, ng, ng), np.uint64)
    roi = (keys >> np.uint64(38)).astype(np.int64)
    d = ((keys >> np.uint64(32)) & np.uint64(63)).astype(np.int64)
    i = ((keys >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    j = (keys & np.uint64(0xFFFF)).astype(np.int64)
    assert np.all(i <= j) and np.all(cnt > 0)
    U[roi, d, i, j] = cnt
    return U


def _triangle(P):
    U = np.triu(P).copy()
    idx = np.arange(P.shape[-1])
    U[..., idx, idx] //= 2
    return U


@pytest.mark.parametrize("name", ["c1_tiny", "c2_small", "c3_small", "c4_small", "c5_small"])
@pytest.mark.parametrize("use_bins", [False, True])
def test_glcm_counts_exact(env, workloads, oracle_mod, name, use_bins):
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} glcm_accumulate bins={use_bins}")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    rois, bins = nyx.nyx_bin_rois(ctx, imgs, w.n_bins, want_bins=use_bins)
    g = nyx.nyx_glcm_accumulate(ctx, imgs, rois, w.n_bins, offs, bins=bins)
    ro = oracle_rois(oracle_mod, w)
    assert g.n_rois == len(ro)
    if w.n_bins > 256:
        # compare ROI by ROI without a dense 4D array
        keys = g.keys.cpu().numpy().view(np.uint64)
        cnt = g.counts.cpu().numpy().view(np.uint64)
        roi = (keys >> np.uint64(38)).astype(np.int64)
        for gi in list(range(0, len(ro), max(1, len(ro) // 25))) + [len(ro) - 1]:
            k, r, st = ro[gi]
            P = oracle_mod.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                                    st["bbox"][r], w.n_bins, np.array(offs, np.int32))
            U = _triangle(P)
            sel = roi == gi
            kk = keys[sel]
            d = ((kk >> np.uint64(32)) & np.uint64(63)).astype(np.int64)
            i = ((kk >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
            j = (kk & np.uint64(0xFFFF)).astype(np.int64)
            nz = np.nonzero(U)
            assert len(kk) == len(nz[0]), gi
            assert np.array_equal(U[d, i, j], cnt[sel]), gi
        return
    U = _dense_from_coo(g, len(ro), len(offs), w.n_bins)
    for gi, (k, r, st) in enumerate(ro):
        P = oracle_mod.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                                st["bbox"][r], w.n_bins, np.array(offs, np.int32))
        assert np.array_equal(U[gi], _triangle(P)), f"ROI {gi}"


# ------------------------------------------------------------------ features from oracle counts
@pytest.mark.parametrize("name,prec", [("c1_tiny", 1), ("c2_small", 0), ("c3_small", 1), ("c4_small", 0),
                                       ("c5_small", 0)])
def test_features_from_oracle_coo(env, workloads, oracle_mod, name, prec):
    import torch
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} glcm_features from oracle COO prec={prec}")
    offs = _offsets(nyx, w)
    K = len(offs)
    ro = oracle_rois(oracle_mod, w)
    keys, cnts, Ps = [], [], []
    for gi, (k, r, st) in enumerate(ro):
        P = oracle_mod.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                                st["bbox"][r], w.n_bins, np.array(offs, np.int32))
        Ps.append(P)
        U = _triangle(P)
        d, i, j = np.nonzero(U)
        keys.append((np.uint64(gi) << np.uint64(38)) | (d.astype(np.uint64) << np.uint64(32)) |
                    (i.astype(np.uint64) << np.uint64(16)) | j.astype(np.uint64))
        cnts.append(U[d, i, j])
    keys = np.concatenate(keys)
    cnts = np.concatenate(cnts).astype(np.uint64)
    order = np.argsort(keys)
    kt = torch.from_numpy(keys[order].view(np.int64)).to(dev)
    ct = torch.from_numpy(cnts[order].view(np.int64)).to(dev)
    g = nyx.Glcm(kt, ct, int(len(keys)), w.n_bins, K, len(ro))
    table = nyx.nyx_glcm_features(ctx, g, prec)
    torch.cuda.synchronize()
    want = np.array([oracle_mod.features_roi(P) for P in Ps])
    _check_features(table.cpu().numpy(), want, Ps, TOL_FP64 if prec == 1 else TOL_FP32, f"{name} coo")


# ------------------------------------------------------------------ batched path
# (workload, accumulation mode, privatised triangle copies: 0 automatic)
MODE_CASES = ([(n, m, 0) for n in SMALL for m in ("auto", "dense-list", "dense-scan", "dense16-scan")
               if not (n == "c5_small" and m != "auto")] +
              [(n, m, c) for n in ("c2_small", "c3_small", "c4_small") for m in ("dense-scan", "dense16-scan")
               for c in (2, 4)] + [("c3_small", "autotune", 0)])


@pytest.mark.parametrize("name,mode,copies", MODE_CASES)
def test_plan_batched_and_per_roi(env, workloads, oracle_mod, name, mode, copies):
    import torch
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} plan_execute + per_roi, mode {mode}, copies {copies}")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    if mode == "autotune":
        plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, nyx.NYX_FP32, autotune=True)
    else:
        try:
            plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, nyx.NYX_FP32, mode=mode, copies=copies)
        except nyx.NyxError as e:
            if e.status == nyx.NYX_ERR_UNSUPPORTED:
                pytest.skip(f"{mode} with {copies} copies does not fit LDS for {name}")
            raise
    desc = nyx.nyx_plan_describe(plan)
    say("  plan:", desc)
    if copies > 0:
        assert f"copies={copies} " in desc
    t1 = nyx.new_table(plan, len(offs))
    t2 = nyx.new_table(plan, len(offs))
    want, Ps = _oracle_table(oracle_mod, w, offs)
    replays = []
    for rep in range(3):
        # every replay writes the whole table: it starts from NaN, so a row a
        # replay leaves unwritten cannot pass as a copy of an earlier replay
        t1.fill_(float("nan"))
        nyx.nyx_plan_execute(plan, t1)
        torch.cuda.synchronize()   # eager work between the replays
        nyx.nyx_plan_check(plan)
        replays.append(t1.cpu().numpy()[:plan.n_rois].copy())
        _check_features(replays[-1], want, Ps, TOL_FP32, f"{name} batched")
    nyx.nyx_plan_execute_per_roi(plan, t2)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    per_roi = t2.cpu().numpy()[:plan.n_rois]
    _check_features(per_roi, want, Ps, TOL_FP32, f"{name} per-roi")
    for rep in range(1, 3):
        assert np.allclose(replays[0], replays[rep], rtol=1e-6, atol=1e-6, equal_nan=True), rep
    if "scan" in desc:
        # ordered nonzero lists: every replay and the per-ROI path agree with
        # the first replay bit for bit
        for rep in range(1, 3):
            assert np.array_equal(replays[0], replays[rep], equal_nan=True), f"replay {rep}"
        assert np.array_equal(replays[0], per_roi, equal_nan=True)


@pytest.mark.parametrize("name,mode,prec", [("c2_small", "dense-list", 0), ("c2_small", "dense-list", 1),
                                            ("c2_small", "dense-scan", 0), ("c5_small", "auto", 0)])
def test_wide_work_groups(env, workloads, oracle_mod, name, mode, prec):
    """Layouts that leave LDS for one work-group per CU run 512-thread
    work-groups (eight waves sharing the item's LDS): the plan says so, and the
    batched and per-ROI tables match the oracle."""
    import torch
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} 512-thread work-groups, mode {mode}, prec {prec}")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    kw = {} if mode == "auto" else {"mode": mode}
    precision = nyx.NYX_FP64 if prec else nyx.NYX_FP32
    tol = TOL_FP64 if prec else TOL_FP32
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, precision, **kw)
    desc = nyx.nyx_plan_describe(plan)
    say("  plan:", desc)
    assert "block=512 " in desc
    want, Ps = _oracle_table(oracle_mod, w, offs)
    t = nyx.new_table(plan, len(offs), precision)
    nyx.nyx_plan_execute(plan, t)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    _check_features(t.cpu().numpy()[:plan.n_rois], want, Ps, tol, f"{name} wide batched")
    t.fill_(float("nan"))
    nyx.nyx_plan_execute_per_roi(plan, t)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    _check_features(t.cpu().numpy()[:plan.n_rois], want, Ps, tol, f"{name} wide per-roi")


# ------------------------------------------------------------------ edge cases
def _run_extract(nyx, ctx, dev, I, L, ng, offs, prec=1, copies=0):
    from types import SimpleNamespace
    w = SimpleNamespace(intensity=I[None], labels=L[None], n_images=1)
    return nyx.nyx_extract_batch(ctx, device_images(w, dev), ng, offs, prec, copies=copies)


def _oracle_direct(oracle, I, L, ng, offs):
    st, t = oracle.extract(I, L, ng, np.array(offs, np.int32))
    Ps = [oracle.glcm_roi(I, L, st["label"][r], st["vmin"][r], st["vmax"][r], st["bbox"][r], ng,
                          np.array(offs, np.int32)) for r in range(st["label"].size)]
    return t, Ps


EDGE = {
    "ragged_many_labels": lambda rng: (rng.integers(0, 3000, (1, 37, 53)), rng.integers(0, 40, (1, 37, 53))),
    "single_voxels": lambda rng: (rng.integers(0, 3000, (1, 9, 9)), np.where(rng.random((1, 9, 9)) < 0.3,
                                                                           np.arange(81).reshape(1, 9, 9) + 1, 0)),
    "thin_lines": lambda rng: (rng.integers(0, 3000, (1, 20, 21)), np.tile(np.arange(21) % 3 == 0, (1, 20, 1)) *
                               (np.arange(21) + 1)),
    "big_labels": lambda rng: (rng.integers(0, 65535, (1, 16, 24)), np.where(rng.random((1, 16, 24)) < 0.8,
                                                                            1_000_000 + rng.integers(0, 3, (1, 16, 24)), 0)),
    "constant": lambda rng: (np.full((1, 12, 10), 777), np.ones((1, 12, 10))),
    "border_touching_3d": lambda rng: (rng.integers(0, 4096, (5, 6, 7)), rng.integers(1, 3, (5, 6, 7))),
}


@pytest.mark.parametrize("copies", [1, 2])
@pytest.mark.parametrize("case", sorted(EDGE))
@pytest.mark.parametrize("ng", [2, 8, 30, 100])
def test_edge_cases(env, oracle_mod, case, ng, copies):
    import torch
    nyx, ctx, dev = env
    rng = np.random.default_rng(sum(map(ord, case)) % 1000 + ng)
    I, L = EDGE[case](rng)
    I = np.ascontiguousarray(I, np.uint16)
    L = np.ascontiguousarray(L, np.uint32)
    dims = 3 if I.shape[0] > 1 else 2
    offs = nyx.nyx_offsets_default(dims, 1)
    say(f"case edge {case} ng={ng} copies={copies}")
    rois, table = _run_extract(nyx, ctx, dev, I, L, ng, offs, copies=copies)
    torch.cuda.synchronize()
    want, Ps = _oracle_direct(oracle_mod, I, L, ng, offs)
    assert rois.n_rois == len(Ps)
    _check_features(table.cpu().numpy(), want, Ps, TOL_FP64, f"edge {case}")


def test_empty_image(env):
    nyx, ctx, dev = env
    I = np.zeros((1, 8, 8), np.uint16)
    L = np.zeros((1, 8, 8), np.uint32)
    rois, table = _run_extract(nyx, ctx, dev, I, L, 8, nyx.nyx_offsets_default(2, 1))
    assert rois.n_rois == 0 and table.shape[0] == 0


_OFF3 = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 1), (0, 1, -1), (1, 0, 1), (1, 0, -1), (1, 1, 0), (1, -1, 0),
         (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)]


# 2D offsets outside the four distance-1 classes, and 3D offsets (given
# backwards, at distance 2, or few): the staged and gather accumulations.
@pytest.mark.parametrize("offs,shape", [([(0, 0, 2), (0, -2, 2), (0, -2, 0), (0, -2, -2)], (1, 30, 31)),
                                        ([(0, 1, 3), (0, 0, -1), (0, 2, 0)], (1, 30, 31)),
                                        ([(0, 0, -1), (0, 1, 1), (0, 1, 0), (0, 1, -1)], (1, 30, 31)),
                                        ([(-a, -b, -c) for a, b, c in _OFF3], (7, 19, 23)),
                                        ([(2 * a, 2 * b, 2 * c) for a, b, c in _OFF3], (9, 17, 15)),
                                        ([(1, 0, 0), (0, -1, 2), (-2, 1, 1)], (8, 12, 40))])
def test_other_offsets(env, oracle_mod, offs, shape):
    import torch
    nyx, ctx, dev = env
    rng = np.random.default_rng(len(offs) + shape[0])
    I = rng.integers(0, 4000, shape).astype(np.uint16)
    L = (rng.integers(1, 5, shape) * (rng.random(shape) < 0.9)).astype(np.uint32)
    say(f"case offsets {offs}")
    rois, table = _run_extract(nyx, ctx, dev, I, L, 16, offs)
    torch.cuda.synchronize()
    want, Ps = _oracle_direct(oracle_mod, I, L, 16, offs)
    _check_features(table.cpu().numpy(), want, Ps, TOL_FP64, "offsets")


def test_checkerboard_closed_form(env):
    import math
    import torch
    nyx, ctx, dev = env
    y, x = np.mgrid[0:8, 0:8]
    I = (((x + y) % 2) * 4095).astype(np.uint16)[None]
    L = np.ones((1, 8, 8), np.uint32)
    rois, table = _run_extract(nyx, ctx, dev, I, L, 8, nyx.nyx_offsets_default(2, 1))
    t = table.cpu().numpy()[0]
    f = dict(zip(NAMES, t[0]))
    assert f["CONTRAST"] == pytest.approx(49.0, rel=1e-14)
    assert f["CORR"] == pytest.approx(-1.0, rel=1e-14)
    assert f["INFOMEAS2"] == pytest.approx(math.sqrt(1 - math.exp(-2)), rel=1e-13)
    assert t[4][NAMES.index("CONTRAST")] == pytest.approx(24.5, rel=1e-14)


# ------------------------------------------------------------------ argument errors
def test_invalid_arguments(env):
    nyx, ctx, dev = env
    from types import SimpleNamespace
    I = np.zeros((1, 8, 8), np.uint16)
    L = np.ones((1, 8, 8), np.uint32)
    w = SimpleNamespace(intensity=I[None], labels=L[None], n_images=1)
    imgs = device_images(w, dev)
    for ng, offs, code in [(1, [(0, 0, 1)], nyx.NYX_ERR_INVALID), (70000, [(0, 0, 1)], nyx.NYX_ERR_INVALID),
                           (8, [(0, 0, 0)], nyx.NYX_ERR_INVALID), (8, [(1, 0, 0)], nyx.NYX_ERR_INVALID),
                           (8, [], nyx.NYX_ERR_INVALID), (9000, [(0, 0, 1)], nyx.NYX_ERR_UNSUPPORTED)]:
        with pytest.raises(nyx.NyxError) as e:
            nyx.nyx_plan_create(ctx, imgs, ng, offs)
        assert e.value.status == code, (ng, offs)
    with pytest.raises(nyx.NyxError) as e:
        nyx.nyx_extract_batch(ctx, imgs, 8, [(0, 0, 1)], capacity=0)
    assert e.value.status == nyx.NYX_ERR_CAPACITY


# ------------------------------------------------------------------ full sizes (sampled)
@pytest.mark.parametrize("name", ["c2_cells", "c3_batch", "c4_3d", "c5_stress"])
def test_full_size_sampled(env, workloads, oracle_mod, name):
    import torch
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} full size: autotuned plan (as the benchmark) + execute")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, nyx.NYX_FP32, autotune=True)
    say("  plan:", nyx.nyx_plan_describe(plan))
    table = nyx.new_table(plan, len(offs))
    rois = nyx.RoiTable(plan.n_rois, dev)
    nyx.nyx_plan_execute(plan, table, rois)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    ro = oracle_rois(oracle_mod, w)
    assert plan.n_rois == len(ro)
    n = np.array([st["count"][r] for _, r, st in ro])
    assert np.array_equal(rois.n_vox.cpu().numpy()[:len(ro)], n)
    rng = np.random.default_rng(7)
    order = np.argsort(n)
    sample = sorted(set([int(order[0]), int(order[-1]), int(order[len(order) // 2])] +
                        rng.choice(len(ro), size=min(20, len(ro)), replace=False).tolist()))
    want, Ps = _oracle_table(oracle_mod, w, offs, rows=sample)
    got = table.cpu().numpy()[sample]
    _check_features(got, want, Ps, TOL_FP32, f"{name} sampled")
    tab = table.cpu().numpy()[:len(ro)]
    assert np.all(np.isfinite(tab[n >= 4][:, -1, 0]))


# ------------------------------------------------------------------ full sizes (every row / giant ROI)
def _host_threads() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


@pytest.mark.timeout(600)
def test_c3_full_table_every_roi(env, workloads, oracle_mod):
    """The benchmark's configuration (64-image batch, autotuned plan, graph
    replay) against the oracle on every ROI and every feature column."""
    import torch
    nyx, ctx, dev = env
    w = workloads("c3_batch")
    say("case c3_batch full table: autotuned plan + execute, every ROI against the oracle")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, nyx.NYX_FP32, autotune=True)
    say("  plan:", nyx.nyx_plan_describe(plan))
    table = nyx.new_table(plan, len(offs))
    table.fill_(float("nan"))
    nyx.nyx_plan_execute(plan, table)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    got = table.cpu().numpy()[:plan.n_rois]
    off = np.array(offs, np.int32)
    threads = _host_threads()
    wants, mags = [], []
    for k in range(w.n_images):
        _, t, mag = oracle_mod.extract(w.intensity[k], w.labels[k], w.n_bins, off, n_threads=threads,
                                       want_shade_magnitude=True)
        wants.append(t)
        mags.append(mag)
    want = np.concatenate(wants)
    M = np.stack([scales_from_magnitudes(m) for m in np.concatenate(mags)])
    assert got.shape == want.shape, (got.shape, want.shape)
    _check_scaled(got, want, M, TOL_FP32, "c3_batch every ROI")


@pytest.mark.timeout(600)
def test_c5_full_counts_exact(env, workloads, oracle_mod):
    """64-bit counts of the 1024-level stress tile at full size: the giant
    ROI (90 % of the tile) and a sample of the small ROIs, bit for bit."""
    nyx, ctx, dev = env
    w = workloads("c5_stress")
    say("case c5_stress full size: glcm_accumulate, giant ROI + sampled small ROIs")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    rois, _ = nyx.nyx_bin_rois(ctx, imgs, w.n_bins)
    g = nyx.nyx_glcm_accumulate(ctx, imgs, rois, w.n_bins, offs)
    ro = oracle_rois(oracle_mod, w)
    assert g.n_rois == len(ro)
    keys = g.keys.cpu().numpy().view(np.uint64)
    cnt = g.counts.cpu().numpy().view(np.uint64)
    assert np.all(keys[1:] > keys[:-1]), "COO keys not strictly sorted"
    roi = (keys >> np.uint64(38)).astype(np.int64)
    n = np.array([st["count"][r] for _, r, st in ro])
    giant = int(np.argmax(n))
    rng = np.random.default_rng(11)
    sample = sorted({giant, 0, len(ro) - 1, *rng.choice(len(ro), size=40, replace=False).tolist()})
    start = np.searchsorted(roi, np.arange(len(ro) + 1))
    for gi in sample:
        k, r, st = ro[gi]
        P = oracle_mod.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                                st["bbox"][r], w.n_bins, np.array(offs, np.int32))
        U = _triangle(P)
        kk, cc = keys[start[gi]:start[gi + 1]], cnt[start[gi]:start[gi + 1]]
        d = ((kk >> np.uint64(32)) & np.uint64(63)).astype(np.int64)
        i = ((kk >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
        j = (kk & np.uint64(0xFFFF)).astype(np.int64)
        assert len(kk) == np.count_nonzero(U), (gi, len(kk), np.count_nonzero(U))
        assert np.array_equal(U[d, i, j], cc), gi
        if gi == giant:
            say(f"  giant ROI {gi}: {int(n[gi])} voxels, {len(kk)} nonzero cells, "
                f"largest count {int(cc.max())}, bit-exact")
    say(f"  {len(sample)} ROIs bit-exact")


# ------------------------------------------------------------------ merged matrices
# NYX_AGG_MERGED: the features of the sum of the offsets' matrices, one block
# per row, through the one-shot call, the plan and the per-ROI launches.
@pytest.mark.parametrize("name,prec", [("c1_tiny", 1), ("c2_small", 0), ("c3_small", 0), ("c3_small", 1),
                                       ("c4_small", 0)])
def test_merged_matrices(env, workloads, oracle_mod, name, prec):
    import torch
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} merged prec={prec}")
    offs = _offsets(nyx, w)
    imgs = device_images(w, dev)
    rois, t0 = nyx.nyx_extract_batch(ctx, imgs, w.n_bins, offs, prec, aggregate=nyx.NYX_AGG_MERGED)
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, prec, aggregate=nyx.NYX_AGG_MERGED)
    say("  plan:", nyx.nyx_plan_describe(plan))
    t1 = nyx.new_table(plan, len(offs), prec, aggregate=nyx.NYX_AGG_MERGED)
    t2 = nyx.new_table(plan, len(offs), prec, aggregate=nyx.NYX_AGG_MERGED)
    nyx.nyx_plan_execute(plan, t1)
    nyx.nyx_plan_execute_per_roi(plan, t2)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    off = np.array(offs, np.int32)
    want, M = [], []
    for k, r, st in oracle_rois(oracle_mod, w):
        P = oracle_mod.glcm_roi(w.intensity[k], w.labels[k], st["label"][r], st["vmin"][r], st["vmax"][r],
                                st["bbox"][r], w.n_bins, off)
        want.append(oracle_mod.features_roi_merged(P))
        M.append(scales(P.sum(axis=0, dtype=np.uint64)[None])[:1])
    want = np.array(want)
    tol = TOL_FP64 if prec == 1 else TOL_FP32
    for tag, got in (("one-shot", t0), ("plan", t1), ("per-roi", t2)):
        got = got.cpu().numpy()[:len(want)]
        assert got.shape == want.shape, (tag, got.shape, want.shape)
        e, fname, idx = worst(np.stack([feature_errors(got[i], want[i], M[i]) for i in range(len(want))]))
        say(f"  {name} merged {tag}: {len(want)} ROIs, max error {e:.3e} ({fname} at {idx})")
        assert e <= tol, (tag, fname, idx)


def test_merged_needs_a_triangle_in_lds(env):
    # 1024 levels: one 32-bit triangle is 2 MB, beyond LDS
    nyx, ctx, dev = env
    rng = np.random.default_rng(4)
    I = rng.integers(0, 4000, (1, 40, 40)).astype(np.uint16)
    L = np.ones((1, 40, 40), np.uint32)
    with pytest.raises(nyx.NyxError) as e:
        _run_extract_merged(nyx, ctx, dev, I, L, 1024)
    assert e.value.status == nyx.NYX_ERR_UNSUPPORTED


def test_merged_checkerboard_closed_form(env):
    import torch
    nyx, ctx, dev = env
    y, x = np.mgrid[0:8, 0:8]
    I = (((x + y) % 2) * 4095).astype(np.uint16)[None]
    L = np.ones((1, 8, 8), np.uint32)
    rois, table = _run_extract_merged(nyx, ctx, dev, I, L, 8)
    f = dict(zip(NAMES, table.cpu().numpy()[0, 0]))
    assert table.shape == (1, 1, 30)
    assert f["CONTRAST"] == pytest.approx(392 / 15, rel=1e-14)
    assert f["DIS"] == pytest.approx(56 / 15, rel=1e-14)


def _run_extract_merged(nyx, ctx, dev, I, L, ng):
    from types import SimpleNamespace
    w = SimpleNamespace(intensity=I[None], labels=L[None], n_images=1)
    return nyx.nyx_extract_batch(ctx, device_images(w, dev), ng, nyx.nyx_offsets_default(2, 1), nyx.NYX_FP64,
                                 aggregate=nyx.NYX_AGG_MERGED)


@pytest.mark.parametrize("offs,shape", [([(2 * a, 2 * b, 2 * c) for a, b, c in _OFF3], (9, 17, 15)),
                                        ([(0, 0, 2), (0, -2, 2), (0, -2, 0), (0, -2, -2), (0, 0, 1)], (1, 30, 31))])
def test_merged_other_offsets(env, oracle_mod, offs, shape):
    # merged matrices through the staged accumulation (3D distance 2; a 2D
    # set mixing distances 1 and 2)
    import torch
    from types import SimpleNamespace
    nyx, ctx, dev = env
    rng = np.random.default_rng(len(offs) + 7 * shape[0])
    I = rng.integers(0, 4000, shape).astype(np.uint16)
    L = (rng.integers(1, 5, shape) * (rng.random(shape) < 0.9)).astype(np.uint32)
    say(f"case merged offsets {offs}")
    w = SimpleNamespace(intensity=I[None], labels=L[None], n_images=1)
    rois, table = nyx.nyx_extract_batch(ctx, device_images(w, dev), 16, offs, nyx.NYX_FP64,
                                        aggregate=nyx.NYX_AGG_MERGED)
    torch.cuda.synchronize()
    off = np.array(offs, np.int32)
    st = oracle_mod.roi_stats(I, L)
    got = table.cpu().numpy()
    assert got.shape == (st["label"].size, 1, 30)
    for r in range(st["label"].size):
        P = oracle_mod.glcm_roi(I, L, st["label"][r], st["vmin"][r], st["vmax"][r], st["bbox"][r], 16, off)
        want = oracle_mod.features_roi_merged(P)
        e = feature_errors(got[r], want, scales(P.sum(axis=0, dtype=np.uint64)[None])[:1])
        assert np.max(e) <= TOL_FP64, (r, NAMES[int(np.argmax(e[0]))], float(np.max(e)))


def test_glcm_features_checks_roi_table(env, workloads):
    # the ROI table passed with a COO list must describe as many ROIs
    nyx, ctx, dev = env
    w = workloads("c2_small")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    rois, _ = nyx.nyx_bin_rois(ctx, imgs, w.n_bins)
    g = nyx.nyx_glcm_accumulate(ctx, imgs, rois, w.n_bins, offs)
    t = nyx.nyx_glcm_features(ctx, g, nyx.NYX_FP32, rois=rois)
    assert t.shape[0] == rois.n_rois
    other = nyx.RoiTable(rois.n_rois + 1, dev)
    other.n.value = rois.n_rois + 1
    with pytest.raises(nyx.NyxError) as e:
        nyx.nyx_glcm_features(ctx, g, nyx.NYX_FP32, rois=other)
    assert e.value.status == nyx.NYX_ERR_INVALID


def test_plan_profile_phases(env, workloads):
    """nyx_plan_profile times every phase of one eager step and leaves the same
    table as a graph replay (scan mode: bit-identical)."""
    import torch
    nyx, ctx, dev = env
    w = workloads("c3_small")
    imgs = device_images(w, dev)
    offs = _offsets(nyx, w)
    plan = nyx.nyx_plan_create(ctx, imgs, w.n_bins, offs, nyx.NYX_FP32, mode="dense16-scan")
    t1 = nyx.new_table(plan, len(offs))
    t2 = torch.full_like(t1, float("nan"))
    nyx.nyx_plan_execute(plan, t1)
    say("profile: c3_small, 16-bit scan mode")
    ms = nyx.nyx_plan_profile(plan, t2)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    assert tuple(ms) == nyx.PHASES
    assert all(v >= 0.0 for v in ms.values()), ms
    assert ms["batch"] > 0.0 and ms["scan"] > 0.0, ms
    a, b = t1.cpu().numpy(), t2.cpu().numpy()
    assert ((a == b) | (np.isnan(a) & np.isnan(b))).all()



# ------------------------------------------------------------------ banded accumulation
# flipped in-plane offsets (the same unordered pairs as the default four,
# pointing the other way) and an in-plane offset at distance 2 (gathered)
_FLIPPED_2D = [(0, 0, -1), (0, 1, 1), (0, 1, 0), (0, 1, -1), (0, -2, 2)]


@pytest.mark.parametrize("shape,ng,smooth,offs", [((28, 44, 44), 512, False, None), ((1, 300, 320), 2048, True, None),
                                                  ((1, 300, 320), 2048, True, _FLIPPED_2D)])
def test_banded_counts_exact(env, oracle_mod, shape, ng, smooth, offs):
    """ROIs above the banded kernel's size threshold at bin counts whose
    triangle exceeds LDS: exact counts through nyx_glcm_accumulate and the
    batched features, with pairs inside the LDS band and (uniform noise) far
    outside it; in 2D the in-plane distance-1 offsets go through the row
    sweep whichever way they point, others through the gather."""
    import torch
    from types import SimpleNamespace
    nyx, ctx, dev = env
    rng = np.random.default_rng(ng)
    if smooth:
        y, x = np.mgrid[0:shape[1], 0:shape[2]]
        I = (20000 + 15000 * np.sin(x / 37.0) * np.cos(y / 23.0) + rng.integers(0, 400, shape[1:]))[None]
    else:
        I = rng.integers(0, 60000, shape)
    I = np.ascontiguousarray(I, np.uint16)
    L = np.ones(shape, np.uint32)
    L[:, :5, :] = 2                                   # a second, smaller ROI
    L[0, 0, 0] = 0
    if offs is None:
        offs = nyx.nyx_offsets_default(3 if shape[0] > 1 else 2, 1)
    say(f"case banded counts {shape} ng={ng} smooth={smooth} offsets={offs}")
    w = SimpleNamespace(intensity=I[None], labels=L[None], n_images=1)
    imgs = device_images(w, dev)
    plan = nyx.nyx_plan_create(ctx, imgs, ng, offs, nyx.NYX_FP64)
    desc = nyx.nyx_plan_describe(plan)
    say("  plan:", desc)
    assert "mode=hash" in desc and "band_vox=0 " not in desc
    rois, _ = nyx.nyx_bin_rois(ctx, imgs, ng)
    g = nyx.nyx_glcm_accumulate(ctx, imgs, rois, ng, offs)
    keys = g.keys.cpu().numpy().view(np.uint64)
    cnt = g.counts.cpu().numpy().view(np.uint64)
    st = oracle_mod.roi_stats(I, L)
    roi = (keys >> np.uint64(38)).astype(np.int64)
    for r in range(st["label"].size):
        P = oracle_mod.glcm_roi(I, L, st["label"][r], st["vmin"][r], st["vmax"][r], st["bbox"][r], ng,
                                np.array(offs, np.int32))
        U = _triangle(P)
        kk, cc = keys[roi == r], cnt[roi == r]
        d = ((kk >> np.uint64(32)) & np.uint64(63)).astype(np.int64)
        i = ((kk >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
        j = (kk & np.uint64(0xFFFF)).astype(np.int64)
        assert len(kk) == np.count_nonzero(U), r
        assert np.array_equal(U[d, i, j], cc), r
    t = nyx.new_table(plan, len(offs), nyx.NYX_FP64)
    nyx.nyx_plan_execute(plan, t)
    torch.cuda.synchronize()
    nyx.nyx_plan_check(plan)
    want, Ps = _oracle_direct(oracle_mod, I, L, ng, offs)
    _check_features(t.cpu().numpy()[:plan.n_rois], want, Ps, TOL_FP64, "banded")
