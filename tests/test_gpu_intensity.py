"""GPU parity of the first-order intensity features (nyx_intensity_features)
against the FP64 oracle (oracle/first_order.py), through the C ABI.

Error of a value: |gpu - oracle| / max(|oracle|, M) with M the magnitude the
odd standardised moments sum from (first_order.magnitude) and 0 elsewhere
(plain relative error); NaN must match NaN.  Bars: 1e-12 for the FP64
table, 1e-5 for the FP32 table.  Order statistics, counts, extremes and the
mode are exact integers (or interpolations of them) and must match exactly
in FP64.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from gpu_util import device_images

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-12}
EXACT = ("MIN", "MAX", "RANGE", "INTEGRATED_INTENSITY", "ENERGY", "MEDIAN", "P01", "P10", "P25", "P75", "P90",
         "P99", "INTERQUARTILE_RANGE", "MODE", "EDGE_INTEGRATED_INTENSITY", "EDGE_MIN", "EDGE_MAX")


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


def _roi_oracle(fo, I, L, lab, bbox, n_bins):
    """Oracle features of one ROI computed on its bounding box (plus a
    one-voxel margin, so edge voxels see their true neighbours), with the
    weighted centroid moved back to image coordinates."""
    x0, y0, z0, x1, y1, z1 = (int(v) for v in bbox)
    nz, ny, nx = I.shape
    a = (max(z0 - 1, 0), max(y0 - 1, 0), max(x0 - 1, 0))
    b = (min(z1 + 2, nz), min(y1 + 2, ny), min(x1 + 2, nx))
    Ib = I[a[0]:b[0], a[1]:b[1], a[2]:b[2]]
    Mb = L[a[0]:b[0], a[1]:b[1], a[2]:b[2]] == lab
    f = fo.features(Ib, Mb, n_bins)
    M = fo.magnitude(Ib, Mb)
    for name, off in (("WEIGHTED_CENTROID_X", a[2]), ("WEIGHTED_CENTROID_Y", a[1]), ("WEIGHTED_CENTROID_Z", a[0])):
        f[fo.NAMES.index(name)] += off
    return f, M


def _rois_of(I, L):
    labs = np.unique(L[L != 0])
    out = []
    for lab in labs:
        zz, yy, xx = np.nonzero(L == lab)
        out.append((int(lab), (xx.min(), yy.min(), zz.min(), xx.max(), yy.max(), zz.max())))
    return out


def _check(fo, got, want, M, prec, tag):
    got = np.asarray(got, np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    assert np.array_equal(nan_g, nan_w), (tag, np.argwhere(nan_g != nan_w)[:5])
    with np.errstate(divide="ignore", invalid="ignore"):
        err = np.abs(got - want) / np.maximum(np.abs(want), M)
    err = np.where(nan_g | (got == want), 0.0, err)
    i = np.unravel_index(np.argmax(err), err.shape)
    say(f"  {tag}: {len(want)} ROIs, max error {err[i]:.3e} ({fo.NAMES[i[1]]} of row {i[0]})")
    assert err[i] <= TOL[prec], (tag, fo.NAMES[i[1]], i, got[i], want[i])
    if prec == 1:
        for name in EXACT:
            q = fo.NAMES.index(name)
            assert np.array_equal(got[:, q], want[:, q]), (tag, name)


def _run(nyx, ctx, dev, images, n_bins, prec):
    import torch
    rois, table = nyx.nyx_intensity_features(ctx, images, n_bins, prec)
    torch.cuda.synchronize()
    return rois, table.cpu().numpy()


@pytest.mark.parametrize("name", ["c1_tiny", "c2_small", "c3_small", "c4_small", "c5_small"])
@pytest.mark.parametrize("prec", [1, 0])
def test_workload_shapes(env, workloads, name, prec):
    from oracle import first_order as fo
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} intensity features prec={prec}")
    rois, got = _run(nyx, ctx, dev, device_images(w, dev), w.n_bins, prec)
    wants, Ms = [], []
    for k in range(w.n_images):
        I, L = w.intensity[k], w.labels[k]
        for lab, bb in _rois_of(I, L):
            f, M = _roi_oracle(fo, I, L, lab, bb, w.n_bins)
            wants.append(f)
            Ms.append(M)
    assert rois.n_rois == len(wants)
    _check(fo, got, np.array(wants), np.array(Ms), prec, f"{name} prec={prec}")


def _edge_images():
    """Small images holding the degenerate cases: one voxel, two voxels of
    different values (no value within [P10, P90]), a constant block, a thin
    line, ROIs on every border, all-zero intensities (no weighted centroid),
    the full 16-bit range, a disconnected label, ties of the mode."""
    rng = np.random.default_rng(5)
    L = np.zeros((1, 24, 40), np.uint32)
    I = rng.integers(0, 4000, L.shape).astype(np.uint16)
    L[0, 2, 2] = 1                                   # one voxel
    L[0, 5, 5:7] = 2; I[0, 5, 5] = 10; I[0, 5, 6] = 20   # two voxels
    L[0, 8:12, 2:6] = 3; I[0, 8:12, 2:6] = 777       # constant block
    L[0, 14, 1:30] = 4                               # thin line
    L[0, 0, :] = 5; L[0, :, 39] = 5                  # on two borders
    L[0, 18:22, 8:12] = 6; I[0, 18:22, 8:12] = 0     # all-zero intensities
    L[0, 16:24, 20:30] = 7
    I[0, 16:24, 20:30] = rng.choice(np.array([0, 65535, 1, 65534, 32768], np.uint16), (8, 10))
    L[0, 3:5, 30:33] = 8; L[0, 9:11, 30:33] = 8      # disconnected
    L[0, 2:4, 10:14] = 9; I[0, 2:4, 10:14] = np.array([[1, 1, 5, 5], [9, 9, 3, 3]], np.uint16)  # mode ties
    V = np.zeros((6, 7, 8), np.uint32)
    IV = rng.integers(0, 60000, V.shape).astype(np.uint16)
    V[1:5, 1:6, 1:7] = 1                             # interior and surface voxels
    V[0, 0, 0] = 2
    V[:, 3, 7] = 3                                   # a column through every plane, on the border
    return [(I, L), (IV, V)]


@pytest.mark.parametrize("n_bins", [2, 8, 100])
@pytest.mark.parametrize("prec", [1, 0])
def test_edge_cases(env, n_bins, prec):
    import torch
    from oracle import first_order as fo
    nyx, ctx, dev = env
    say(f"case intensity edge images n_bins={n_bins} prec={prec}")
    for I, L in _edge_images():
        imgs = [(torch.from_numpy(I.view(np.int16)).to(dev), torch.from_numpy(L.view(np.int32)).to(dev))]
        rois, got = _run(nyx, ctx, dev, imgs, n_bins, prec)
        wants, Ms = [], []
        for lab, bb in _rois_of(I, L):
            f, M = _roi_oracle(fo, I, L, lab, bb, n_bins)
            wants.append(f)
            Ms.append(M)
        assert rois.n_rois == len(wants)
        assert np.array_equal(rois.label.cpu().numpy()[:len(wants)], [lab for lab, _ in _rois_of(I, L)])
        _check(fo, got, np.array(wants), np.array(Ms), prec, f"edge {I.shape} n_bins={n_bins}")


def test_whole_image_oracle_route(env, workloads):
    """The c1 field of view through the oracle's own whole-image table (no
    bounding-box cropping in the reference)."""
    from oracle import first_order as fo
    nyx, ctx, dev = env
    w = workloads("c1_tiny")
    rois, got = _run(nyx, ctx, dev, device_images(w, dev), w.n_bins, 1)
    labels, want = fo.table(w.intensity[0], w.labels[0], w.n_bins)
    M = np.stack([fo.magnitude(w.intensity[0], w.labels[0] == lab) for lab in labels])
    _check(fo, got, want, M, 1, "c1 whole image")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,n_sample", [("c3_batch", 400), ("c4_3d", 60), ("c5_stress", 60)])
def test_full_size_sampled(env, workloads, name, n_sample):
    from oracle import first_order as fo
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} full size intensity features, sampled ROIs")
    rois, got = _run(nyx, ctx, dev, device_images(w, dev), w.n_bins, 0)
    n = rois.n_rois
    lab = rois.label.cpu().numpy()[:n].astype(np.int64) & 0xFFFFFFFF
    img = rois.image.cpu().numpy()[:n]
    bbox = rois.bbox.cpu().numpy()[:n]
    nvox = rois.n_vox.cpu().numpy()[:n]
    rng = np.random.default_rng(3)
    order = np.argsort(nvox)
    sample = set(rng.choice(n, size=min(n_sample, n), replace=False).tolist())
    sample |= {int(order[0]), int(order[len(order) // 2])}
    if name != "c5_stress":
        sample.add(int(order[-1]))          # the 90 % ROI of the stress tile is checked on its own below
    sample = sorted(sample)
    wants, Ms = [], []
    for r in sample:
        f, M = _roi_oracle(fo, w.intensity[img[r]], w.labels[img[r]], int(lab[r]), bbox[r], w.n_bins)
        wants.append(f)
        Ms.append(M)
    _check(fo, got[sample], np.array(wants), np.array(Ms), 0, f"{name} sampled")


@pytest.mark.timeout(600)
def test_c5_giant_roi_exact_statistics(env, workloads):
    """The 90 % ROI of the stress tile (about 60 M voxels, one work-group):
    the statistics that integer arithmetic fixes exactly -- count-based
    sums, extremes, every percentile (from a full sort), the level-histogram
    mode -- against numpy on the same voxels, at the FP32 output's rounding."""
    from oracle import first_order as fo
    nyx, ctx, dev = env
    w = workloads("c5_stress")
    say("case c5_stress giant ROI: exact statistics")
    rois, got = _run(nyx, ctx, dev, device_images(w, dev), w.n_bins, 0)
    nvox = rois.n_vox.cpu().numpy()[:rois.n_rois]
    g = int(np.argmax(nvox))
    lab = int(rois.label.cpu().numpy()[g]) & 0xFFFFFFFF
    I, L = w.intensity[0], w.labels[0]
    x = I[L == lab].astype(np.int64)
    n = x.size
    assert n == nvox[g]
    xs = np.sort(x)
    want = {"MIN": xs[0], "MAX": xs[-1], "RANGE": xs[-1] - xs[0], "INTEGRATED_INTENSITY": int(x.sum()),
            "ENERGY": int((x * x).sum()), "MEAN": int(x.sum()) / n}
    for p in (1, 10, 25, 50, 75, 90, 99):
        want["MEDIAN" if p == 50 else f"P{p:02d}"] = fo.percentile_sorted(xs, p)
    lv = fo.fbn_levels(x, int(xs[0]), int(xs[-1]), w.n_bins)
    want["MODE"] = 1 + int(np.argmax(np.bincount(lv, minlength=w.n_bins + 1)[1:]))
    row = dict(zip(fo.NAMES, got[g].astype(np.float64)))
    for k, v in want.items():
        assert row[k] == pytest.approx(float(v), rel=1e-7, abs=0), (k, row[k], v)
    say(f"  giant ROI {g}: {n} voxels, median {want['MEDIAN']}, mode level {want['MODE']}")
