"""Pins of the first-order intensity oracle (oracle/first_order.py) against
what the definitions and independent routines fix: a hand-derived golden,
a constant ROI, numpy / scipy / statistics implementations of the same
statistics, a brute-force edge-voxel count, and exact invariances."""
from __future__ import annotations

import math
import os
import statistics

import numpy as np
import pytest
import scipy.ndimage
import scipy.stats

from oracle import first_order as fo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "first_order_1234.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, expr = line.split()
        out[name] = float(eval(expr, {"__builtins__": {}, "sqrt": math.sqrt}))  # literal fractions
    return out


def test_golden_1234():
    I = np.array([[[1, 2], [3, 4]]], np.uint16)
    got = fo.features(I, np.ones_like(I, bool), 4)
    want = _golden()
    assert set(want) == set(fo.NAMES)
    for k, name in enumerate(fo.NAMES):
        assert got[k] == pytest.approx(want[name], rel=1e-13, abs=1e-13), name


def test_constant_roi():
    I = np.full((1, 3, 3), 7, np.uint16)
    f = dict(zip(fo.NAMES, fo.features(I, np.ones_like(I, bool), 8)))
    for k in ("MEAN", "MIN", "MAX", "MEDIAN", "P01", "P99", "EDGE_MEAN", "EDGE_MIN", "EDGE_MAX"):
        assert f[k] == 7.0, k
    for k in ("RANGE", "VARIANCE", "STDDEV", "SKEWNESS", "KURTOSIS", "HYPERSKEWNESS", "HYPERFLATNESS",
              "MEAN_ABSOLUTE_DEVIATION", "MEDIAN_ABSOLUTE_DEVIATION", "INTERQUARTILE_RANGE",
              "ROBUST_MEAN_ABSOLUTE_DEVIATION", "ENTROPY", "EDGE_STDDEV"):
        assert f[k] == 0.0, k
    assert f["UNIFORMITY"] == 1.0 and f["MODE"] == 1.0 and f["UNIFORMITY_PIU"] == 100.0
    assert f["EDGE_INTEGRATED_INTENSITY"] == 8 * 7.0   # the 8 border voxels of a 3x3 block
    assert (f["WEIGHTED_CENTROID_X"], f["WEIGHTED_CENTROID_Y"]) == (1.0, 1.0)


def test_robust_deviation_hand_cases():
    # three values 10, 15, 20: P10 = 10 + 0.2 * 5 = 11, P90 = 15 + 0.8 * 5 = 19,
    # so only 15 lies within [P10, P90] and its distance to its own mean is 0
    I = np.array([[[10, 15, 20]]], np.uint16)
    f = dict(zip(fo.NAMES, fo.features(I, np.ones_like(I, bool), 8)))
    assert (f["P10"], f["P90"]) == (11.0, 19.0)
    assert f["ROBUST_MEAN_ABSOLUTE_DEVIATION"] == 0.0
    # two values 10, 20: P10 = 11, P90 = 19 and no value lies within
    I = np.array([[[10, 20]]], np.uint16)
    f = dict(zip(fo.NAMES, fo.features(I, np.ones_like(I, bool), 8)))
    assert (f["P10"], f["P90"]) == (11.0, 19.0)
    assert math.isnan(f["ROBUST_MEAN_ABSOLUTE_DEVIATION"])
    # 10, 20, 30, 40: P10 = 13, P90 = 37, values 20 and 30, mean 25, distance 5
    I = np.array([[[10, 20, 30, 40]]], np.uint16)
    f = dict(zip(fo.NAMES, fo.features(I, np.ones_like(I, bool), 8)))
    assert (f["P10"], f["P90"], f["ROBUST_MEAN_ABSOLUTE_DEVIATION"]) == (13.0, 37.0, 5.0)


def _random_roi(seed, shape=(1, 23, 31), vmax=4000):
    rng = np.random.default_rng(seed)
    I = rng.integers(0, vmax, shape).astype(np.uint16)
    mask = rng.random(shape) < 0.6
    return I, mask


@pytest.mark.parametrize("seed,shape", [(1, (1, 23, 31)), (2, (5, 9, 11)), (3, (1, 1, 40))])
def test_against_independent_routines(seed, shape):
    I, mask = _random_roi(seed, shape)
    x = I[mask].astype(np.float64)
    f = dict(zip(fo.NAMES, fo.features(I, mask, 16)))
    assert f["MEAN"] == pytest.approx(np.mean(x), rel=1e-14)
    assert f["VARIANCE"] == pytest.approx(np.var(x, ddof=1), rel=1e-12)
    assert f["STANDARD_ERROR"] == pytest.approx(scipy.stats.sem(x), rel=1e-12)
    assert f["SKEWNESS"] == pytest.approx(scipy.stats.skew(x), rel=1e-10, abs=1e-12)
    assert f["KURTOSIS"] == pytest.approx(scipy.stats.kurtosis(x, fisher=False), rel=1e-12)
    m2 = scipy.stats.moment(x, 2)
    assert f["HYPERSKEWNESS"] == pytest.approx(scipy.stats.moment(x, 5) / m2 ** 2.5, rel=1e-9, abs=1e-12)
    assert f["HYPERFLATNESS"] == pytest.approx(scipy.stats.moment(x, 6) / m2 ** 3, rel=1e-12)
    assert f["MEDIAN"] == pytest.approx(statistics.median(x.tolist()), rel=1e-15)
    for p in (1, 10, 25, 75, 90, 99):
        assert f[f"P{p:02d}"] == pytest.approx(np.percentile(x, p, method="linear"), rel=1e-14), p
    assert f["INTERQUARTILE_RANGE"] == pytest.approx(scipy.stats.iqr(x), rel=1e-13)
    assert f["MEAN_ABSOLUTE_DEVIATION"] == pytest.approx(np.mean(np.abs(x - x.mean())), rel=1e-13)
    assert f["MEDIAN_ABSOLUTE_DEVIATION"] == pytest.approx(np.mean(np.abs(x - np.median(x))), rel=1e-13)
    lo, hi = np.percentile(x, [10, 90])
    sub = x[(x >= lo) & (x <= hi)]
    assert f["ROBUST_MEAN_ABSOLUTE_DEVIATION"] == pytest.approx(np.mean(np.abs(sub - sub.mean())), rel=1e-13)
    assert f["RMS"] == pytest.approx(math.sqrt(np.mean(x * x)), rel=1e-14)
    # histogram features from an independently binned histogram
    lv = np.floor(16 * (x - x.min()) / (x.max() - x.min())).astype(int) + 1
    lv = np.minimum(lv, 16)
    cnt = np.bincount(lv, minlength=17)[1:]
    assert f["ENTROPY"] == pytest.approx(scipy.stats.entropy(cnt, base=2), rel=1e-13)
    assert f["UNIFORMITY"] == pytest.approx(float(np.sum((cnt / x.size) ** 2)), rel=1e-13)
    assert f["MODE"] == 1 + int(np.flatnonzero(cnt == cnt.max())[0])
    # intensity-weighted centre of mass (z, y, x)
    cz, cy, cx = scipy.ndimage.center_of_mass(np.where(mask, I.astype(np.float64), 0.0))
    assert (f["WEIGHTED_CENTROID_Z"], f["WEIGHTED_CENTROID_Y"], f["WEIGHTED_CENTROID_X"]) == pytest.approx(
        (cz, cy, cx), rel=1e-12, abs=1e-12)


def test_edge_voxels_brute_force():
    for seed, shape in ((4, (1, 13, 17)), (5, (4, 6, 7))):
        I, mask = _random_roi(seed, shape)
        nz, ny, nx = shape
        nb = [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0)] + ([(1, 0, 0), (-1, 0, 0)] if nz > 1 else [])
        edge = []
        for z, y, x in zip(*np.nonzero(mask)):
            for dz, dy, dx in nb:
                w = (z + dz, y + dy, x + dx)
                if not (0 <= w[0] < nz and 0 <= w[1] < ny and 0 <= w[2] < nx) or not mask[w]:
                    edge.append(int(I[z, y, x]))
                    break
        f = dict(zip(fo.NAMES, fo.features(I, mask, 8)))
        assert f["EDGE_INTEGRATED_INTENSITY"] == sum(edge)
        assert f["EDGE_MIN"] == min(edge) and f["EDGE_MAX"] == max(edge)
        assert f["EDGE_STDDEV"] == pytest.approx(statistics.stdev(edge), rel=1e-12)


def test_shift_and_permutation_invariance():
    I, mask = _random_roi(6)
    base = dict(zip(fo.NAMES, fo.features(I, mask, 16)))
    c = 1234
    shifted = dict(zip(fo.NAMES, fo.features((I.astype(np.int64) + c).astype(np.uint16), mask, 16)))
    n = int(mask.sum())
    for k in ("MEAN", "MIN", "MAX", "MEDIAN", "P01", "P10", "P25", "P75", "P90", "P99", "EDGE_MEAN",
              "EDGE_MIN", "EDGE_MAX"):
        assert shifted[k] == pytest.approx(base[k] + c, rel=1e-13), k
    for k in ("RANGE", "VARIANCE", "STDDEV", "SKEWNESS", "KURTOSIS", "HYPERSKEWNESS", "HYPERFLATNESS",
              "MEAN_ABSOLUTE_DEVIATION", "MEDIAN_ABSOLUTE_DEVIATION", "INTERQUARTILE_RANGE",
              "ROBUST_MEAN_ABSOLUTE_DEVIATION", "EDGE_STDDEV"):
        assert shifted[k] == pytest.approx(base[k], rel=1e-9, abs=1e-9), k
    for k in ("MODE", "ENTROPY", "UNIFORMITY"):           # the levels do not move
        assert shifted[k] == base[k], k
    assert shifted["INTEGRATED_INTENSITY"] == base["INTEGRATED_INTENSITY"] + c * n
    # values permuted among the ROI's voxels: every statistic of the multiset stays
    rng = np.random.default_rng(7)
    J = I.copy()
    J[mask] = rng.permutation(I[mask])
    perm = dict(zip(fo.NAMES, fo.features(J, mask, 16)))
    for k in fo.NAMES:
        if k.startswith(("WEIGHTED_CENTROID", "EDGE_")):
            continue
        assert perm[k] == pytest.approx(base[k], rel=1e-12, abs=1e-12), k


def test_mode_ties_take_the_lowest_level():
    I = np.array([[[10, 10, 20, 20, 30]]], np.uint16)
    f = dict(zip(fo.NAMES, fo.features(I, np.ones_like(I, bool), 3)))
    # levels 1 + floor(3 (x - 10) / 20): 1, 1, 2, 2, 4 -> 3: counts 2, 2, 1
    assert f["MODE"] == 1.0


def test_table_rows_in_label_order():
    I, _ = _random_roi(8, (1, 12, 12))
    L = np.zeros(I.shape, np.uint32)
    L[0, :6, :] = 9
    L[0, 6:, :6] = 3
    L[0, 6:, 6:] = 4_000_000_000
    labels, t = fo.table(I, L, 8)
    assert labels.tolist() == [3, 9, 4_000_000_000]
    assert t[1] == pytest.approx(fo.features(I, L == 9, 8), nan_ok=True)
