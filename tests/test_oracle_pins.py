"""Pins of the FP64 oracle against things other than itself.

Each group targets one part of the path:
  binning      exact-rational bin edges via bisect; extremes; affine invariance
  counts       brute-force pair enumeration; box-total closed form (golden);
               popcount totals for arbitrary masks; symmetry; transposes,
               flips, 3D axis permutations, translation, label permutation
  features     hand-derived checkerboard and constant-ROI values (golden);
               the pair-list route through numpy/scipy/sklearn statistics;
               algebraic identities; empty directions; iid statistics
"""
from __future__ import annotations

import bisect
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from pairlist import count_matrix, features_from_pairs, ordered_pairs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAMES = ["ASM", "ACOR", "CLUPROM", "CLUSHADE", "CLUTEND", "CONTRAST", "CORR", "DIFAVE",
         "DIFENTRO", "DIFVAR", "DIS", "ENERGY", "ENTROPY", "HOM1", "HOM2", "IDM", "INFOMEAS1",
         "INFOMEAS2", "IDMN", "ID", "IDN", "IV", "JAVE", "JE", "JMAX", "SUMAVE", "SUMENT",
         "JVAR", "SUMVAR", "VARIANCE"]


def _rand_scene(rng, shape, n_labels, fill=0.7, lo=0, hi=4095):
    I = rng.integers(lo, hi + 1, shape).astype(np.uint16)
    L = rng.integers(1, n_labels + 1, shape).astype(np.uint32)
    L[rng.random(shape) > fill] = 0
    return I, L


def test_feature_names(oracle_mod):
    assert oracle_mod.feature_names() == NAMES


# ------------------------------------------------------------------ binning
def _bin_by_edges(I, lo, hi, ng):
    """Level = 1 + number of bin edges lo + k (hi - lo) / ng (k = 1..ng-1) at or
    below I, with exact rational edges located by bisect."""
    if hi == lo:
        return 1
    edge = lambda k: Fraction(lo) + Fraction(k * (hi - lo), ng)
    return 1 + bisect.bisect_right(range(1, ng), Fraction(I), key=edge)


@pytest.mark.parametrize("ng", [2, 3, 8, 10, 30, 64, 100, 256, 1024, 65535])
def test_binning_matches_rational_edges(oracle_mod, ng):
    rng = np.random.default_rng(ng)
    for _ in range(60):
        lo = int(rng.integers(0, 65535))
        hi = int(rng.integers(lo, 65536))
        for I in {lo, hi, (lo + hi) // 2, int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))}:
            assert oracle_mod.bin_value(I, lo, hi, ng) == _bin_by_edges(I, lo, hi, ng)


def test_binning_extremes_and_constant(oracle_mod):
    for ng in (2, 8, 64, 1024, 65535):
        assert oracle_mod.bin_value(0, 0, 65535, ng) == 1
        assert oracle_mod.bin_value(65535, 0, 65535, ng) == ng
        assert oracle_mod.bin_value(777, 777, 777, ng) == 1


def test_binning_equal_width_histogram(oracle_mod):
    # range split into ng equal integer-width bins: each bin holds m values,
    # the last one also holds the maximum.
    ng, m = 16, 37
    h = np.zeros(ng + 1, int)
    for I in range(0, ng * m + 1):
        h[oracle_mod.bin_value(I, 0, ng * m, ng)] += 1
    assert h[0] == 0 and all(h[1:ng] == m) and h[ng] == m + 1


def test_bin_image_histogram_totals(oracle_mod):
    rng = np.random.default_rng(5)
    I, L = _rand_scene(rng, (1, 23, 31), 5)
    st = oracle_mod.roi_stats(I, L)
    B = oracle_mod.bin_image(I, L, 7, st)
    assert np.all((B == 0) == (L == 0))
    for r, lab in enumerate(st["label"]):
        sel = B[L == lab]
        assert sel.size == st["count"][r]
        assert sel.min() >= 1 and sel.max() <= 7


def test_affine_intensity_invariance(oracle_mod):
    rng = np.random.default_rng(11)
    I, L = _rand_scene(rng, (1, 19, 21), 4, hi=2000)
    off = oracle_mod.default_offsets(2)
    _, t1 = oracle_mod.extract(I, L, 9, off)
    _, t2 = oracle_mod.extract((3 * I.astype(np.int64) + 1234).astype(np.uint16), L, 9, off)
    assert np.array_equal(np.nan_to_num(t1, nan=-7), np.nan_to_num(t2, nan=-7))


# -------------------------------------------------------------- ROI table
def test_roi_stats_brute_force(oracle_mod):
    rng = np.random.default_rng(3)
    I, L = _rand_scene(rng, (3, 9, 11), 6)
    L[L == 4] = 4000000000  # arbitrary u32 label values
    st = oracle_mod.roi_stats(I, L)
    labs = sorted(set(L.ravel().tolist()) - {0})
    assert st["label"].tolist() == labs
    for r, lab in enumerate(labs):
        zz, yy, xx = np.nonzero(L == lab)
        assert st["count"][r] == zz.size
        assert st["vmin"][r] == I[L == lab].min() and st["vmax"][r] == I[L == lab].max()
        assert st["bbox"][r].tolist() == [xx.min(), yy.min(), zz.min(), xx.max(), yy.max(), zz.max()]
    assert st["count"].sum() == np.count_nonzero(L)


# ------------------------------------------------------------------ counts
@pytest.mark.parametrize("dims,distance,seed", [(2, 1, 1), (2, 2, 2), (3, 1, 3), (3, 2, 4)])
def test_counts_brute_force(oracle_mod, dims, distance, seed):
    rng = np.random.default_rng(seed)
    shape = (1, 8, 9) if dims == 2 else (4, 5, 6)
    I, L = _rand_scene(rng, shape, 3, fill=0.8)
    ng = 6
    st = oracle_mod.roi_stats(I, L)
    B = oracle_mod.bin_image(I, L, ng, st)
    off = oracle_mod.default_offsets(dims, distance)
    for r, lab in enumerate(st["label"]):
        P = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], ng, off)
        for k, d in enumerate(off):
            Pb = count_matrix(ordered_pairs(B, L, lab, d), ng)
            assert np.array_equal(P[k], Pb), (lab, d)


def test_counts_random_offsets_brute_force(oracle_mod):
    rng = np.random.default_rng(21)
    I, L = _rand_scene(rng, (3, 6, 7), 2, fill=0.9)
    st = oracle_mod.roi_stats(I, L)
    B = oracle_mod.bin_image(I, L, 5, st)
    off = np.array([[0, 0, 3], [1, -2, 1], [2, 1, -3], [0, 3, 0]], np.int32)
    for r, lab in enumerate(st["label"]):
        P = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], 5, off)
        for k, d in enumerate(off):
            assert np.array_equal(P[k], count_matrix(ordered_pairs(B, L, lab, d), 5))


def _golden_box():
    rows = []
    for line in open(os.path.join(GOLDEN, "box_totals.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden_box())
def test_box_total_closed_form(oracle_mod, row):
    nz, ny, nx, dz, dy, dx, T = row
    # the box sits inside a larger canvas, next to another label
    I = np.random.default_rng(1).integers(0, 4096, (nz + 4, ny + 4, nx + 4)).astype(np.uint16)
    L = np.zeros(I.shape, np.uint32)
    L[2:2 + nz, 2:2 + ny, 2:2 + nx] = 5
    L[0, 0, :] = 9
    st = oracle_mod.roi_stats(I, L)
    r = int(np.nonzero(st["label"] == 5)[0][0])
    P = oracle_mod.glcm_roi(I, L, 5, st["vmin"][r], st["vmax"][r], st["bbox"][r], 8,
                            np.array([[dz, dy, dx]], np.int32))
    assert int(P.sum()) == T


def _shift_overlap(mask: np.ndarray, d) -> int:
    """#{v : mask[v] and mask[v + d]} via array slicing."""
    sl_a, sl_b = [], []
    for n, s in zip(mask.shape, d):
        if s >= 0:
            sl_a.append(slice(0, n - s)); sl_b.append(slice(s, n))
        else:
            sl_a.append(slice(-s, n)); sl_b.append(slice(0, n + s))
    return int(np.count_nonzero(mask[tuple(sl_a)] & mask[tuple(sl_b)]))


@pytest.mark.parametrize("dims", [2, 3])
def test_totals_popcount(oracle_mod, dims):
    rng = np.random.default_rng(40 + dims)
    shape = (1, 40, 37) if dims == 2 else (9, 11, 10)
    I, L = _rand_scene(rng, shape, 4, fill=0.85)
    st = oracle_mod.roi_stats(I, L)
    off = oracle_mod.default_offsets(dims, 1)
    for r, lab in enumerate(st["label"]):
        P = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], 13, off)
        for k, d in enumerate(off):
            assert int(P[k].sum()) == 2 * _shift_overlap(L == lab, d)
            assert np.array_equal(P[k], P[k].T)
            assert np.all(np.diag(P[k]) % 2 == 0)


def test_transpose_and_flip_swap_directions(oracle_mod):
    rng = np.random.default_rng(8)
    I, L = _rand_scene(rng, (1, 17, 17), 3)
    off = oracle_mod.default_offsets(2)  # 0, 45, 90, 135 degrees
    _, t = oracle_mod.extract(I, L, 11, off)
    _, tt = oracle_mod.extract(np.ascontiguousarray(I.transpose(0, 2, 1)),
                               np.ascontiguousarray(L.transpose(0, 2, 1)), 11, off)
    _, tf = oracle_mod.extract(np.ascontiguousarray(I[:, :, ::-1]),
                               np.ascontiguousarray(L[:, :, ::-1]), 11, off)
    eq = lambda a, b: np.allclose(a, b, rtol=1e-12, atol=1e-12, equal_nan=True)
    # transposing x <-> y swaps 0 and 90 degrees and keeps 45 and 135
    assert eq(t[:, 0], tt[:, 2]) and eq(t[:, 2], tt[:, 0])
    assert eq(t[:, 1], tt[:, 1]) and eq(t[:, 3], tt[:, 3])
    # flipping x swaps 45 and 135 degrees
    assert eq(t[:, 1], tf[:, 3]) and eq(t[:, 3], tf[:, 1])
    assert eq(t[:, 0], tf[:, 0]) and eq(t[:, 2], tf[:, 2])


def test_3d_axis_permutation_permutes_offsets(oracle_mod):
    rng = np.random.default_rng(9)
    I, L = _rand_scene(rng, (6, 7, 8), 2)
    off = oracle_mod.default_offsets(3)
    st = oracle_mod.roi_stats(I, L)
    perm = (2, 0, 1)  # new axis a is old axis perm[a]
    Ip = np.ascontiguousarray(I.transpose(perm))
    Lp = np.ascontiguousarray(L.transpose(perm))
    stp = oracle_mod.roi_stats(Ip, Lp)
    for r, lab in enumerate(st["label"]):
        P = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], 6, off)
        rp = int(np.nonzero(stp["label"] == lab)[0][0])
        moved = np.array([[d[perm[0]], d[perm[1]], d[perm[2]]] for d in off], np.int32)
        Pp = oracle_mod.glcm_roi(Ip, Lp, lab, stp["vmin"][rp], stp["vmax"][rp], stp["bbox"][rp], 6, moved)
        assert np.array_equal(P, Pp)


def test_translation_and_label_permutation(oracle_mod):
    rng = np.random.default_rng(12)
    I, L = _rand_scene(rng, (1, 15, 14), 4)
    off = oracle_mod.default_offsets(2)
    st, t = oracle_mod.extract(I, L, 10, off)
    I2 = np.zeros((1, 25, 30), np.uint16)
    L2 = np.zeros((1, 25, 30), np.uint32)
    I2[:, 7:22, 9:23] = I
    perm = {1: 40, 2: 7, 3: 900, 4: 3}
    L2[:, 7:22, 9:23] = np.vectorize(lambda v: perm.get(int(v), 0))(L)
    st2, t2 = oracle_mod.extract(I2, L2, 10, off)
    for r, lab in enumerate(st["label"]):
        r2 = int(np.nonzero(st2["label"] == perm[int(lab)])[0][0])
        assert np.array_equal(np.nan_to_num(t[r], nan=-1), np.nan_to_num(t2[r2], nan=-1))


# ---------------------------------------------------------------- features
def _golden_eval(expr: str) -> float:
    H = lambda a, b: -a * math.log2(a) - b * math.log2(b)
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt, "exp": math.exp, "H": H}))


def test_checkerboard_golden(oracle_mod):
    n = 8
    y, x = np.mgrid[0:n, 0:n]
    I = (((x + y) % 2) * 4095).astype(np.uint16)[None]
    L = np.ones((1, n, n), np.uint32)
    _, t = oracle_mod.extract(I, L, 8, oracle_mod.default_offsets(2))
    checked = 0
    for line in open(os.path.join(GOLDEN, "checkerboard_ng8_n8.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        blk, name, expr = line.split(None, 2)
        want = _golden_eval(expr)
        got = t[0, int(blk), NAMES.index(name)]
        assert got == pytest.approx(want, rel=1e-13, abs=1e-12), (blk, name)
        checked += 1
    assert checked == 128


@pytest.mark.parametrize("shape,ng", [((1, 5, 6), 8), ((1, 12, 3), 64), ((3, 4, 4), 1024)])
def test_constant_roi_golden(oracle_mod, shape, ng):
    I = np.full(shape, 1234, np.uint16)
    L = np.ones(shape, np.uint32)
    dims = 3 if shape[0] > 1 else 2
    off = oracle_mod.default_offsets(dims)
    _, t = oracle_mod.extract(I, L, ng, off)
    for line in open(os.path.join(GOLDEN, "constant_roi.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        name, expr = line.split(None, 1)
        want = _golden_eval(expr)
        for blk in range(len(off) + 1):
            assert t[0, blk, NAMES.index(name)] == pytest.approx(want, abs=1e-15), (blk, name)


def _pairlist_compare(oracle_mod, I, L, ng, off, rel=1e-11):
    st, t = oracle_mod.extract(I, L, ng, off)
    B = oracle_mod.bin_image(I, L, ng, st)
    n_checked = 0
    for r, lab in enumerate(st["label"]):
        for k, d in enumerate(off):
            f = features_from_pairs(ordered_pairs(B, L, lab, d), ng)
            if f is None:
                assert np.all(np.isnan(t[r, k]))
                continue
            for q, name in enumerate(NAMES):
                want = f[name]
                scale = max(abs(want), 1.0)
                assert abs(t[r, k, q] - want) <= rel * scale, (lab, tuple(d), name, t[r, k, q], want)
            n_checked += 1
    return n_checked


@pytest.mark.parametrize("ng,seed", [(8, 1), (10, 2), (30, 3), (100, 4), (5, 5)])
def test_features_pairlist_route_2d(oracle_mod, ng, seed):
    rng = np.random.default_rng(100 + seed)
    I, L = _rand_scene(rng, (1, 9, 10), 3, fill=0.9, hi=60)
    n = _pairlist_compare(oracle_mod, I, L, ng, oracle_mod.default_offsets(2))
    assert n >= 8


def test_features_pairlist_route_smooth_2d(oracle_mod):
    # correlated neighbours (a ramp plus small noise): large mutual information
    rng = np.random.default_rng(7)
    y, x = np.mgrid[0:10, 0:11]
    I = (40 * x + 25 * y + rng.integers(0, 30, (10, 11))).astype(np.uint16)[None]
    L = np.ones((1, 10, 11), np.uint32)
    L[0, :3, :4] = 2
    assert _pairlist_compare(oracle_mod, I, L, 16, oracle_mod.default_offsets(2)) == 8


def test_features_pairlist_route_3d(oracle_mod):
    rng = np.random.default_rng(33)
    I, L = _rand_scene(rng, (4, 4, 5), 2, fill=0.95, hi=40)
    assert _pairlist_compare(oracle_mod, I, L, 7, oracle_mod.default_offsets(3)) >= 20


def _random_sym(rng, ng, density=0.5, hi=50):
    C = rng.integers(0, hi, (ng, ng)) * (rng.random((ng, ng)) < density)
    return (C + C.T).astype(np.uint64)


@pytest.mark.parametrize("ng", [2, 7, 16, 64])
def test_feature_identities(oracle_mod, ng):
    rng = np.random.default_rng(ng)
    for _ in range(20):
        P = _random_sym(rng, ng)
        if P.sum() == 0:
            continue
        f = dict(zip(NAMES, oracle_mod.features(P)))
        tol = 1e-9
        assert f["CLUTEND"] == pytest.approx(f["SUMVAR"], rel=tol, abs=tol)
        assert f["CONTRAST"] == pytest.approx(2 * f["JVAR"] * (1 - f["CORR"]), rel=tol, abs=tol)
        assert f["DIFVAR"] == pytest.approx(f["CONTRAST"] - f["DIFAVE"] ** 2, rel=tol, abs=tol)
        assert f["SUMAVE"] == pytest.approx(2 * f["JAVE"], rel=tol)
        assert f["DIS"] == pytest.approx(f["DIFAVE"], rel=tol, abs=tol)
        for a, b in [("ASM", "ENERGY"), ("ENTROPY", "JE"), ("HOM1", "ID"), ("HOM2", "IDM"),
                     ("JVAR", "VARIANCE")]:
            assert f[a] == f[b]
        assert -1 - tol <= f["CORR"] <= 1 + tol
        assert 0 <= f["INFOMEAS2"] < 1
        assert 0 < f["ASM"] <= 1
        assert f["JMAX"] == pytest.approx(float(P.max()) / float(P.sum()), rel=1e-15)


def test_empty_direction_is_nan_and_skipped_in_mean(oracle_mod):
    # a one-pixel-wide vertical line has no horizontal or diagonal pairs
    I = np.arange(20, dtype=np.uint16).reshape(1, 20, 1) * 100
    I = np.concatenate([I, np.zeros_like(I)], axis=2)
    L = np.zeros_like(I, dtype=np.uint32)
    L[0, :, 0] = 1
    off = oracle_mod.default_offsets(2)
    _, t = oracle_mod.extract(I, L, 8, off)
    for k in (0, 1, 3):
        assert np.all(np.isnan(t[0, k]))
    assert not np.any(np.isnan(t[0, 2]))
    assert np.array_equal(t[0, 4], t[0, 2])
    # a single voxel has no pair at all: the mean is undefined as well
    L1 = np.zeros((1, 3, 3), np.uint32)
    L1[0, 1, 1] = 1
    _, t1 = oracle_mod.extract(np.ones((1, 3, 3), np.uint16), L1, 8, off)
    assert np.all(np.isnan(t1))


def test_iid_uniform_statistics(oracle_mod, synth_mod):
    # iid uniform levels on 8 bins: contrast ~ 2 Var(U{1..8}) = 10.5, corr ~ 0,
    # joint entropy ~ 6 bits (loose sanity check)
    w = synth_mod.make("c1_tiny")
    _, t = oracle_mod.extract(w.intensity[0], w.labels[0], 8, oracle_mod.default_offsets(2))
    m = dict(zip(NAMES, t[0, 4]))
    assert abs(m["CONTRAST"] - 10.5) < 0.5
    assert abs(m["CORR"]) < 0.05
    assert abs(m["JE"] - 6.0) < 0.05
    P = None
    st = oracle_mod.roi_stats(w.intensity[0], w.labels[0])
    P = oracle_mod.glcm_roi(w.intensity[0], w.labels[0], 1, st["vmin"][0], st["vmax"][0],
                            st["bbox"][0], 8, oracle_mod.default_offsets(2))
    assert P.sum(axis=(1, 2)).tolist() == [8064, 7938, 8064, 7938]


# ---------------------------------------------------------------- merged matrices
# Reading A15: the offsets' counts pooled into one symmetric matrix, then the
# 30 features of that matrix.
@pytest.mark.parametrize("dims,seed", [(2, 1), (2, 2), (3, 3)])
def test_merged_pairlist_route(oracle_mod, dims, seed):
    # independent route: the brute-force pair lists of all offsets pooled
    rng = np.random.default_rng(500 + seed)
    shape = (1, 9, 10) if dims == 2 else (4, 4, 5)
    I, L = _rand_scene(rng, shape, 3 if dims == 2 else 2, fill=0.9, hi=60 if dims == 2 else 40)
    ng = 9
    off = oracle_mod.default_offsets(dims)
    st = oracle_mod.roi_stats(I, L)
    B = oracle_mod.bin_image(I, L, ng, st)
    n = 0
    for r, lab in enumerate(st["label"]):
        P = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], ng, off)
        got = oracle_mod.features_roi_merged(P)
        assert got.shape == (1, 30)
        f = features_from_pairs(np.concatenate([ordered_pairs(B, L, lab, d) for d in off]), ng)
        if f is None:
            assert np.all(np.isnan(got))
            continue
        for q, name in enumerate(NAMES):
            want = f[name]
            assert abs(got[0, q] - want) <= 1e-11 * max(abs(want), 1.0), (lab, name, got[0, q], want)
        n += 1
    assert n >= 2


def test_merged_checkerboard_contrast(oracle_mod):
    # 8 x 8 two-level checkerboard at 8 levels (1 and 8): the 0 and 90 degree
    # offsets give 56 + 56 unordered pairs of levels (1, 8), the diagonals
    # 49 + 49 same-level pairs.  Pooled symmetric counts: T = 2 (112 + 98) =
    # 420, of which 224 at |i - j| = 7, so CONTRAST = 224 * 49 / 420 = 392/15
    # and DIS = 224 * 7 / 420 = 56/15.
    n = 8
    y, x = np.mgrid[0:n, 0:n]
    I = (((x + y) % 2) * 4095).astype(np.uint16)[None]
    L = np.ones((1, n, n), np.uint32)
    st = oracle_mod.roi_stats(I, L)
    P = oracle_mod.glcm_roi(I, L, 1, st["vmin"][0], st["vmax"][0], st["bbox"][0], 8, oracle_mod.default_offsets(2))
    f = oracle_mod.features_roi_merged(P)[0]
    assert f[NAMES.index("CONTRAST")] == pytest.approx(392 / 15, rel=1e-14)
    assert f[NAMES.index("DIS")] == pytest.approx(56 / 15, rel=1e-14)


def test_merged_scale_invariance(oracle_mod):
    # an offset listed twice doubles every count: the normalised matrix, and
    # so every feature, is that of the offset alone
    rng = np.random.default_rng(91)
    I, L = _rand_scene(rng, (1, 12, 11), 2, fill=0.9)
    st = oracle_mod.roi_stats(I, L)
    for r, lab in enumerate(st["label"]):
        one = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], 16,
                                  np.array([[0, 1, 1]], np.int32))
        two = oracle_mod.glcm_roi(I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], 16,
                                  np.array([[0, 1, 1], [0, -1, -1]], np.int32))
        assert np.array_equal(two.sum(axis=0), 2 * one[0])
        np.testing.assert_allclose(oracle_mod.features_roi_merged(two)[0], oracle_mod.features_roi(one)[0],
                                   rtol=1e-12, atol=1e-13)


# ------------------------------------------------------------------ sanitizers
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    """The oracle's C entry points on small seeded inputs, built with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code only)."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    exe = str(tmp_path / "oracle_sanitized")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=undefined", "-o", exe, os.path.join(here, "oracle_sanitize_main.c"),
                           os.path.join(root, "oracle", "oracle.c"), "-lm"])
    # the ASan runtime is linked into the driver; a library the environment
    # preloads ahead of it is accepted rather than refused
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "oracle sanitized run ok" in r.stdout


# ------------------------------------------------------------------ error-measure scale
def test_shade_magnitude_definition(oracle_mod):
    """sum |i + j - mux - muy|^3 p, the cluster-shade error scale, against an
    independent numpy evaluation on random (also non-symmetric) matrices, the
    checkerboard closed form, and the bound |CLUSHADE| <= magnitude."""
    rng = np.random.default_rng(17)
    for ng in (2, 5, 16):
        for sym in (True, False):
            P = rng.integers(0, 50, (ng, ng)).astype(np.uint64)
            if sym:
                P = P + P.T
            p = P.astype(np.float64) / P.sum()
            lv = np.arange(1, ng + 1)
            mux, muy = (p.sum(axis=1) * lv).sum(), (p.sum(axis=0) * lv).sum()
            want = (np.abs(lv[:, None] + lv[None, :] - mux - muy) ** 3 * p).sum()
            got = oracle_mod.shade_magnitude(P)
            assert got == pytest.approx(want, rel=1e-12)
            if sym:
                assert abs(oracle_mod.features(P)[3]) <= got * (1 + 1e-12)
    # checkerboard at 0 degrees: both cells sit on i + j = 1 + Ng = mux + muy
    P = np.zeros((8, 8), np.uint64)
    P[0, 7] = P[7, 0] = 56
    assert oracle_mod.shade_magnitude(P) == 0.0
    # two diagonal cells (1,1) weight q, (Ng,Ng) weight 1-q: mu = q + Ng (1 - q)
    P = np.zeros((8, 8), np.uint64)
    P[0, 0], P[7, 7] = 30, 10
    q, mu = 0.75, 0.75 + 8 * 0.25
    assert oracle_mod.shade_magnitude(P) == pytest.approx(q * abs(2 - 2 * mu) ** 3 + (1 - q) * abs(16 - 2 * mu) ** 3,
                                                          rel=1e-14)
    assert np.isnan(oracle_mod.shade_magnitude(np.zeros((4, 4), np.uint64)))


# ------------------------------------------------------------------ non-symmetric matrices [A16]
@pytest.mark.parametrize("dims,distance,seed", [(2, 1, 41), (2, 2, 42), (3, 1, 43)])
def test_ordered_counts_brute_force(oracle_mod, dims, distance, seed):
    """Ordered counts C against the brute-force pair list (each pair once, in
    its own order), their sum with the transpose against the symmetric
    matrix, and the reversed offset giving the transpose."""
    rng = np.random.default_rng(seed)
    shape = (1, 8, 9) if dims == 2 else (4, 5, 6)
    I, L = _rand_scene(rng, shape, 3, fill=0.8)
    ng = 6
    st = oracle_mod.roi_stats(I, L)
    B = oracle_mod.bin_image(I, L, ng, st)
    off = oracle_mod.default_offsets(dims, distance)
    for r, lab in enumerate(st["label"]):
        args = (I, L, lab, st["vmin"][r], st["vmax"][r], st["bbox"][r], ng)
        C = oracle_mod.glcm_roi(*args, off, symmetric=False)
        Cneg = oracle_mod.glcm_roi(*args, -off, symmetric=False)
        P = oracle_mod.glcm_roi(*args, off)
        for k, d in enumerate(off):
            assert np.array_equal(C[k], count_matrix(ordered_pairs(B, L, lab, d), ng, symmetric=False)), (lab, d)
            assert np.array_equal(C[k] + C[k].T, P[k])
            assert np.array_equal(Cneg[k], C[k].T)


def _pairlist_compare_ordered(oracle_mod, I, L, ng, off, rel=1e-11):
    st, t = oracle_mod.extract(I, L, ng, off, symmetric=False)
    B = oracle_mod.bin_image(I, L, ng, st)
    n_checked = 0
    for r, lab in enumerate(st["label"]):
        for k, d in enumerate(off):
            f = features_from_pairs(ordered_pairs(B, L, lab, d), ng, symmetric=False)
            if f is None:
                assert np.all(np.isnan(t[r, k]))
                continue
            for q, name in enumerate(NAMES):
                want = f[name]
                assert abs(t[r, k, q] - want) <= rel * max(abs(want), 1.0), (lab, tuple(d), name, t[r, k, q], want)
            n_checked += 1
    return n_checked


@pytest.mark.parametrize("ng,seed", [(8, 11), (10, 12), (30, 13), (5, 14)])
def test_ordered_features_pairlist_route_2d(oracle_mod, ng, seed):
    rng = np.random.default_rng(200 + seed)
    I, L = _rand_scene(rng, (1, 9, 10), 3, fill=0.9, hi=60)
    assert _pairlist_compare_ordered(oracle_mod, I, L, ng, oracle_mod.default_offsets(2)) >= 8


def test_ordered_features_pairlist_route_ramp_and_3d(oracle_mod):
    # a ramp: the level at v + d differs systematically from the level at v,
    # so the two marginals and means differ
    y, x = np.mgrid[0:10, 0:11]
    I = (40 * x + 25 * y).astype(np.uint16)[None]
    L = np.ones((1, 10, 11), np.uint32)
    assert _pairlist_compare_ordered(oracle_mod, I, L, 16, oracle_mod.default_offsets(2)) == 4
    rng = np.random.default_rng(34)
    I, L = _rand_scene(rng, (4, 4, 5), 2, fill=0.95, hi=40)
    assert _pairlist_compare_ordered(oracle_mod, I, L, 7, oracle_mod.default_offsets(3)) >= 20


def test_ordered_single_level_marginal(oracle_mod):
    """A matrix with one occupied row but several columns: the product of its
    marginals, so CORR = 1, INFOMEAS1 = INFOMEAS2 = 0 [A16], and the other
    features from the column marginal alone."""
    C = np.zeros((5, 5), np.uint64)
    C[2, [0, 1, 4]] = [1, 2, 3]   # level 3 at v; levels 1, 2, 5 at v + d with p = 1/6, 2/6, 3/6
    f = dict(zip(NAMES, oracle_mod.features(C)))
    assert (f["CORR"], f["INFOMEAS1"], f["INFOMEAS2"]) == (1.0, 0.0, 0.0)
    p = np.array([1, 2, 3]) / 6.0
    j = np.array([1, 2, 5])
    assert f["JAVE"] == pytest.approx(3.0, rel=1e-15)
    assert f["JVAR"] == 0.0 and f["VARIANCE"] == 0.0   # one occupied row level [A17]
    assert f["SUMAVE"] == pytest.approx(3.0 + float(np.sum(j * p)), rel=1e-14)
    assert f["CONTRAST"] == pytest.approx(float(np.sum((3 - j) ** 2 * p)), rel=1e-14)
    assert f["JE"] == pytest.approx(float(-np.sum(p * np.log2(p))), rel=1e-14)
    assert f["ACOR"] == pytest.approx(3.0 * float(np.sum(j * p)), rel=1e-14)


def test_centred_moments_of_one_value_are_exactly_zero(oracle_mod):
    """[A17] Sum and difference marginals concentrated on one value: the
    cluster moments, the sum variance and the difference variance are 0
    exactly, where summing with a rounded mean would leave ~1e-31; a matrix
    whose sum marginal has two values keeps the plain sums."""
    P = np.zeros((9, 9), np.uint64)
    P[0, 6] = P[6, 0] = 5; P[2, 4] = P[4, 2] = 3; P[3, 3] = 7    # i + j = 8 everywhere (0-based 6)
    f = dict(zip(NAMES, oracle_mod.features(P)))
    for k in ("CLUPROM", "CLUSHADE", "CLUTEND", "SUMVAR"):
        assert f[k] == 0.0, k
    assert f["SUMAVE"] == pytest.approx(8.0, rel=1e-15)
    Q = np.zeros((9, 9), np.uint64)
    Q[0, 2] = 4; Q[3, 5] = 1; Q[6, 8] = 6; Q[8, 6] = 2            # |i - j| = 2 everywhere
    g = dict(zip(NAMES, oracle_mod.features(Q)))
    assert g["DIFVAR"] == 0.0 and g["DIFAVE"] == pytest.approx(2.0, rel=1e-15)
    assert g["CONTRAST"] == pytest.approx(4.0, rel=1e-15)
    R = P.copy(); R[0, 0] = 1                                      # a second sum value
    h = dict(zip(NAMES, oracle_mod.features(R)))
    assert h["CLUTEND"] > 0 and h["SUMVAR"] == pytest.approx(h["CLUTEND"], rel=1e-12)
