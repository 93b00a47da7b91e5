"""Pins of the neighbourhood texture oracle (oracle/neighbourhood.py: NGLDM,
NGTDM, GLDM) against what the definitions fix independently of it: a
hand-derived 3x3 golden, a constant ROI, a vectorised shift-based
recomputation of the per-voxel scan, count totals, the all-dependent limit
of a large alpha, and the invariances of a symmetric neighbourhood."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from oracle import neighbourhood as nb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "neighbourhood_3x3.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, expr = line.split()
        out[name] = float(eval(expr, {"__builtins__": {}, "log2": math.log2}))
    return out


def test_golden_3x3():
    I = np.array([[[1, 2, 1], [2, 3, 2], [1, 2, 1]]], np.uint16)
    got = dict(zip(nb.NAMES, nb.features(I, np.ones_like(I, bool), 3)))
    want = _golden()
    assert set(want) == set(nb.NAMES)
    for name in nb.NAMES:
        assert got[name] == pytest.approx(want[name], rel=1e-13, abs=1e-13), name


def test_constant_roi():
    """One level everywhere: no grey-tone difference (the flat-texture
    values), every neighbour dependent."""
    I = np.full((1, 4, 5), 9, np.uint16)
    M = np.ones_like(I, bool)
    f = dict(zip(nb.NAMES, nb.features(I, M, 8)))
    assert f["NGTDM_COARSENESS"] == nb.COARSENESS_FLAT
    for k in ("NGTDM_BUSYNESS", "NGTDM_COMPLEXITY", "NGTDM_CONTRAST", "NGTDM_STRENGTH", "NGLDM_GLV"):
        assert f[k] == 0.0, k
    S, n, s = nb.matrices(I, M, 8)
    # dependence = 1 + neighbours in the ROI: 3 at a corner, 5 on an edge, 8 inside
    assert S[0, 3] == 4 and S[0, 5] == 2 * (3 + 2) and S[0, 8] == 3 * 2 and S.sum() == 20
    assert f["NGLDM_GLM"] == 1.0 and f["NGLDM_GLNU"] == 20.0 and f["NGLDM_GLNUN"] == 1.0


def _scan_by_shifts(I, M, n_bins, alpha):
    """The per-voxel scan recomputed with whole-array shifts (a different
    algorithm from the oracle's voxel loop)."""
    nz = I.shape[0]
    offs = nb.neighbour_offsets(2 if nz == 1 else 3)
    vals = I[M].astype(np.int64)
    lev = np.zeros(I.shape, np.int64)
    lo, hi = int(vals.min()), int(vals.max())
    lev[M] = 1 if hi == lo else np.minimum(1 + (n_bins * (vals - lo)) // (hi - lo), n_bins)
    P = np.pad(lev, 1)
    Q = np.pad(M, 1)
    cnt = np.zeros(I.shape, np.int64)
    tot = np.zeros(I.shape, np.int64)
    dep = np.ones(I.shape, np.int64)
    core = (slice(1, -1),) * 3
    for dz, dy, dx in offs:
        sl = tuple(slice(1 + d, P.shape[a] - 1 + d) for a, d in enumerate((dz, dy, dx)))
        m = Q[sl]
        cnt += m
        tot += P[sl] * m
        dep += m & (np.abs(P[sl] - P[core]) <= alpha)
    S = np.zeros((n_bins, len(offs) + 1), np.int64)
    np.add.at(S, (lev[M] - 1, dep[M] - 1), 1)
    has = M & (cnt > 0)
    n = np.bincount(lev[has] - 1, minlength=n_bins)
    diff = np.abs(lev[has] - tot[has] / cnt[has])
    s = np.zeros(n_bins)
    np.add.at(s, lev[has] - 1, diff)
    return S, n, s


@pytest.mark.parametrize("shape,fill,n_bins,alpha,seed", [((1, 9, 11), 0.7, 8, 0, 1), ((1, 12, 7), 0.9, 30, 2, 2),
                                                          ((4, 5, 6), 0.6, 6, 0, 3), ((3, 6, 6), 0.95, 50, 5, 4)])
def test_scan_matches_shift_route(shape, fill, n_bins, alpha, seed):
    rng = np.random.default_rng(seed)
    I = rng.integers(0, 3000, shape).astype(np.uint16)
    M = rng.random(shape) < fill
    S, n, s = nb.matrices(I, M, n_bins, alpha)
    S2, n2, s2 = _scan_by_shifts(I, M, n_bins, alpha)
    assert np.array_equal(S, S2) and np.array_equal(n, n2)
    assert np.allclose(s, s2, rtol=1e-13, atol=1e-13)
    # every ROI voxel has one dependence; the level totals are the level histogram
    lev = nb.fbn_levels(I[M], int(I[M].min()), int(I[M].max()), n_bins)
    assert S.sum() == M.sum()
    assert np.array_equal(S.sum(axis=1), np.bincount(lev - 1, minlength=n_bins))


def test_large_alpha_counts_every_neighbour():
    rng = np.random.default_rng(9)
    I = rng.integers(0, 500, (1, 8, 10)).astype(np.uint16)
    M = rng.random(I.shape) < 0.8
    S, _, _ = nb.matrices(I, M, 16, alpha=16)
    # with every neighbour dependent, the dependence is 1 + the neighbours in the ROI
    Q = np.pad(M[0], 1)
    nbrs = sum(Q[1 + dy:Q.shape[0] - 1 + dy, 1 + dx:Q.shape[1] - 1 + dx].astype(int)
               for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0))
    assert np.array_equal(S.sum(axis=0), np.bincount(1 + nbrs[M[0]] - 1, minlength=9))


def test_invariances():
    """Transposing or flipping the image maps the neighbourhood onto itself;
    translation, label renaming and an increasing affine map of the
    intensities change nothing."""
    rng = np.random.default_rng(12)
    I = rng.integers(0, 4000, (1, 10, 13)).astype(np.uint16)
    L = rng.integers(0, 4, (1, 10, 13)).astype(np.uint32)
    _, t = nb.table(I, L, 10)
    eq = lambda a, b: np.allclose(a, b, rtol=1e-12, atol=1e-12, equal_nan=True)
    _, tt = nb.table(np.ascontiguousarray(I.transpose(0, 2, 1)), np.ascontiguousarray(L.transpose(0, 2, 1)), 10)
    assert eq(t, tt)
    _, tf = nb.table(np.ascontiguousarray(I[:, ::-1]), np.ascontiguousarray(L[:, ::-1]), 10)
    assert eq(t, tf)
    Ip = np.zeros((1, 14, 17), np.uint16); Lp = np.zeros((1, 14, 17), np.uint32)
    Ip[:, 3:13, 2:15] = I; Lp[:, 3:13, 2:15] = L
    assert eq(t, nb.table(Ip, Lp, 10)[1])
    assert eq(t, nb.table((3 * I.astype(np.int64) + 7).astype(np.uint16), L, 10)[1])
    perm = np.array([0, 3, 1, 2], np.uint32)
    labs, tp = nb.table(I, perm[L], 10)
    assert eq(t[[1, 2, 0]], tp)   # labels 1, 2, 3 became 3, 1, 2


def test_isolated_voxels():
    """Voxels with no neighbour in the ROI: dependence 1, no grey-tone
    difference entry; an ROI of such voxels only has NaN NGTDM features."""
    I = np.array([[[5, 0, 9], [0, 0, 0], [7, 0, 5]]], np.uint16)
    M = I > 0
    S, n, s = nb.matrices(I, M, 4)
    assert S[:, 0].sum() == 4 and S[:, 1:].sum() == 0 and n.sum() == 0
    f = dict(zip(nb.NAMES, nb.features(I, M, 4)))
    assert all(math.isnan(f["NGTDM_" + k]) for k in nb.NGTDM_NAMES)
    assert f["NGLDM_DCM"] == 1.0 and f["NGLDM_LDE"] == 1.0 and f["GLDM_SDE"] == 1.0
    assert f["NGLDM_DCV"] == 0.0 and f["GLDM_DV"] == 0.0   # one dependence value
