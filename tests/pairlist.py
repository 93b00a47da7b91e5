"""Independent route to the GLCM quantities, used to pin the oracle.

Instead of building a co-occurrence matrix and applying the matrix formulas,
this module enumerates the ROI's voxel pairs by brute force (all pairs of ROI
voxels whose coordinate difference equals the offset, O(n^2)) and computes
every feature as a statistic of the list of ordered level pairs (x, y) taken
in both orders, with numpy / scipy / scikit-learn routines: means, variances,
central moments, Pearson correlation, histogram entropies and the mutual
information score.  A wrong term, sign, index or operand in the oracle's
matrix formulas therefore shows up as a mismatch.

Only for tiny ROIs (tens of voxels).
"""
from __future__ import annotations

import math
from collections import Counter

import numpy as np
from scipy import stats
from sklearn.metrics import mutual_info_score


def ordered_pairs(bins: np.ndarray, labels: np.ndarray, label: int, offset) -> np.ndarray:
    """All (b_v, b_w) with v, w voxels of the ROI and coords(w) - coords(v) = offset,
    found by testing every pair of ROI voxels.  bins/labels are (nz, ny, nx)."""
    coords = np.argwhere(labels == label)  # (n, 3) as z, y, x
    d = np.asarray(offset, np.int64)
    diff = coords[None, :, :] - coords[:, None, :]          # [a, b] = coords[b] - coords[a]
    a_idx, b_idx = np.nonzero(np.all(diff == d, axis=2))     # every pair of ROI voxels tested
    bv = bins[tuple(coords[a_idx].T)].astype(np.int64)
    bw = bins[tuple(coords[b_idx].T)].astype(np.int64)
    return np.stack([bv, bw], axis=1).reshape(-1, 2)


def count_matrix(pairs: np.ndarray, n_bins: int, symmetric: bool = True) -> np.ndarray:
    """Counts from brute-force ordered pairs: both orders (symmetric), or
    each pair once in its own order."""
    P = np.zeros((n_bins, n_bins), np.uint64)
    for x, y in pairs:
        P[x - 1, y - 1] += 1
        if symmetric:
            P[y - 1, x - 1] += 1
    return P


def _entropy_bits(values) -> float:
    c = np.array(list(Counter(values).values()), float)
    return float(stats.entropy(c, base=2))


def features_from_pairs(pairs: np.ndarray, n_bins: int, symmetric: bool = True) -> dict:
    """The 30 features from the pair list (both orders when symmetric, else
    each pair in its own order: x the level at v, y the level at v + d), via
    library statistics."""
    if len(pairs) == 0:
        return None
    if symmetric:
        x = np.concatenate([pairs[:, 0], pairs[:, 1]]).astype(float)
        y = np.concatenate([pairs[:, 1], pairs[:, 0]]).astype(float)
    else:
        x = pairs[:, 0].astype(float)
        y = pairs[:, 1].astype(float)
    s = x + y
    d = x - y
    ad = np.abs(d)
    joint = Counter(zip(x.tolist(), y.tolist()))
    q = np.array(list(joint.values()), float) / len(x)
    f = {}
    f["ASM"] = f["ENERGY"] = float(np.sum(q ** 2))
    f["ACOR"] = float(np.mean(x * y))
    f["CLUPROM"] = float(stats.moment(s, 4))
    f["CLUSHADE"] = float(stats.moment(s, 3))
    f["CLUTEND"] = float(np.var(s))
    f["CONTRAST"] = float(np.mean(d ** 2))
    # one level in either coordinate: the correlation is 0/0 and the mutual
    # information exactly 0
    single = len(np.unique(x)) == 1 or len(np.unique(y)) == 1
    f["CORR"] = 1.0 if single else float(np.corrcoef(x, y)[0, 1])
    f["DIFAVE"] = float(np.mean(ad))
    f["DIFENTRO"] = _entropy_bits(ad.tolist())
    f["DIFVAR"] = float(np.var(ad))
    f["DIS"] = float(np.mean(ad))
    hxy = float(stats.entropy(q, base=2))
    f["ENTROPY"] = f["JE"] = hxy
    f["HOM1"] = f["ID"] = float(np.mean(1.0 / (1.0 + ad)))
    f["HOM2"] = f["IDM"] = float(np.mean(1.0 / (1.0 + d ** 2)))
    hx = _entropy_bits(x.tolist())
    hy = _entropy_bits(y.tolist())
    mi = mutual_info_score(x.astype(int), y.astype(int)) / math.log(2.0)  # bits
    f["INFOMEAS1"] = 0.0 if single else -mi / max(hx, hy)
    f["INFOMEAS2"] = 0.0 if single else math.sqrt(1.0 - math.exp(-2.0 * max(mi, 0.0)))
    f["IDMN"] = float(np.mean(1.0 / (1.0 + d ** 2 / n_bins ** 2)))
    f["IDN"] = float(np.mean(1.0 / (1.0 + ad / n_bins)))
    nz = d != 0
    f["IV"] = float(np.sum(1.0 / d[nz] ** 2) / len(d))
    f["JAVE"] = float(np.mean(x))
    f["JMAX"] = float(np.max(q))
    f["SUMAVE"] = float(np.mean(s))
    f["SUMENT"] = _entropy_bits(s.tolist())
    f["JVAR"] = f["VARIANCE"] = float(np.var(x))
    f["SUMVAR"] = float(np.var(s))
    return f
