"""First-order intensity features per ROI -- TEST INFRASTRUCTURE ONLY.

A plain FP64 numpy reference for the intensity feature group of the paper
(Supplementary Table S1, "2-dimensional intensity features", the rows marked
NY; the 3D list of Table S5 holds the same statistics).  The paper prints no
formulas: it names the features and, in "Feature Control and Tunability",
states that first-order statistics take O(m) time in the voxel count m while
the entropy feature needs a histogram of a predefined number of intensity
bins h, O(m, h).  Each feature below is the usual statistical definition,
computed directly from the ROI's voxel values; readings of points the paper
leaves open carry [F#] labels (the design notes list them).

Only the test-suite may import this module; the product library never does.
It shares no code with the HIP path.
"""
from __future__ import annotations

import math

import numpy as np

# Column order of the intensity feature table.
NAMES = (
    "MEAN", "MIN", "MAX", "RANGE", "INTEGRATED_INTENSITY", "ENERGY", "RMS",
    "VARIANCE", "STDDEV", "STANDARD_ERROR", "SKEWNESS", "KURTOSIS", "HYPERSKEWNESS", "HYPERFLATNESS",
    "MEAN_ABSOLUTE_DEVIATION", "MEDIAN", "MEDIAN_ABSOLUTE_DEVIATION",
    "P01", "P10", "P25", "P75", "P90", "P99", "INTERQUARTILE_RANGE", "ROBUST_MEAN_ABSOLUTE_DEVIATION",
    "MODE", "ENTROPY", "UNIFORMITY", "UNIFORMITY_PIU",
    "WEIGHTED_CENTROID_X", "WEIGHTED_CENTROID_Y", "WEIGHTED_CENTROID_Z",
    "EDGE_INTEGRATED_INTENSITY", "EDGE_MIN", "EDGE_MAX", "EDGE_MEAN", "EDGE_STDDEV",
)
NFO = len(NAMES)
PERCENTILES = (1, 10, 25, 50, 75, 90, 99)


def fbn_levels(x: np.ndarray, vmin: int, vmax: int, n_bins: int) -> np.ndarray:
    """Fixed-bin-number levels 1..n_bins over [vmin, vmax], exact integers; a
    constant ROI is level 1 (the same discretisation as the texture
    features)."""
    x = x.astype(np.int64)
    if vmax == vmin:
        return np.ones(x.shape, np.int64)
    b = 1 + (n_bins * (x - vmin)) // (vmax - vmin)
    return np.minimum(b, n_bins)


def percentile_sorted(xs: np.ndarray, p: float) -> float:
    """Linear interpolation between the closest ranks [F3]: with the n values
    sorted ascending and h = (n - 1) p / 100, the value x_(floor h) +
    (h - floor h) (x_(floor h + 1) - x_(floor h))."""
    n = xs.size
    h = (n - 1) * p / 100.0
    lo = int(math.floor(h))
    hi = min(lo + 1, n - 1)
    return float(xs[lo]) + (h - lo) * (float(xs[hi]) - float(xs[lo]))


def _fsum(a) -> float:
    return math.fsum(np.asarray(a, np.float64).ravel().tolist())


def edge_mask(mask: np.ndarray) -> np.ndarray:
    """ROI voxels with at least one face neighbour (4 in a 2D image, 6 in a
    volume) outside the image or outside the ROI [F10]; mask is (nz, ny, nx)
    boolean."""
    nz = mask.shape[0]
    pad = np.pad(mask, 1, constant_values=False)
    inner = pad[1:-1, 1:-1, 1:-1]
    all_in = inner.copy()
    axes = (1, 2) if nz == 1 else (0, 1, 2)
    for ax in axes:
        for s in (-1, 1):
            all_in &= np.roll(pad, s, axis=ax)[1:-1, 1:-1, 1:-1]
    return mask & ~all_in


def features(I: np.ndarray, mask: np.ndarray, n_bins: int) -> np.ndarray:
    """The NFO intensity features of one ROI: I is the (nz, ny, nx) intensity
    image, mask the ROI's voxels.  Returns float64[NFO] in NAMES order."""
    I = np.asarray(I)
    x = I[mask].astype(np.float64)
    n = x.size
    out = np.full(NFO, np.nan)
    if n == 0:
        return out
    f = dict.fromkeys(NAMES, np.nan)
    s1 = _fsum(x)
    mu = s1 / n
    f["MEAN"] = mu
    f["MIN"] = float(x.min())
    f["MAX"] = float(x.max())
    f["RANGE"] = f["MAX"] - f["MIN"]
    f["INTEGRATED_INTENSITY"] = s1
    f["ENERGY"] = _fsum(x * x)
    f["RMS"] = math.sqrt(f["ENERGY"] / n)
    d = x - mu
    m = {k: _fsum(d ** k) / n for k in (2, 3, 4, 5, 6)}
    # unbiased variance [F1]; a single voxel has variance 0
    f["VARIANCE"] = m[2] * n / (n - 1) if n > 1 else 0.0
    f["STDDEV"] = math.sqrt(f["VARIANCE"])
    f["STANDARD_ERROR"] = f["STDDEV"] / math.sqrt(n)
    # standardised central moments of the biased moments; 0 for a constant ROI [F2]
    if m[2] > 0:
        f["SKEWNESS"] = m[3] / m[2] ** 1.5
        f["KURTOSIS"] = m[4] / m[2] ** 2
        f["HYPERSKEWNESS"] = m[5] / m[2] ** 2.5
        f["HYPERFLATNESS"] = m[6] / m[2] ** 3
    else:
        f["SKEWNESS"] = f["KURTOSIS"] = f["HYPERSKEWNESS"] = f["HYPERFLATNESS"] = 0.0
    f["MEAN_ABSOLUTE_DEVIATION"] = _fsum(np.abs(d)) / n
    xs = np.sort(x)
    pv = {p: percentile_sorted(xs, p) for p in PERCENTILES}
    f["MEDIAN"] = pv[50]
    # mean distance to the median [F4]
    f["MEDIAN_ABSOLUTE_DEVIATION"] = _fsum(np.abs(x - pv[50])) / n
    for p in (1, 10, 25, 75, 90, 99):
        f[f"P{p:02d}"] = pv[p]
    f["INTERQUARTILE_RANGE"] = pv[75] - pv[25]
    # mean distance to the mean of the values within [P10, P90] [F5]; undefined
    # (NaN) when no value lies there, which happens for two distinct values
    sub = x[(x >= pv[10]) & (x <= pv[90])]
    if sub.size:
        mus = _fsum(sub) / sub.size
        f["ROBUST_MEAN_ABSOLUTE_DEVIATION"] = _fsum(np.abs(sub - mus)) / sub.size
    # histogram of the fixed-bin-number levels [F6]
    lv = fbn_levels(I[mask], int(x.min()), int(x.max()), n_bins)
    cnt = np.bincount(lv, minlength=n_bins + 1)[1:]
    f["MODE"] = float(1 + int(np.argmax(cnt)))      # lowest level among ties [F7]
    pb = cnt[cnt > 0] / n
    f["ENTROPY"] = -_fsum(pb * np.log2(pb))
    f["UNIFORMITY"] = _fsum(pb * pb)
    # percent image uniformity [F8]
    tot = f["MAX"] + f["MIN"]
    f["UNIFORMITY_PIU"] = 100.0 * (1.0 - (f["MAX"] - f["MIN"]) / tot) if tot > 0 else 100.0
    # intensity-weighted centroid in image coordinates (column x, row y, plane z) [F9]
    zz, yy, xx = np.nonzero(mask)
    if s1 > 0:
        f["WEIGHTED_CENTROID_X"] = _fsum(xx * x) / s1
        f["WEIGHTED_CENTROID_Y"] = _fsum(yy * x) / s1
        f["WEIGHTED_CENTROID_Z"] = _fsum(zz * x) / s1
    e = I[edge_mask(mask)].astype(np.float64)
    ne = e.size
    f["EDGE_INTEGRATED_INTENSITY"] = _fsum(e)
    f["EDGE_MIN"] = float(e.min())
    f["EDGE_MAX"] = float(e.max())
    f["EDGE_MEAN"] = f["EDGE_INTEGRATED_INTENSITY"] / ne
    f["EDGE_STDDEV"] = math.sqrt(_fsum((e - f["EDGE_MEAN"]) ** 2) / (ne - 1)) if ne > 1 else 0.0
    return np.array([f[k] for k in NAMES], np.float64)


def table(I: np.ndarray, L: np.ndarray, n_bins: int) -> tuple[np.ndarray, np.ndarray]:
    """(labels ascending, features (n_rois, NFO)) for every nonzero label of
    one (nz, ny, nx) image."""
    labels = np.unique(L[L != 0])
    out = np.empty((labels.size, NFO))
    for r, lab in enumerate(labels):
        out[r] = features(I, L == lab, n_bins)
    return labels, out


def magnitude(I: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Error floors for the parity tests, not features: for the odd
    standardised moments the magnitude their signed terms sum from,
    (sum |x - mu|^k / n) / m2^(k/2); 0 elsewhere (plain relative error)."""
    x = I[mask].astype(np.float64)
    M = np.zeros(NFO)
    d = np.abs(x - x.mean())
    m2 = float(np.mean(d * d))
    if m2 > 0:
        M[NAMES.index("SKEWNESS")] = float(np.mean(d ** 3)) / m2 ** 1.5
        M[NAMES.index("HYPERSKEWNESS")] = float(np.mean(d ** 5)) / m2 ** 2.5
    return M
