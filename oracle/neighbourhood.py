"""Neighbourhood texture features per ROI -- TEST INFRASTRUCTURE ONLY.

A plain FP64 numpy reference for three texture families of the paper's
feature list that share one per-voxel neighbourhood scan: the neighbouring
grey level dependence matrix (NGLDM, Supplementary Table S3 rows 175-192),
the neighbourhood grey tone difference matrix (NGTDM, rows 246-250) and the
grey level dependence matrix (GLDM, rows 251-264), the rows marked NY.  The
paper names the features only (Materials and methods, "Feature Control and
Tunability" treats texture cost as growing with voxels, grey levels and
neighbourhood); each definition below is the usual one for these matrices,
computed by an explicit loop over every ROI voxel and its neighbours.
Readings of points the paper leaves open carry [N#] labels (the design notes
list them).

Only the test-suite may import this module; the product library never does.
It shares no code with the HIP path.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

NGLDM_NAMES = ("DCENRG", "DCENT", "DCNU", "DCNUN", "DCM", "DCV", "GLNU", "GLNUN", "GLM", "GLV", "HDE", "HDHGLE",
               "HDLGLE", "HGLCE", "LDE", "LDHGLE", "LDLGLE", "LGLCE")
NGTDM_NAMES = ("BUSYNESS", "COARSENESS", "COMPLEXITY", "CONTRAST", "STRENGTH")
GLDM_NAMES = ("SDE", "LDE", "GLN", "DN", "DNN", "GLV", "DV", "DE", "LGLE", "HGLE", "SDLGLE", "SDHGLE", "LDLGLE",
              "LDHGLE")
NAMES = (tuple("NGLDM_" + n for n in NGLDM_NAMES) + tuple("NGTDM_" + n for n in NGTDM_NAMES) +
         tuple("GLDM_" + n for n in GLDM_NAMES))
NNF = len(NAMES)
COARSENESS_FLAT = 1.0e6   # [N3]


def fbn_levels(x: np.ndarray, vmin: int, vmax: int, n_bins: int) -> np.ndarray:
    """Fixed-bin-number levels 1..n_bins over [vmin, vmax] (exact integers; a
    constant ROI is level 1), the texture features' discretisation."""
    x = np.asarray(x, np.int64)
    if vmax == vmin:
        return np.ones(x.shape, np.int64)
    return np.minimum(1 + (n_bins * (x - vmin)) // (vmax - vmin), n_bins)


def neighbour_offsets(dims: int) -> list[tuple[int, int, int]]:
    """Chebyshev distance 1 [N1]: the 8 in-plane neighbours of a 2D image, the
    26 of a volume, as (dz, dy, dx)."""
    zs = (0,) if dims == 2 else (-1, 0, 1)
    return [(dz, dy, dx) for dz, dy, dx in itertools.product(zs, (-1, 0, 1), (-1, 0, 1)) if (dz, dy, dx) != (0, 0, 0)]


def matrices(I: np.ndarray, mask: np.ndarray, n_bins: int, alpha: int = 0):
    """Per-voxel neighbourhood scan of one ROI (I, mask: (nz, ny, nx)).

    Returns (S, n, s): S the dependence matrix, S[i - 1, k - 1] = voxels of
    level i with dependence k, k = 1 + the number of neighbours inside the
    ROI whose level differs by at most alpha [N4, N5]; n[i - 1] the voxels of
    level i with at least one neighbour in the ROI and s[i - 1] the sum over
    them of |i - mean level of those neighbours| [N2]."""
    nz, ny, nx = I.shape
    dims = 2 if nz == 1 else 3
    offs = neighbour_offsets(dims)
    vals = I[mask]
    lev = np.zeros(I.shape, np.int64)
    lev[mask] = fbn_levels(vals, int(vals.min()), int(vals.max()), n_bins)
    S = np.zeros((n_bins, len(offs) + 1), np.int64)
    n = np.zeros(n_bins, np.int64)
    s = np.zeros(n_bins, np.float64)
    s_terms = [[] for _ in range(n_bins)]
    for z, y, x in zip(*np.nonzero(mask)):
        i = int(lev[z, y, x])
        k = 1
        tot, cnt = 0, 0
        for dz, dy, dx in offs:
            wz, wy, wx = z + dz, y + dy, x + dx
            if 0 <= wz < nz and 0 <= wy < ny and 0 <= wx < nx and mask[wz, wy, wx]:
                j = int(lev[wz, wy, wx])
                cnt += 1
                tot += j
                if abs(j - i) <= alpha:
                    k += 1
        S[i - 1, k - 1] += 1
        if cnt:
            n[i - 1] += 1
            s_terms[i - 1].append(abs(i - tot / cnt))
    for i in range(n_bins):
        s[i] = math.fsum(s_terms[i])
    return S, n, s


def _fsum(a) -> float:
    return math.fsum(np.asarray(a, np.float64).ravel().tolist())


def dependence_features(S: np.ndarray) -> dict:
    """The NGLDM and GLDM features of one dependence matrix (levels i and
    dependences k both 1-based), with p = S / Ns, Ns = the ROI's voxels."""
    Ns = int(S.sum())
    ng, nk = S.shape
    i = np.arange(1, ng + 1, dtype=np.float64)[:, None]
    k = np.arange(1, nk + 1, dtype=np.float64)[None, :]
    p = S.astype(np.float64) / Ns
    rows = S.sum(axis=1).astype(np.float64)   # per level
    cols = S.sum(axis=0).astype(np.float64)   # per dependence
    glm = _fsum(i * p)
    dcm = _fsum(k * p)
    nz = p > 0
    f = {
        "DCENRG": _fsum(p * p),
        "DCENT": -_fsum(p[nz] * np.log2(p[nz])),   # 0 log 0 = 0 [N6]
        "DCNU": _fsum(cols * cols) / Ns,
        "DCNUN": _fsum(cols * cols) / (float(Ns) * Ns),
        "DCM": dcm,
        "DCV": _fsum((k - dcm) ** 2 * p),
        "GLNU": _fsum(rows * rows) / Ns,
        "GLNUN": _fsum(rows * rows) / (float(Ns) * Ns),
        "GLM": glm,
        "GLV": _fsum((i - glm) ** 2 * p),
        "HDE": _fsum(k * k * p),
        "HDHGLE": _fsum(i * i * k * k * p),
        "HDLGLE": _fsum(k * k / (i * i) * p),
        "HGLCE": _fsum(i * i * p),
        "LDE": _fsum(p / (k * k)),
        "LDHGLE": _fsum(i * i / (k * k) * p),
        "LDLGLE": _fsum(p / (i * i * k * k)),
        "LGLCE": _fsum(p / (i * i)),
    }
    # a variance of a distribution on one value is exactly 0 [A17 of the
    # GLCM readings, decided on the integer counts]
    if np.count_nonzero(rows) == 1:
        f["GLV"] = 0.0
    if np.count_nonzero(cols) == 1:
        f["DCV"] = 0.0
    # the GLDM names of the same quantities [N7]
    g = {"SDE": f["LDE"], "LDE": f["HDE"], "GLN": f["GLNU"], "DN": f["DCNU"], "DNN": f["DCNUN"], "GLV": f["GLV"],
         "DV": f["DCV"], "DE": f["DCENT"], "LGLE": f["LGLCE"], "HGLE": f["HGLCE"], "SDLGLE": f["LDLGLE"],
         "SDHGLE": f["LDHGLE"], "LDLGLE": f["HDLGLE"], "LDHGLE": f["HDHGLE"]}
    return f, g


def ngtdm_features(n: np.ndarray, s: np.ndarray) -> dict:
    """The NGTDM features from the per-level counts n and sums s; p_i =
    n_i / Nvp over the levels present.  NaN when no voxel has a neighbour in
    the ROI [N2]; the flat-texture values of [N3]."""
    Nvp = int(n.sum())
    out = dict.fromkeys(NGTDM_NAMES, np.nan)
    if Nvp == 0:
        return out
    lv = np.nonzero(n)[0]
    i = (lv + 1).astype(np.float64)
    p = n[lv].astype(np.float64) / Nvp
    si = s[lv]
    ps = _fsum(p * si)
    ssum = _fsum(s)
    ngp = lv.size
    pi, pj = p[:, None], p[None, :]
    ii, jj = i[:, None], i[None, :]
    sI, sJ = si[:, None], si[None, :]
    out["COARSENESS"] = 1.0 / ps if ps > 0 else COARSENESS_FLAT
    out["CONTRAST"] = (_fsum(pi * pj * (ii - jj) ** 2) / (ngp * (ngp - 1)) * ssum / Nvp) if ngp > 1 else 0.0
    den = _fsum(np.abs(ii * pi - jj * pj))
    out["BUSYNESS"] = ps / den if den > 0 else 0.0
    out["COMPLEXITY"] = _fsum(np.abs(ii - jj) * (pi * sI + pj * sJ) / (pi + pj)) / Nvp
    out["STRENGTH"] = _fsum((pi + pj) * (ii - jj) ** 2) / ssum if ssum > 0 else 0.0
    return out


def features(I: np.ndarray, mask: np.ndarray, n_bins: int, alpha: int = 0) -> np.ndarray:
    """The NNF features of one ROI in NAMES order (float64)."""
    I = np.asarray(I)
    S, n, s = matrices(I, mask, n_bins, alpha)
    f, g = dependence_features(S)
    t = ngtdm_features(n, s)
    return np.array([f[k] for k in NGLDM_NAMES] + [t[k] for k in NGTDM_NAMES] + [g[k] for k in GLDM_NAMES],
                    np.float64)


def table(I: np.ndarray, L: np.ndarray, n_bins: int, alpha: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """(labels ascending, features (n_rois, NNF)) for every nonzero label of
    one (nz, ny, nx) image."""
    labels = np.unique(L[L != 0])
    out = np.empty((labels.size, NNF))
    for r, lab in enumerate(labels):
        out[r] = features(I, L == lab, n_bins, alpha)
    return labels, out
