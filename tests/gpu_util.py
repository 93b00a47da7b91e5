"""Helpers for the GPU parity tests: device upload, oracle references and the
error measure of the precision contract.

Error of a feature value: |gpu - oracle| / max(|oracle|, M_f) with
  M_f = 1 for features bounded by 1 whose value can cancel to zero (CORR,
        INFOMEAS1, INFOMEAS2) and for entropies (bits),
  M_f = sum |i + j - mu_x - mu_y|^3 p for cluster shade (the magnitude its
        signed terms sum from),
  M_f = 0 (plain relative error) for every other feature: sums of
        non-negative terms (ASM, ENERGY, JMAX, the homogeneities, contrast,
        ...) and the even centred moments.
NaN must match NaN.  The direction-mean block uses the mean of the M_f.

Besides the bar, every comparison is recorded: the largest error per feature
under this measure and the strict relative error |gpu - oracle| / |oracle|
over values with |oracle| > 1e-3, per case; the table is written as JSON to
gpurun_out/parity_feature_errors.json when the session ends.
"""
from __future__ import annotations

import json
import os

import numpy as np

NAMES = ["ASM", "ACOR", "CLUPROM", "CLUSHADE", "CLUTEND", "CONTRAST", "CORR", "DIFAVE", "DIFENTRO", "DIFVAR",
         "DIS", "ENERGY", "ENTROPY", "HOM1", "HOM2", "IDM", "INFOMEAS1", "INFOMEAS2", "IDMN", "ID", "IDN", "IV",
         "JAVE", "JE", "JMAX", "SUMAVE", "SUMENT", "JVAR", "SUMVAR", "VARIANCE"]
UNIT_SCALE = {"CORR", "INFOMEAS1", "INFOMEAS2", "JE", "ENTROPY", "DIFENTRO", "SUMENT"}
SHADE = NAMES.index("CLUSHADE")
STRICT_FLOOR = 1e-3

_RECORD: dict = {}


def device_images(w, dev):
    import torch
    out = []
    for k in range(w.n_images):
        I = torch.from_numpy(np.ascontiguousarray(w.intensity[k]).view(np.int16)).to(dev)
        L = torch.from_numpy(np.ascontiguousarray(w.labels[k]).view(np.int32)).to(dev)
        out.append((I, L))
    return out


def shade_scale(P: np.ndarray) -> float:
    T = P.sum(dtype=np.float64)
    if T == 0:
        return np.nan
    p = P.astype(np.float64) / T
    ng = P.shape[0]
    lv = np.arange(1, ng + 1, dtype=np.float64)
    mux = float((lv[:, None] * p).sum())
    muy = float((lv[None, :] * p).sum())
    s = lv[:, None] + lv[None, :] - mux - muy
    return float((np.abs(s) ** 3 * p).sum())


def scales_from_magnitudes(mag) -> np.ndarray:
    """(K + 1, 30) floor M_f for one ROI from its K cluster-shade magnitudes
    (NaN for an empty direction)."""
    mag = np.asarray(mag, np.float64)
    K = mag.shape[0]
    M = np.zeros((K + 1, 30))
    for q, n in enumerate(NAMES):
        if n in UNIT_SCALE:
            M[:, q] = 1.0
    valid = ~np.isnan(mag)
    M[:K, SHADE] = np.where(valid, mag, 0.0)
    M[K, SHADE] = float(mag[valid].mean()) if valid.any() else 0.0
    return M


def scales(Ps: np.ndarray) -> np.ndarray:
    """(K + 1, 30) floor M_f for one ROI from its (K, Ng, Ng) matrices."""
    return scales_from_magnitudes([shade_scale(Ps[k]) for k in range(Ps.shape[0])])


def feature_errors(got: np.ndarray, want: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Elementwise error; +inf where NaN-ness differs."""
    got = got.astype(np.float64)
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    with np.errstate(divide="ignore", invalid="ignore"):
        err = np.abs(got - want) / np.maximum(np.abs(want), M)
    err = np.where(nan_g & nan_w, 0.0, err)
    err = np.where(nan_g != nan_w, np.inf, err)
    # exact zeros on both sides (0 / 0)
    err = np.where((got == want), 0.0, err)
    return err


def strict_errors(got: np.ndarray, want: np.ndarray) -> np.ndarray:
    """|gpu - oracle| / |oracle| where |oracle| > STRICT_FLOOR, else 0."""
    got = got.astype(np.float64)
    big = np.abs(want) > STRICT_FLOOR
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.abs(got - want) / np.abs(want)
    return np.where(big & np.isfinite(r), r, 0.0)


def worst(err: np.ndarray):
    """(max error, feature name, index) for reporting."""
    i = np.unravel_index(np.nanargmax(err), err.shape)
    return float(err[i]), NAMES[i[-1]], i


def record(case: str, err: np.ndarray, got: np.ndarray, want: np.ndarray, n_rois: int, tol: float) -> None:
    """Keeps the per-feature maxima of one comparison (err: (..., 30))."""
    e = err.reshape(-1, 30)
    s = strict_errors(got.reshape(-1, 30), want.reshape(-1, 30))
    prev = _RECORD.get(case)
    cur = {"rois": int(n_rois), "tolerance": tol,
           "max_error": {n: float(v) for n, v in zip(NAMES, e.max(axis=0))},
           "max_strict_relative": {n: float(v) for n, v in zip(NAMES, s.max(axis=0))}}
    if prev is not None:
        cur["rois"] += prev["rois"]
        for key in ("max_error", "max_strict_relative"):
            cur[key] = {n: max(cur[key][n], prev[key][n]) for n in NAMES}
    _RECORD[case] = cur


def write_record(root: str) -> str | None:
    if not _RECORD:
        return None
    out = os.path.join(root, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    path = os.path.join(out, "parity_feature_errors.json")
    with open(path, "w") as f:
        json.dump(_RECORD, f, indent=1, sort_keys=True)
    return path


def oracle_rois(oracle, w):
    """Per-image ROI statistics in the (image, label) order the library uses."""
    rows = []
    for k in range(w.n_images):
        st = oracle.roi_stats(w.intensity[k], w.labels[k])
        for r in range(st["label"].size):
            rows.append((k, r, st))
    return rows
