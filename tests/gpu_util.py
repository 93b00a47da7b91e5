"""Helpers for the GPU parity tests: device upload, oracle references and the
error measure of the precision contract.

Error of a feature value: |gpu - oracle| / max(|oracle|, M_f) with
  M_f = 1 for bounded features and for entropies (bits),
  M_f = sum |i + j - 2 mu|^3 p for cluster shade (the magnitude its signed
        terms sum from),
  M_f = 0 (plain relative error) otherwise.
NaN must match NaN.  The direction-mean block uses the mean of the M_f.
"""
from __future__ import annotations

import numpy as np

NAMES = ["ASM", "ACOR", "CLUPROM", "CLUSHADE", "CLUTEND", "CONTRAST", "CORR", "DIFAVE", "DIFENTRO", "DIFVAR",
         "DIS", "ENERGY", "ENTROPY", "HOM1", "HOM2", "IDM", "INFOMEAS1", "INFOMEAS2", "IDMN", "ID", "IDN", "IV",
         "JAVE", "JE", "JMAX", "SUMAVE", "SUMENT", "JVAR", "SUMVAR", "VARIANCE"]
UNIT_SCALE = {"ASM", "ENERGY", "JMAX", "CORR", "HOM1", "HOM2", "ID", "IDM", "IDN", "IDMN", "INFOMEAS1",
              "INFOMEAS2", "JE", "ENTROPY", "DIFENTRO", "SUMENT"}
SHADE = NAMES.index("CLUSHADE")


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
    mu = float((lv[:, None] * p).sum())
    s = lv[:, None] + lv[None, :] - 2 * mu
    return float((np.abs(s) ** 3 * p).sum())


def scales(Ps: np.ndarray) -> np.ndarray:
    """(K + 1, 30) floor M_f for one ROI from its (K, Ng, Ng) matrices."""
    K = Ps.shape[0]
    M = np.zeros((K + 1, 30))
    for q, n in enumerate(NAMES):
        if n in UNIT_SCALE:
            M[:, q] = 1.0
    valid = []
    for k in range(K):
        s = shade_scale(Ps[k])
        M[k, SHADE] = 0.0 if np.isnan(s) else s
        if not np.isnan(s):
            valid.append(s)
    M[K, SHADE] = float(np.mean(valid)) if valid else 0.0
    return M


def feature_errors(got: np.ndarray, want: np.ndarray, M: np.ndarray) -> np.ndarray:
    """Elementwise error; +inf where NaN-ness differs."""
    got = got.astype(np.float64)
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    err = np.abs(got - want) / np.maximum(np.abs(want), M)
    err = np.where(nan_g & nan_w, 0.0, err)
    err = np.where(nan_g != nan_w, np.inf, err)
    # exact zeros on both sides (0 / 0)
    err = np.where((got == want), 0.0, err)
    return err


def worst(err: np.ndarray):
    """(max error, feature name, index) for reporting."""
    i = np.unravel_index(np.nanargmax(err), err.shape)
    return float(err[i]), NAMES[i[-1]], i


def oracle_rois(oracle, w):
    """Per-image ROI statistics in the (image, label) order the library uses."""
    rows = []
    for k in range(w.n_images):
        st = oracle.roi_stats(w.intensity[k], w.labels[k])
        for r in range(st["label"].size):
            rows.append((k, r, st))
    return rows
