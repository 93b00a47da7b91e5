"""FP64 CPU oracle for per-ROI GLCM texture -- TEST INFRASTRUCTURE ONLY.

This package wraps ``oracle.c`` (plain C, binary64, Neumaier sums) with ctypes
and numpy.  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product library never does.  It shares no
code with the HIP path.

Definitions follow the paper's problem statement (one row of measurements per
unique nonzero label of the mask, Supplementary Table S7) and its GLCM feature
list (Supplementary Table S3, rows 140-174 marked NY; 3D: Table S5, row 361),
with the standard IBSI formulas the paper defers to.  Readings of points the
paper leaves open carry [A#] labels where they are applied.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NFEAT = 30


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.oracle_feature_count.restype = i32
    lib.oracle_feature_name.restype = ctypes.c_char_p
    lib.oracle_feature_name.argtypes = [i32]
    lib.oracle_bin.restype = u32
    lib.oracle_bin.argtypes = [u32, u32, u32, i32]
    lib.oracle_roi_count.restype = i64
    lib.oracle_roi_count.argtypes = [P, i64]
    lib.oracle_roi_stats.restype = i64
    lib.oracle_roi_stats.argtypes = [P, P, i64, i64, i64, i64, P, P, P, P, P]
    lib.oracle_bin_image.restype = ctypes.c_int
    lib.oracle_bin_image.argtypes = [P, P, i64, i64, P, P, P, i32, P]
    lib.oracle_glcm_roi.restype = ctypes.c_int
    lib.oracle_glcm_roi.argtypes = [P, P, i64, i64, i64, u32, ctypes.c_uint16,
                                    ctypes.c_uint16, P, i32, P, i32, i32, P]
    lib.oracle_features.restype = None
    lib.oracle_features.argtypes = [P, i32, P]
    lib.oracle_features_roi.restype = None
    lib.oracle_features_roi.argtypes = [P, i32, i32, P]
    lib.oracle_extract.restype = ctypes.c_int
    lib.oracle_extract.argtypes = [P, P, i64, i64, i64, i32, P, i32, i64,
                                   P, P, P, P, P, P, i32, i32]
    lib.oracle_shade_magnitude.restype = ctypes.c_double
    lib.oracle_shade_magnitude.argtypes = [P, i32]
    lib.oracle_default_offsets.restype = i32
    lib.oracle_default_offsets.argtypes = [i32, i32, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _img3(a: np.ndarray, dtype) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.ndim == 2:
        a = a[None]
    if a.ndim != 3:
        raise ValueError("expected a 2D or 3D array")
    return a


def feature_names() -> list[str]:
    lib = _load()
    return [lib.oracle_feature_name(f).decode() for f in range(lib.oracle_feature_count())]


def default_offsets(dims: int, distance: int = 1) -> np.ndarray:
    """(K, 3) int32 array of (dz, dy, dx) offsets: K = 4 in 2D, 13 in 3D."""
    lib = _load()
    out = np.zeros((13, 3), np.int32)
    k = lib.oracle_default_offsets(dims, distance, _ptr(out))
    if k < 0:
        raise ValueError("dims must be 2 or 3")
    return out[:k].copy()


def bin_value(intensity: int, vmin: int, vmax: int, n_bins: int) -> int:
    return int(_load().oracle_bin(intensity, vmin, vmax, n_bins))


def roi_stats(intensity: np.ndarray, labels: np.ndarray) -> dict:
    """Per-ROI statistics of one image, ascending label order.

    Returns dict(label u32, count u64, vmin u16, vmax u16, bbox (n, 6) i32 with
    x_min, y_min, z_min, x_max, y_max, z_max inclusive)."""
    lib = _load()
    I = _img3(intensity, np.uint16)
    L = _img3(labels, np.uint32)
    if I.shape != L.shape:
        raise ValueError("intensity and labels differ in shape")
    nz, ny, nx = I.shape
    n = lib.oracle_roi_count(_ptr(L), L.size)
    label = np.zeros(max(n, 1), np.uint32)
    count = np.zeros(max(n, 1), np.uint64)
    vmin = np.zeros(max(n, 1), np.uint16)
    vmax = np.zeros(max(n, 1), np.uint16)
    bbox = np.zeros((max(n, 1), 6), np.int32)
    got = lib.oracle_roi_stats(_ptr(I), _ptr(L), nz, ny, nx, n, _ptr(label), _ptr(count),
                               _ptr(vmin), _ptr(vmax), _ptr(bbox))
    if got != n:
        raise RuntimeError("oracle_roi_stats failed")
    return dict(label=label[:n], count=count[:n], vmin=vmin[:n], vmax=vmax[:n], bbox=bbox[:n])


def bin_image(intensity: np.ndarray, labels: np.ndarray, n_bins: int, stats: dict | None = None) -> np.ndarray:
    """Level of every ROI voxel under its own ROI's range; 0 for background."""
    lib = _load()
    I = _img3(intensity, np.uint16)
    L = _img3(labels, np.uint32)
    st = stats if stats is not None else roi_stats(I, L)
    out = np.zeros(I.shape, np.uint16)
    lab = np.ascontiguousarray(st["label"], np.uint32)
    lo = np.ascontiguousarray(st["vmin"], np.uint16)
    hi = np.ascontiguousarray(st["vmax"], np.uint16)
    rc = lib.oracle_bin_image(_ptr(I), _ptr(L), I.size, lab.size, _ptr(lab), _ptr(lo), _ptr(hi),
                              n_bins, _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle_bin_image failed")
    return out


def glcm_roi(intensity, labels, label: int, vmin: int, vmax: int, bbox, n_bins: int,
             offsets: np.ndarray, symmetric: bool = True) -> np.ndarray:
    """(K, Ng, Ng) uint64 co-occurrence matrices of one ROI: symmetric
    P = C + C^T [A6], or the ordered counts C when symmetric is False [A16]."""
    lib = _load()
    I = _img3(intensity, np.uint16)
    L = _img3(labels, np.uint32)
    nz, ny, nx = I.shape
    off = np.ascontiguousarray(offsets, np.int32).reshape(-1, 3)
    bb = np.ascontiguousarray(bbox, np.int32).reshape(6)
    P = np.zeros((off.shape[0], n_bins, n_bins), np.uint64)
    lib.oracle_glcm_roi(_ptr(I), _ptr(L), nz, ny, nx, int(label), int(vmin), int(vmax), _ptr(bb),
                        n_bins, _ptr(off), off.shape[0], 1 if symmetric else 0, _ptr(P))
    return P


def features(P: np.ndarray) -> np.ndarray:
    """The 30 features of one (Ng, Ng) count matrix (symmetric or not)."""
    lib = _load()
    M = np.ascontiguousarray(P, np.uint64)
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("expected a square matrix")
    out = np.zeros(NFEAT, np.float64)
    lib.oracle_features(_ptr(M), M.shape[0], _ptr(out))
    return out


def features_roi(P: np.ndarray) -> np.ndarray:
    """(K + 1, 30): per-direction features then the mean over non-empty directions."""
    lib = _load()
    M = np.ascontiguousarray(P, np.uint64)
    K, ng, _ = M.shape
    out = np.zeros((K + 1, NFEAT), np.float64)
    lib.oracle_features_roi(_ptr(M), ng, K, _ptr(out))
    return out


def features_roi_merged(P: np.ndarray) -> np.ndarray:
    """(1, 30): the features of the sum of the K direction matrices of one ROI
    (the offsets' counts pooled into one symmetric matrix before any feature
    is taken; reading A15)."""
    M = np.ascontiguousarray(P, np.uint64)
    if M.ndim != 3 or M.shape[1] != M.shape[2]:
        raise ValueError("expected (K, Ng, Ng) matrices")
    return features(M.sum(axis=0, dtype=np.uint64))[None, :]


def shade_magnitude(P: np.ndarray) -> float:
    """sum |i + j - mux - muy|^3 p of one (Ng, Ng) count matrix: the
    magnitude the signed cluster-shade sum is formed from (the parity tests'
    error scale for that feature); NaN for an empty matrix."""
    M = np.ascontiguousarray(P, np.uint64)
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("expected a square matrix")
    return float(_load().oracle_shade_magnitude(_ptr(M), M.shape[0]))


def extract(intensity, labels, n_bins: int, offsets: np.ndarray, stats: dict | None = None,
            rois=None, n_threads: int = 1, want_shade_magnitude: bool = False, symmetric: bool = True):
    """Feature table of one image: (stats, table (n, K + 1, 30) float64),
    plus the (n, K) cluster-shade magnitudes (shade_magnitude of each
    direction's matrix) when want_shade_magnitude is set.

    ``rois`` optionally selects ROI indices (into the ascending-label order);
    the table then has one row per selected ROI."""
    lib = _load()
    I = _img3(intensity, np.uint16)
    L = _img3(labels, np.uint32)
    nz, ny, nx = I.shape
    st = stats if stats is not None else roi_stats(I, L)
    idx = np.arange(st["label"].size) if rois is None else np.asarray(rois, np.int64)
    lab = np.ascontiguousarray(st["label"][idx], np.uint32)
    lo = np.ascontiguousarray(st["vmin"][idx], np.uint16)
    hi = np.ascontiguousarray(st["vmax"][idx], np.uint16)
    bb = np.ascontiguousarray(st["bbox"][idx], np.int32)
    off = np.ascontiguousarray(offsets, np.int32).reshape(-1, 3)
    K = off.shape[0]
    table = np.zeros((idx.size, K + 1, NFEAT), np.float64)
    mag = np.zeros((idx.size, K), np.float64) if want_shade_magnitude else None
    rc = lib.oracle_extract(_ptr(I), _ptr(L), nz, ny, nx, n_bins, _ptr(off), K, idx.size,
                            _ptr(lab), _ptr(lo), _ptr(hi), _ptr(bb), _ptr(table),
                            _ptr(mag) if mag is not None else None, 1 if symmetric else 0, n_threads)
    if rc != 0:
        raise RuntimeError("oracle_extract failed")
    return (st, table, mag) if want_shade_magnitude else (st, table)
