"""Seeded synthetic workloads: intensity images + label masks.

Input generation only (no binning, counting or feature arithmetic lives here);
shared by the tests and the benchmark.  The recipes stand in for the paper's
workloads (Results, "Scalability" and Materials and methods, "Datasets"):
2D fluorescence-like images with many small cell regions (TissueNet-like),
3D volumes with few large regions (Decathlon-like), and a huge-region /
many-tiny-region tile for the ROI-size sweep.  No dataset item is reproduced.

Every array is produced by ``synth.c`` (SplitMix64, counter-based), so the
same seed gives the same bytes on any machine and thread count.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    P, i64, u64, d, i32, u32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_double, ctypes.c_int, ctypes.c_uint32)
    lib.synth_uniform12.argtypes = [u64, i64, P]
    lib.synth_blob_image.argtypes = [u64, i64, i64, i64, d, d, d, d, d, P]
    lib.synth_blob_images.argtypes = [P, i64, i64, i64, i64, d, d, d, d, d, P]
    lib.synth_grf_volume.argtypes = [u64, i64, i64, i64, d, d, d, d, P]
    lib.synth_ellipse_labels.restype = i64
    lib.synth_ellipse_labels.argtypes = [u64, i64, i64, i64, i32, d, d, d, d, d, d, u32,
                                         i64, i64, P]
    lib.synth_ellipse_label_images.argtypes = [P, i64, i64, i64, i64, i32, d, d, d, d, d, d,
                                               P, P]
    lib.synth_ellipsoid_labels.restype = i64
    lib.synth_ellipsoid_labels.argtypes = [u64, i64, i64, i64, i64, d, d, d, P]
    lib.synth_fill_rows.restype = i64
    lib.synth_fill_rows.argtypes = [i64, i64, d, u32, P]
    _lib = lib
    return lib


# ----------------------------------------------------------------- primitives
def uniform12(seed: int, shape) -> np.ndarray:
    out = np.empty(shape, np.uint16)
    _load().synth_uniform12(seed, out.size, out.ctypes.data)
    return out


def blob_image(seed: int, ny: int, nx: int, n_blobs: int, sigma=(3.0, 15.0),
               amp=(200.0, 2000.0), background=100.0) -> np.ndarray:
    out = np.empty((ny, nx), np.uint16)
    _load().synth_blob_image(seed, ny, nx, n_blobs, sigma[0], sigma[1], amp[0], amp[1],
                             background, out.ctypes.data)
    return out


def blob_images(seeds, ny: int, nx: int, n_blobs: int, sigma=(3.0, 15.0),
                amp=(200.0, 2000.0), background=100.0) -> np.ndarray:
    s = np.ascontiguousarray(seeds, np.uint64)
    out = np.empty((s.size, ny, nx), np.uint16)
    _load().synth_blob_images(s.ctypes.data, s.size, ny, nx, n_blobs, sigma[0], sigma[1],
                              amp[0], amp[1], background, out.ctypes.data)
    return out


def grf_volume(seed: int, nz: int, ny: int, nx: int, sigma=3.0, mean=1000.0, sd_g=250.0,
               sd_n=20.0) -> np.ndarray:
    out = np.empty((nz, ny, nx), np.uint16)
    _load().synth_grf_volume(seed, nz, ny, nx, sigma, mean, sd_g, sd_n, out.ctypes.data)
    return out


def ellipse_labels(seed: int, ny: int, nx: int, n_target: int, dist: str = "loguniform",
                   p0: float = 100.0, p1: float = 5000.0, lo: float = 0.0, hi: float = 1e18,
                   ratio_hi: float = 3.0, min_keep: float = 0.0, first_label: int = 1,
                   rows=None, out: np.ndarray | None = None) -> tuple[np.ndarray, int]:
    """Non-overlapping ellipses; dist 'loguniform' on [p0, p1] or 'lognormal'
    (median p0, log-sd p1, truncated to [lo, hi])."""
    o = np.zeros((ny, nx), np.uint32) if out is None else out
    r0, r1 = (0, ny) if rows is None else rows
    n = _load().synth_ellipse_labels(seed, ny, nx, n_target, 0 if dist == "loguniform" else 1,
                                     p0, p1, lo, hi, ratio_hi, min_keep, first_label, r0, r1,
                                     o.ctypes.data)
    return o, int(n)


def ellipse_label_images(seeds, ny: int, nx: int, n_target: int, dist: str = "lognormal",
                         p0: float = 800.0, p1: float = 1.0, lo: float = 20.0,
                         hi: float = 200000.0, ratio_hi: float = 3.0, min_keep: float = 20.0):
    s = np.ascontiguousarray(seeds, np.uint64)
    out = np.zeros((s.size, ny, nx), np.uint32)
    placed = np.zeros(s.size, np.int64)
    _load().synth_ellipse_label_images(s.ctypes.data, s.size, ny, nx, n_target,
                                       0 if dist == "loguniform" else 1, p0, p1, lo, hi,
                                       ratio_hi, min_keep, out.ctypes.data, placed.ctypes.data)
    return out, placed


def ellipsoid_labels(seed: int, nz: int, ny: int, nx: int, n_target: int, v_lo=1e3,
                     v_hi=60.0 ** 3, r_hi=2.0) -> tuple[np.ndarray, int]:
    out = np.zeros((nz, ny, nx), np.uint32)
    n = _load().synth_ellipsoid_labels(seed, nz, ny, nx, n_target, v_lo, v_hi, r_hi,
                                       out.ctypes.data)
    return out, int(n)


def fill_rows(labels2d: np.ndarray, frac: float, label: int) -> int:
    ny, nx = labels2d.shape
    return int(_load().synth_fill_rows(ny, nx, frac, label, labels2d.ctypes.data))


# ------------------------------------------------------------------ workloads
@dataclasses.dataclass
class Workload:
    name: str
    intensity: np.ndarray   # (n_images, nz, ny, nx) uint16
    labels: np.ndarray      # (n_images, nz, ny, nx) uint32, 0 = background
    n_bins: int
    dims: int               # 2 -> 4 offsets, 3 -> 13 offsets (distance 1)
    precision: str          # "fp64" or "fp32" feature output
    description: str

    @property
    def n_images(self) -> int:
        return self.intensity.shape[0]

    def roi_voxels(self) -> int:
        return int(np.count_nonzero(self.labels))


def _c1() -> Workload:
    I = uniform12(1, (1, 1, 64, 64))
    L = np.ones((1, 1, 64, 64), np.uint32)
    return Workload("c1_tiny", I, L, 8, 2, "fp64",
                    "2D 64x64 uniform [0,4095], whole image one ROI, 8 bins, 4 offsets, FP64")


def _c2(ny=2048, nx=2048, n_blobs=4000, n_rois=2000, seed=2, lseed=102, name="c2_cells") -> Workload:
    I = blob_image(seed, ny, nx, n_blobs)[None, None]
    L, _ = ellipse_labels(lseed, ny, nx, n_rois, "loguniform", 100.0, 5000.0, min_keep=100.0)
    return Workload(name, I, L[None, None], 256, 2, "fp32",
                    f"2D {ny}x{nx} blob image, ~{n_rois} ellipse ROIs of 100-5000 px, 256 bins")


def _c3(n_images=64, ny=2048, nx=2048, n_blobs=4000, n_rois=2344, name="c3_batch") -> Workload:
    I = blob_images([3000 + k for k in range(n_images)], ny, nx, n_blobs)
    L, _ = ellipse_label_images([3100 + k for k in range(n_images)], ny, nx, n_rois,
                                "lognormal", 800.0, 1.0, 20.0, 200000.0, 3.0, 20.0)
    return Workload(name, I[:, None], L[:, None], 64, 2, "fp32",
                    f"{n_images} x 2D {ny}x{nx}, ~{n_rois} log-normal ROIs per image "
                    "(median 800 px, 20-200000 px), 64 bins")


def _c4(nz=256, ny=512, nx=512, n_rois=500, name="c4_3d") -> Workload:
    I = grf_volume(4, nz, ny, nx)
    L, _ = ellipsoid_labels(104, nz, ny, nx, n_rois)
    return Workload(name, I[None], L[None], 64, 3, "fp32",
                    f"3D {nx}x{ny}x{nz} smoothed Gaussian field, ~{n_rois} ellipsoids "
                    "of 10^3-60^3 voxels, 64 bins, 13 offsets")


def _c5(n=8192, n_blobs=64000, n_small=10000, name="c5_stress", n_bins=1024) -> Workload:
    I = blob_image(5, n, n, n_blobs)
    L, _ = ellipse_labels(105, n, n, n_small, "loguniform", 30.0, 300.0, min_keep=30.0,
                          first_label=2)
    fill_rows(L, 0.9, 1)
    return Workload(name, I[None, None], L[None, None], n_bins, 2, "fp32",
                    f"2D {n}x{n}, one ROI over 90% of the tile plus {n_small} ROIs of "
                    f"30-300 px, {n_bins} bins, 64-bit counts")


def _small(name: str) -> Workload:
    """Reduced versions of each recipe, sized for the oracle (seconds) while
    still spanning several tiles and ragged edges."""
    if name == "c2_small":
        return _c2(ny=300, nx=333, n_blobs=60, n_rois=40, seed=22, lseed=122, name=name)
    if name == "c3_small":
        return _c3(n_images=3, ny=256, nx=250, n_blobs=60, n_rois=40, name=name)
    if name == "c4_small":
        I = grf_volume(44, 40, 48, 45)
        L, _ = ellipsoid_labels(144, 40, 48, 45, 12, v_lo=100.0, v_hi=6000.0)
        return Workload(name, I[None], L[None], 64, 3, "fp32", "3D 45x48x40 reduced C4 recipe")
    if name == "c5_small":
        return _c5(n=400, n_blobs=150, n_small=150, name=name)
    raise KeyError(name)


_BUILDERS = {"c1_tiny": _c1, "c2_cells": _c2, "c3_batch": _c3, "c4_3d": _c4, "c5_stress": _c5}
FULL = tuple(_BUILDERS)
SMALL = ("c2_small", "c3_small", "c4_small", "c5_small")


def make(name: str) -> Workload:
    if name in _BUILDERS:
        return _BUILDERS[name]()
    return _small(name)
