"""ctypes binding of libnyx.so (include/nyx.h): same names, argument marshalling only.

Every step of the path runs in the HIP kernels of libnyx.so; this module only
turns torch device tensors into pointers and sizes, and status codes into
exceptions.  There is no CPU fallback: if the library is missing or no GPU is
present, calls raise.

torch is imported before the library is loaded, so libnyx.so binds to the HIP
runtime torch already loaded (same soname), and torch streams and device
pointers are valid inside the library.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_int, c_int32, c_int64, c_void_p

import torch  # noqa: F401  (loads the HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnyx.so")

NYX_OK, NYX_ERR_INVALID, NYX_ERR_OOM, NYX_ERR_DEVICE, NYX_ERR_CAPACITY, NYX_ERR_UNSUPPORTED, NYX_ERR_INTERNAL = range(7)
NYX_FP32, NYX_FP64 = 0, 1


class NyxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"nyx status {status}: {message}")
        self.status = status


class nyx_offset(ctypes.Structure):
    _fields_ = [("dz", c_int32), ("dy", c_int32), ("dx", c_int32)]


class nyx_image(ctypes.Structure):
    _fields_ = [("intensity", c_void_p), ("labels", c_void_p), ("nz", c_int64), ("ny", c_int64), ("nx", c_int64)]


class nyx_roi_table(ctypes.Structure):
    _fields_ = [("label", c_void_p), ("image", c_void_p), ("n_vox", c_void_p), ("vmin", c_void_p),
                ("vmax", c_void_p), ("bbox", c_void_p), ("capacity", c_int64), ("n_rois_host", POINTER(c_int64))]


class nyx_glcm(ctypes.Structure):
    _fields_ = [("key", c_void_p), ("count", c_void_p), ("capacity", c_int64), ("nnz_host", POINTER(c_int64)),
                ("n_bins", c_int32), ("n_offsets", c_int32), ("symmetric", c_int32), ("n_rois", c_int64)]


class nyx_extract_opts(ctypes.Structure):
    _fields_ = [("n_bins", c_int32), ("offsets_host", POINTER(nyx_offset)), ("n_offsets", c_int32),
                ("symmetric", c_int32), ("precision", c_int), ("autotune", c_int32), ("accum_mode", c_int32),
                ("copies", c_int32), ("workspace_cap_bytes", c_int64), ("aggregate", c_int32)]


_lib = None

# Every symbol include/nyx.h declares.
EXPORTS = ("nyx_create", "nyx_destroy", "nyx_last_error", "nyx_status_string", "nyx_offsets_default",
           "nyx_feature_count", "nyx_feature_name", "nyx_bin_rois", "nyx_glcm_accumulate", "nyx_glcm_features",
           "nyx_extract_batch", "nyx_extract_batch_noalloc", "nyx_plan_create", "nyx_plan_execute", "nyx_plan_execute_per_roi",
           "nyx_plan_check", "nyx_plan_describe", "nyx_plan_destroy", "nyx_plan_profile",
           "nyx_intensity_feature_count", "nyx_intensity_feature_name", "nyx_intensity_features",
           "nyx_neighbourhood_feature_count", "nyx_neighbourhood_feature_name", "nyx_neighbourhood_features")

PHASES = ("reset", "scan", "compact", "zero", "batch", "band", "split", "features")


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    L.nyx_create.argtypes = [POINTER(P), c_int]
    L.nyx_destroy.argtypes = [P]
    L.nyx_destroy.restype = None
    L.nyx_last_error.argtypes = [P]
    L.nyx_last_error.restype = c_char_p
    L.nyx_status_string.argtypes = [c_int]
    L.nyx_status_string.restype = c_char_p
    L.nyx_offsets_default.argtypes = [c_int32, c_int32, POINTER(nyx_offset), POINTER(c_int32)]
    L.nyx_feature_count.restype = c_int32
    L.nyx_feature_name.argtypes = [c_int32]
    L.nyx_feature_name.restype = c_char_p
    L.nyx_bin_rois.argtypes = [P, POINTER(nyx_image), c_int32, c_int32, POINTER(nyx_roi_table), P, P]
    L.nyx_glcm_accumulate.argtypes = [P, POINTER(nyx_image), c_int32, POINTER(nyx_roi_table), P,
                                      POINTER(nyx_offset), c_int32, c_int32, c_int32, POINTER(nyx_glcm), P]
    L.nyx_glcm_features.argtypes = [P, POINTER(nyx_glcm), POINTER(nyx_roi_table), c_int, P, c_int64, P]
    L.nyx_intensity_feature_count.restype = c_int32
    L.nyx_intensity_feature_name.argtypes = [c_int32]
    L.nyx_intensity_feature_name.restype = c_char_p
    L.nyx_intensity_features.argtypes = [P, POINTER(nyx_image), c_int32, c_int32, c_int, POINTER(nyx_roi_table), P,
                                         c_int64, P]
    L.nyx_neighbourhood_feature_count.restype = c_int32
    L.nyx_neighbourhood_feature_name.argtypes = [c_int32]
    L.nyx_neighbourhood_feature_name.restype = c_char_p
    L.nyx_neighbourhood_features.argtypes = [P, POINTER(nyx_image), c_int32, c_int32, c_int32, c_int,
                                             POINTER(nyx_roi_table), P, c_int64, P]
    L.nyx_extract_batch.argtypes = [P, POINTER(nyx_image), c_int32, POINTER(nyx_extract_opts),
                                    POINTER(nyx_roi_table), P, c_int64, P]
    L.nyx_extract_batch_noalloc.argtypes = [P, POINTER(nyx_image), c_int32, POINTER(nyx_extract_opts),
                                            POINTER(nyx_roi_table), P, c_int64, P]
    L.nyx_plan_create.argtypes = [P, POINTER(nyx_image), c_int32, POINTER(nyx_extract_opts), POINTER(P),
                                  POINTER(c_int64)]
    L.nyx_plan_execute.argtypes = [P, POINTER(nyx_roi_table), P, P]
    L.nyx_plan_execute_per_roi.argtypes = [P, POINTER(nyx_roi_table), P, P]
    L.nyx_plan_check.argtypes = [P, P]
    L.nyx_plan_profile.argtypes = [P, P, POINTER(ctypes.c_float), P]
    L.nyx_plan_describe.argtypes = [P]
    L.nyx_plan_describe.restype = c_char_p
    L.nyx_plan_destroy.argtypes = [P]
    L.nyx_plan_destroy.restype = None
    for name in ("nyx_create", "nyx_offsets_default", "nyx_bin_rois", "nyx_intensity_features", "nyx_neighbourhood_features", "nyx_glcm_accumulate", "nyx_glcm_features",
                 "nyx_extract_batch", "nyx_extract_batch_noalloc", "nyx_plan_create", "nyx_plan_execute", "nyx_plan_execute_per_roi",
                 "nyx_plan_check", "nyx_plan_profile"):
        getattr(L, name).restype = c_int
    _lib = L
    return L


# ------------------------------------------------------------------ helpers
def _check(status: int, ctx=None):
    if status != NYX_OK:
        msg = lib().nyx_status_string(status).decode()
        if ctx is not None and ctx.handle:
            detail = lib().nyx_last_error(ctx.handle)
            if detail:
                msg = detail.decode()
        raise NyxError(status, msg)


def _stream(stream):
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_void_p(stream.cuda_stream)
    return c_void_p(int(stream))


def _images(images):
    """images: sequence of (intensity, labels) CUDA tensors of shape (nz, ny, nx)
    or (ny, nx), 2-byte and 4-byte integer dtypes, C-contiguous."""
    arr = (nyx_image * len(images))()
    for k, (I, L) in enumerate(images):
        for t, size in ((I, 2), (L, 4)):
            if not t.is_cuda or not t.is_contiguous() or t.element_size() != size:
                raise ValueError("image tensors must be contiguous CUDA tensors (2-byte intensity, 4-byte labels)")
        shape = tuple(I.shape)
        if tuple(L.shape) != shape:
            raise ValueError("intensity and labels differ in shape")
        if len(shape) == 2:
            shape = (1,) + shape
        if len(shape) != 3:
            raise ValueError("images must be 2D or 3D")
        arr[k] = nyx_image(I.data_ptr(), L.data_ptr(), shape[0], shape[1], shape[2])
    return arr


def _offsets(offsets):
    offs = list(offsets)
    arr = (nyx_offset * max(len(offs), 1))()
    for k, (dz, dy, dx) in enumerate(offs):
        arr[k] = nyx_offset(int(dz), int(dy), int(dx))
    return arr, len(offs)


MODES = {"auto": -1, "dense-list": 0, "hash": 1, "dense-scan": 2, "dense16-scan": 3}
NYX_AGG_PER_OFFSET, NYX_AGG_MERGED = 0, 1


def _opts(n_bins, offsets, precision, autotune=0, workspace_cap=0, mode="auto", copies=0,
          aggregate=NYX_AGG_PER_OFFSET, symmetric=True):
    arr, K = _offsets(offsets)
    o = nyx_extract_opts(int(n_bins), ctypes.cast(arr, POINTER(nyx_offset)), K, 1 if symmetric else 0, int(precision),
                         int(autotune), int(MODES[mode] if isinstance(mode, str) else mode), int(copies),
                         int(workspace_cap), int(aggregate))
    return o, arr


def table_blocks(n_offsets: int, aggregate: int = NYX_AGG_PER_OFFSET) -> int:
    """Blocks of 30 features per table row: one per offset plus their mean, or
    the one block of the merged matrix."""
    return 1 if aggregate == NYX_AGG_MERGED else n_offsets + 1


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


# ------------------------------------------------------------------ objects
class Ctx:
    def __init__(self, handle):
        self.handle = handle
        self._destroy = lib().nyx_destroy   # kept: module globals may be gone at interpreter exit

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None


class RoiTable:
    """Device ROI table (torch tensors); bbox is (n, 6): x0, y0, z0, x1, y1, z1."""

    def __init__(self, capacity: int, device):
        c = max(int(capacity), 1)
        self.label = torch.zeros(c, dtype=torch.int32, device=device)
        self.image = torch.zeros(c, dtype=torch.int32, device=device)
        self.n_vox = torch.zeros(c, dtype=torch.int64, device=device)
        self.vmin = torch.zeros(c, dtype=torch.int16, device=device)
        self.vmax = torch.zeros(c, dtype=torch.int16, device=device)
        self.bbox = torch.zeros((c, 6), dtype=torch.int32, device=device)
        self.capacity = int(capacity)
        self.n = c_int64(0)

    def struct(self) -> nyx_roi_table:
        return nyx_roi_table(self.label.data_ptr(), self.image.data_ptr(), self.n_vox.data_ptr(),
                             self.vmin.data_ptr(), self.vmax.data_ptr(), self.bbox.data_ptr(),
                             self.capacity, ctypes.pointer(self.n))

    @property
    def n_rois(self) -> int:
        return int(self.n.value)


class Glcm:
    """Sorted COO of counts: keys roi<<38 | dir<<32 | (i-1)<<16 | (j-1); the upper
    triangle of symmetric matrices, or every cell of ordered (non-symmetric) ones."""

    def __init__(self, keys, counts, nnz, n_bins, n_offsets, n_rois, symmetric=True):
        self.keys, self.counts = keys, counts
        self.nnz, self.n_bins, self.n_offsets, self.n_rois = nnz, n_bins, n_offsets, n_rois
        self.symmetric = bool(symmetric)

    def struct(self, nnz_box: c_int64) -> nyx_glcm:
        return nyx_glcm(self.keys.data_ptr() if self.nnz else None, self.counts.data_ptr() if self.nnz else None,
                        self.nnz, ctypes.pointer(nnz_box), self.n_bins, self.n_offsets, 1 if self.symmetric else 0,
                        self.n_rois)


class Plan:
    def __init__(self, ctx, handle, n_rois, keep):
        self.ctx, self.handle, self.n_rois, self._keep = ctx, handle, n_rois, keep
        self._destroy = lib().nyx_plan_destroy

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None


# ------------------------------------------------------------------ API
def nyx_create(device: int = 0) -> Ctx:
    h = c_void_p()
    _check(lib().nyx_create(byref(h), int(device)))
    return Ctx(h)


def nyx_status_string(status: int) -> str:
    return lib().nyx_status_string(int(status)).decode()


def nyx_offsets_default(dims: int, distance: int = 1):
    arr = (nyx_offset * 13)()
    n = c_int32(0)
    _check(lib().nyx_offsets_default(int(dims), int(distance), arr, byref(n)))
    return [(arr[k].dz, arr[k].dy, arr[k].dx) for k in range(n.value)]


def nyx_feature_count() -> int:
    return int(lib().nyx_feature_count())


def nyx_feature_name(f: int):
    s = lib().nyx_feature_name(int(f))
    return None if s is None else s.decode()


def nyx_bin_rois(ctx: Ctx, images, n_bins: int, want_bins: bool = False, stream=None, capacity=None):
    """ROI table (and optionally the per-voxel level image, flattened over the images)."""
    imgs = _images(images)
    dev = _dev()
    if capacity is None:
        probe = RoiTable(0, dev)
        st = probe.struct()
        status = lib().nyx_bin_rois(ctx.handle, imgs, len(images), int(n_bins), byref(st), None, _stream(stream))
        if status not in (NYX_OK, NYX_ERR_CAPACITY):
            _check(status, ctx)
        capacity = probe.n_rois
    rois = RoiTable(capacity, dev)
    bins = None
    if want_bins:
        total = sum(int(I.numel()) for I, _ in images)
        bins = torch.zeros(max(total, 1), dtype=torch.int16, device=dev)
    st = rois.struct()
    _check(lib().nyx_bin_rois(ctx.handle, imgs, len(images), int(n_bins), byref(st),
                              bins.data_ptr() if bins is not None else None, _stream(stream)), ctx)
    return rois, bins


def nyx_glcm_accumulate(ctx: Ctx, images, rois: RoiTable, n_bins: int, offsets, bins=None, stream=None,
                        symmetric: bool = True) -> Glcm:
    imgs = _images(images)
    offs, K = _offsets(offsets)
    dev = _dev()
    nnz = c_int64(0)
    out = nyx_glcm(None, None, 0, ctypes.pointer(nnz), 0, 0, 1, 0)
    rs = rois.struct() if rois is not None else None
    bptr = bins.data_ptr() if bins is not None else None
    status = lib().nyx_glcm_accumulate(ctx.handle, imgs, len(images), byref(rs) if rs is not None else None, bptr,
                                       offs, K, 1 if symmetric else 0, int(n_bins), byref(out), _stream(stream))
    if status not in (NYX_OK, NYX_ERR_CAPACITY):
        _check(status, ctx)
    n = int(nnz.value)
    keys = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    counts = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)
    out = nyx_glcm(keys.data_ptr(), counts.data_ptr(), n, ctypes.pointer(nnz), 0, 0, 1, 0)
    _check(lib().nyx_glcm_accumulate(ctx.handle, imgs, len(images), byref(rs) if rs is not None else None, bptr,
                                     offs, K, 1 if symmetric else 0, int(n_bins), byref(out), _stream(stream)), ctx)
    return Glcm(keys[:n], counts[:n], n, int(n_bins), K, int(out.n_rois), symmetric)


def nyx_glcm_features(ctx: Ctx, glcm: Glcm, precision: int = NYX_FP32, stream=None, capacity=None,
                      rois: RoiTable | None = None):
    dtype = torch.float64 if precision == NYX_FP64 else torch.float32
    rows = glcm.n_rois if capacity is None else int(capacity)
    table = torch.zeros((max(rows, 1), glcm.n_offsets + 1, 30), dtype=dtype, device=_dev())
    nnz = c_int64(glcm.nnz)
    g = glcm.struct(nnz)
    rs = rois.struct() if rois is not None else None
    _check(lib().nyx_glcm_features(ctx.handle, byref(g), byref(rs) if rs is not None else None, int(precision),
                                   table.data_ptr(), rows, _stream(stream)), ctx)
    return table[:glcm.n_rois]


def nyx_intensity_feature_count() -> int:
    return int(lib().nyx_intensity_feature_count())


def nyx_intensity_feature_name(f: int):
    s = lib().nyx_intensity_feature_name(int(f))
    return None if s is None else s.decode()


def nyx_intensity_features(ctx: Ctx, images, n_bins: int, precision: int = NYX_FP32, stream=None, capacity=None):
    """First-order intensity features: returns (RoiTable, table (n, 37))."""
    imgs = _images(images)
    dev = _dev()
    if capacity is None:
        probe = RoiTable(0, dev)
        st = probe.struct()
        status = lib().nyx_intensity_features(ctx.handle, imgs, len(images), int(n_bins), int(precision), byref(st),
                                              None, 0, _stream(stream))
        if status not in (NYX_OK, NYX_ERR_CAPACITY):
            _check(status, ctx)
        capacity = probe.n_rois
    rois = RoiTable(capacity, dev)
    dtype = torch.float64 if precision == NYX_FP64 else torch.float32
    table = torch.full((max(capacity, 1), nyx_intensity_feature_count()), float("nan"), dtype=dtype, device=dev)
    st = rois.struct()
    _check(lib().nyx_intensity_features(ctx.handle, imgs, len(images), int(n_bins), int(precision), byref(st),
                                        table.data_ptr(), int(capacity), _stream(stream)), ctx)
    return rois, table[:rois.n_rois]


def nyx_neighbourhood_feature_count() -> int:
    return int(lib().nyx_neighbourhood_feature_count())


def nyx_neighbourhood_feature_name(f: int):
    s = lib().nyx_neighbourhood_feature_name(int(f))
    return None if s is None else s.decode()


def nyx_neighbourhood_features(ctx: Ctx, images, n_bins: int, alpha: int = 0, precision: int = NYX_FP32,
                               stream=None, capacity=None):
    """NGLDM, NGTDM and GLDM features: returns (RoiTable, table (n, 37))."""
    imgs = _images(images)
    dev = _dev()
    if capacity is None:
        probe = RoiTable(0, dev)
        st = probe.struct()
        status = lib().nyx_neighbourhood_features(ctx.handle, imgs, len(images), int(n_bins), int(alpha),
                                                  int(precision), byref(st), None, 0, _stream(stream))
        if status not in (NYX_OK, NYX_ERR_CAPACITY):
            _check(status, ctx)
        capacity = probe.n_rois
    rois = RoiTable(capacity, dev)
    dtype = torch.float64 if precision == NYX_FP64 else torch.float32
    table = torch.full((max(capacity, 1), nyx_neighbourhood_feature_count()), float("nan"), dtype=dtype, device=dev)
    st = rois.struct()
    _check(lib().nyx_neighbourhood_features(ctx.handle, imgs, len(images), int(n_bins), int(alpha), int(precision),
                                            byref(st), table.data_ptr(), int(capacity), _stream(stream)), ctx)
    return rois, table[:rois.n_rois]


def nyx_extract_batch(ctx: Ctx, images, n_bins: int, offsets, precision: int = NYX_FP32, stream=None,
                      capacity=None, mode="auto", copies: int = 0, aggregate: int = NYX_AGG_PER_OFFSET,
                      symmetric: bool = True):
    """One-shot extraction: returns (RoiTable, table (n, blocks, 30)), blocks = K + 1, or 1 when the
    offsets' matrices are merged."""
    imgs = _images(images)
    opts, keep = _opts(n_bins, offsets, precision, mode=mode, copies=copies, aggregate=aggregate, symmetric=symmetric)
    dev = _dev()
    if capacity is None:
        probe = RoiTable(0, dev)
        st = probe.struct()
        status = lib().nyx_extract_batch(ctx.handle, imgs, len(images), byref(opts), byref(st), None, 0,
                                         _stream(stream))
        if status not in (NYX_OK, NYX_ERR_CAPACITY):
            _check(status, ctx)
        capacity = probe.n_rois
    rois = RoiTable(capacity, dev)
    dtype = torch.float64 if precision == NYX_FP64 else torch.float32
    table = torch.zeros((max(capacity, 1), table_blocks(opts.n_offsets, aggregate), 30), dtype=dtype, device=dev)
    st = rois.struct()
    _check(lib().nyx_extract_batch(ctx.handle, imgs, len(images), byref(opts), byref(st), table.data_ptr(),
                                   int(capacity), _stream(stream)), ctx)
    return rois, table[:rois.n_rois]


def nyx_extract_batch_noalloc(ctx: Ctx, images, n_bins: int, offsets, rois: RoiTable, table,
                              precision: int = NYX_FP32, stream=None, mode="auto", copies: int = 0,
                              aggregate: int = NYX_AGG_PER_OFFSET, symmetric: bool = True) -> int:
    """The pass of nyx_extract_batch into caller-allocated `rois` and `table`
    without any device allocation in the library; returns the ROI count."""
    imgs = _images(images)
    opts, keep = _opts(n_bins, offsets, precision, mode=mode, copies=copies, aggregate=aggregate, symmetric=symmetric)
    st = rois.struct()
    cap = int(table.shape[0]) if table is not None else 0
    _check(lib().nyx_extract_batch_noalloc(ctx.handle, imgs, len(images), byref(opts), byref(st),
                                           table.data_ptr() if table is not None else None, cap,
                                           _stream(stream)), ctx)
    return rois.n_rois


def nyx_plan_create(ctx: Ctx, images, n_bins: int, offsets, precision: int = NYX_FP32, autotune: bool = False,
                    workspace_cap: int = 0, mode="auto", copies: int = 0,
                    aggregate: int = NYX_AGG_PER_OFFSET, symmetric: bool = True) -> Plan:
    """mode: accumulation mode name (MODES) or -1/auto; copies: privatised LDS triangle copies per
    direction (0 automatic, else 1, 2 or 4)."""
    imgs = _images(images)
    opts, keep = _opts(n_bins, offsets, precision, int(autotune), workspace_cap, mode, copies, aggregate, symmetric)
    h = c_void_p()
    n = c_int64(0)
    _check(lib().nyx_plan_create(ctx.handle, imgs, len(images), byref(opts), byref(h), byref(n)), ctx)
    return Plan(ctx, h, int(n.value), (images, keep))


def nyx_plan_execute(plan: Plan, table, rois: RoiTable | None = None, stream=None):
    st = rois.struct() if rois is not None else None
    _check(lib().nyx_plan_execute(plan.handle, byref(st) if st is not None else None, table.data_ptr(),
                                  _stream(stream)), plan.ctx)


def nyx_plan_execute_per_roi(plan: Plan, table, rois: RoiTable | None = None, stream=None):
    st = rois.struct() if rois is not None else None
    _check(lib().nyx_plan_execute_per_roi(plan.handle, byref(st) if st is not None else None, table.data_ptr(),
                                          _stream(stream)), plan.ctx)


def nyx_plan_check(plan: Plan, stream=None):
    _check(lib().nyx_plan_check(plan.handle, _stream(stream)), plan.ctx)


def nyx_plan_profile(plan: Plan, table, stream=None) -> dict:
    """One eager step with HIP events between phases: {phase: milliseconds}."""
    ms = (ctypes.c_float * len(PHASES))()
    _check(lib().nyx_plan_profile(plan.handle, table.data_ptr(), ms, _stream(stream)), plan.ctx)
    return dict(zip(PHASES, [float(v) for v in ms]))


def nyx_plan_describe(plan: Plan) -> str:
    return lib().nyx_plan_describe(plan.handle).decode()


def nyx_plan_destroy(plan: Plan):
    if getattr(plan, "handle", None):
        plan._destroy(plan.handle)
        plan.handle = None


def new_table(plan: Plan, n_offsets: int, precision: int = NYX_FP32, aggregate: int = NYX_AGG_PER_OFFSET):
    dtype = torch.float64 if precision == NYX_FP64 else torch.float32
    return torch.zeros((max(plan.n_rois, 1), table_blocks(n_offsets, aggregate), 30), dtype=dtype, device=_dev())
