"""ctypes binding of libnyx_micro.so: the machine-ceiling kernels (copy and
read bandwidth, LDS atomic rate) that the GLCM kernels' rooflines are read
against.  Measurement only; not part of the feature path."""
from __future__ import annotations

import ctypes
import os
from ctypes import c_int, c_uint32, c_uint64, c_void_p

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnyx_micro.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime for torch and the library)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.nyx_micro_copy.argtypes = [c_void_p, c_void_p, c_uint64, c_void_p]
        L.nyx_micro_read.argtypes = [c_void_p, c_uint64, c_void_p, c_void_p]
        L.nyx_micro_lds_atomic.argtypes = [c_uint32, c_uint32, c_void_p, c_void_p]
        for f in (L.nyx_micro_copy, L.nyx_micro_read, L.nyx_micro_lds_atomic):
            f.restype = c_int
        _lib = L
    return _lib


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _timed(fn, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """Device copy of nbytes: (read + write bytes) / time, in GB/s."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(7)
    dst = torch.empty_like(src)
    L = lib()

    def run():
        if L.nyx_micro_copy(c_void_p(src.data_ptr()), c_void_p(dst.data_ptr()), nbytes, _stream()):
            raise RuntimeError("nyx_micro_copy failed")
    t = _timed(run, reps)
    assert torch.equal(src[:4096], dst[:4096])
    return {"bytes": nbytes, "seconds": t, "GBps": 2.0 * nbytes / t / 1e9}


def read_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> dict:
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(3)
    sink = torch.zeros(256 * 64, dtype=torch.int32, device="cuda")
    L = lib()

    def run():
        if L.nyx_micro_read(c_void_p(src.data_ptr()), nbytes, c_void_p(sink.data_ptr()), _stream()):
            raise RuntimeError("nyx_micro_read failed")
    t = _timed(run, reps)
    return {"bytes": nbytes, "seconds": t, "GBps": nbytes / t / 1e9}


def lds_atomic_rate(blocks: int = 256 * 8, iters: int = 4096, reps: int = 5) -> dict:
    """Chip-wide conflict-free ds_add_u32 rate (lane-atomics per second)."""
    import torch
    out = torch.zeros(blocks, dtype=torch.int32, device="cuda")
    L = lib()

    def run():
        if L.nyx_micro_lds_atomic(blocks, iters, c_void_p(out.data_ptr()), _stream()):
            raise RuntimeError("nyx_micro_lds_atomic failed")
    t = _timed(run, reps)
    n = blocks * 256 * 4 * iters
    assert int(out[0].item()) == 4 * iters * 256
    return {"lane_atomics": n, "seconds": t, "per_second": n / t}
