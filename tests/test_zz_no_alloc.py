"""The no-allocation entry point against nyx_extract_batch.

nyx_extract_batch_noalloc carves every scratch buffer from one library-owned
array per GPU; its results must equal nyx_extract_batch's (same untimed
configuration, same kernels) on consecutive calls, the second smaller than
the first, so a stale ROI, counter or matrix left in the array by the first
call would show.  A batch whose scratch exceeds the array is refused with
NYX_ERR_CAPACITY before any device work on it.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from gpu_util import device_images

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2603_12016_amd import nyx
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    return nyx, nyx.nyx_create(0), dev


def _compare(nyx, ctx, dev, w, prec, mode="auto"):
    """Both entry points on the same images.  The scan accumulation modes visit
    the cells in a fixed order, so their tables must be bit-identical; the
    list / hash modes follow atomic timing, so theirs are compared to the
    precision contract (1e-5 FP32, 1e-12 FP64) relative to each feature's
    magnitude over the table."""
    import torch
    imgs = device_images(w, dev)
    offs = nyx.nyx_offsets_default(w.dims, 1)
    rois_ref, table_ref = nyx.nyx_extract_batch(ctx, imgs, w.n_bins, offs, prec, mode=mode)
    n = rois_ref.n_rois
    rois = nyx.RoiTable(n, dev)
    dtype = torch.float64 if prec == nyx.NYX_FP64 else torch.float32
    # filled with NaN / garbage so rows the call does not write would show
    table = torch.full((max(n, 1), len(offs) + 1, 30), float("nan"), dtype=dtype, device=dev)
    rois.label.fill_(-1)
    got_n = nyx.nyx_extract_batch_noalloc(ctx, imgs, w.n_bins, offs, rois, table, prec, mode=mode)
    torch.cuda.synchronize()
    assert got_n == n
    for name in ("label", "image", "n_vox", "vmin", "vmax", "bbox"):
        a = getattr(rois, name)[:n].cpu().numpy()
        b = getattr(rois_ref, name)[:n].cpu().numpy()
        assert np.array_equal(a, b), name
    got = table[:n].cpu().numpy().astype(np.float64)
    want = table_ref.cpu().numpy().astype(np.float64)
    nan = np.isnan(got) & np.isnan(want)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    if mode in ("dense-scan", "dense16-scan"):
        same = (got == want) | nan
        assert same.all(), (np.argwhere(~same)[:5], got[~same][:5], want[~same][:5])
    else:
        tol = 1e-12 if prec == nyx.NYX_FP64 else 1e-5
        mag = np.nanmax(np.abs(want).reshape(-1, 30), axis=0) if n else np.ones(30)
        err = np.where(nan, 0.0, np.abs(got - want) / np.maximum(np.abs(want), np.maximum(mag, 1e-300) * 1e-3))
        assert float(err.max(initial=0.0)) <= tol, float(err.max())
    return n


def test_noalloc_matches_extract_batch_twice(env):
    import synth
    nyx, ctx, dev = env
    first = synth.make("c3_small")
    second = synth.make("c2_small")
    assert first.labels.size > second.labels.size
    say("noalloc: c3_small (3 images) then c2_small (1 smaller image), FP32, automatic mode")
    n1 = _compare(nyx, ctx, dev, first, nyx.NYX_FP32)
    n2 = _compare(nyx, ctx, dev, second, nyx.NYX_FP32)
    say(f"  {n1} then {n2} ROIs match nyx_extract_batch")
    say("noalloc: the same two batches, 16-bit scan mode (bit-identical)")
    _compare(nyx, ctx, dev, first, nyx.NYX_FP32, mode="dense16-scan")
    _compare(nyx, ctx, dev, second, nyx.NYX_FP32, mode="dense16-scan")
    say("noalloc: c1_tiny, FP64")
    _compare(nyx, ctx, dev, synth.make("c1_tiny"), nyx.NYX_FP64)
    # label values near 2^32: discovery takes the per-image label dictionary,
    # whose arrays come from the same scratch array
    from test_gpu_labels import relabel
    say("noalloc: c3_small with label values near 2^32 (label dictionary)")
    _compare(nyx, ctx, dev, relabel(first, seed=5), nyx.NYX_FP32, mode="dense16-scan")


def test_noalloc_rejects_batches_beyond_its_scratch(env):
    import torch
    nyx, ctx, dev = env
    # 2^23 distinct labels (every voxel of a 4096 x 2048 image its own ROI):
    # the per-label statistics alone need 10 x 4 B x 2^23 = 320 MiB, more
    # than the 256 MiB array
    I = torch.zeros((4096, 2048), dtype=torch.int16, device=dev)
    L = torch.arange(1, 4096 * 2048 + 1, dtype=torch.int32, device=dev).reshape(4096, 2048)
    rois = nyx.RoiTable(2, dev)
    table = torch.zeros((2, 5, 30), dtype=torch.float32, device=dev)
    say("noalloc: 2^23 labels (scratch too small)")
    with pytest.raises(nyx.NyxError) as e:
        nyx.nyx_extract_batch_noalloc(ctx, [(I, L)], 8, nyx.nyx_offsets_default(2, 1), rois, table)
    assert e.value.status == nyx.NYX_ERR_CAPACITY
    assert "no-allocation scratch" in str(e.value)
    # the entry point still works afterwards
    L2 = torch.ones((64, 64), dtype=torch.int32, device=dev)
    I2 = torch.arange(64 * 64, dtype=torch.int32, device=dev).reshape(64, 64).remainder(4096).to(torch.int16)
    n = nyx.nyx_extract_batch_noalloc(ctx, [(I2, L2)], 8, nyx.nyx_offsets_default(2, 1), rois, table)
    torch.cuda.synchronize()
    assert n == 1
    assert np.isfinite(table[0].cpu().numpy()).all()
