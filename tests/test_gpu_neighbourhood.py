"""GPU parity of the neighbourhood texture features (nyx_neighbourhood_features:
NGLDM, NGTDM, GLDM) against the FP64 oracle (oracle/neighbourhood.py),
through the C ABI.

Error of a value: |gpu - oracle| / max(|oracle|, M) with M = 1 bit for the
two entropies (DCENT, DE) and 0 elsewhere (plain relative error); NaN must
match NaN.  Bars: 1e-12 for the FP64 table, 1e-5 for the FP32 table."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from gpu_util import device_images

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-12}


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


@pytest.fixture(scope="module")
def workloads(synth_mod):
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = synth_mod.make(name)
        return cache[name]
    return get


def _roi_oracle(nb, I, L, lab, bbox, n_bins, alpha):
    """Oracle features of one ROI on its bounding box plus a one-voxel margin
    (neighbours outside the box are outside the ROI, so nothing changes);
    a 3D image stays 3D."""
    x0, y0, z0, x1, y1, z1 = (int(v) for v in bbox)
    nz, ny, nx = I.shape
    a = (max(z0 - 1, 0), max(y0 - 1, 0), max(x0 - 1, 0))
    b = (min(z1 + 2, nz), min(y1 + 2, ny), min(x1 + 2, nx))
    Ib = I[a[0]:b[0], a[1]:b[1], a[2]:b[2]]
    Mb = L[a[0]:b[0], a[1]:b[1], a[2]:b[2]] == lab
    if nz > 1 and Ib.shape[0] == 1:
        Ib = np.concatenate([Ib, np.zeros_like(Ib)])
        Mb = np.concatenate([Mb, np.zeros_like(Mb)])
    return nb.features(Ib, Mb, n_bins, alpha)


def _rois_of(I, L):
    labs = np.unique(L[L != 0])
    out = []
    for lab in labs:
        zz, yy, xx = np.nonzero(L == lab)
        out.append((int(lab), (xx.min(), yy.min(), zz.min(), xx.max(), yy.max(), zz.max())))
    return out


def _check(nb, got, want, prec, tag):
    got = np.asarray(got, np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    assert np.array_equal(nan_g, nan_w), (tag, np.argwhere(nan_g != nan_w)[:5])
    M = np.zeros(want.shape[1])
    M[[nb.NAMES.index("NGLDM_DCENT"), nb.NAMES.index("GLDM_DE")]] = 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        err = np.abs(got - want) / np.maximum(np.abs(want), M)
    err = np.where(nan_g | (got == want), 0.0, err)
    i = np.unravel_index(np.argmax(err), err.shape)
    say(f"  {tag}: {len(want)} ROIs, max error {err[i]:.3e} ({nb.NAMES[i[1]]} of row {i[0]})")
    assert err[i] <= TOL[prec], (tag, nb.NAMES[i[1]], i, got[i], want[i])


def _run(nyx, images, ctx, n_bins, alpha, prec):
    import torch
    rois, table = nyx.nyx_neighbourhood_features(ctx, images, n_bins, alpha, prec)
    torch.cuda.synchronize()
    return rois, table.cpu().numpy()


@pytest.mark.parametrize("name", ["c1_tiny", "c2_small", "c3_small", "c4_small", "c5_small"])
@pytest.mark.parametrize("prec", [1, 0])
def test_workload_shapes(env, workloads, name, prec):
    from oracle import neighbourhood as nb
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} neighbourhood features prec={prec}")
    rois, got = _run(nyx, device_images(w, dev), ctx, w.n_bins, 0, prec)
    want = [_roi_oracle(nb, w.intensity[k], w.labels[k], lab, bb, w.n_bins, 0)
            for k in range(w.n_images) for lab, bb in _rois_of(w.intensity[k], w.labels[k])]
    assert rois.n_rois == len(want)
    _check(nb, got, np.array(want), prec, f"{name} prec={prec}")


def _edge_images():
    rng = np.random.default_rng(8)
    L = np.zeros((1, 18, 30), np.uint32)
    I = rng.integers(0, 4000, L.shape).astype(np.uint16)
    L[0, 1, 1] = 1                                   # one voxel: no neighbour
    L[0, 3, 3] = 2; L[0, 5, 5] = 2                   # two isolated voxels
    L[0, 7, 1:20] = 3                                # line
    L[0, 9:13, 2:7] = 4; I[0, 9:13, 2:7] = 500       # constant block: flat texture
    L[0, 0, :] = 5; L[0, :, 29] = 5                  # two borders
    L[0, 14:18, 10:28] = 6                           # block on the border
    L[0, 9:13, 10:14] = 7                            # checkerboard of two values
    I[0, 9:13, 10:14] = (np.indices((4, 4)).sum(axis=0) % 2) * 3000 + 10
    V = np.zeros((5, 6, 7), np.uint32)
    IV = rng.integers(0, 60000, V.shape).astype(np.uint16)
    V[1:4, 1:5, 1:6] = 1
    V[0, 0, 0] = 2
    V[:, 5, 6] = 3                                   # a column through every plane on the border
    return [(I, L), (IV, V)]


@pytest.mark.parametrize("n_bins,alpha", [(2, 0), (8, 0), (8, 1), (100, 0), (100, 7)])
@pytest.mark.parametrize("prec", [1, 0])
def test_edge_cases(env, n_bins, alpha, prec):
    import torch
    from oracle import neighbourhood as nb
    nyx, ctx, dev = env
    say(f"case neighbourhood edge images n_bins={n_bins} alpha={alpha} prec={prec}")
    for I, L in _edge_images():
        imgs = [(torch.from_numpy(I.view(np.int16)).to(dev), torch.from_numpy(L.view(np.int32)).to(dev))]
        rois, got = _run(nyx, imgs, ctx, n_bins, alpha, prec)
        labs = _rois_of(I, L)
        want = np.array([nb.features(I, L == lab, n_bins, alpha) for lab, _ in labs])
        assert rois.n_rois == len(labs)
        _check(nb, got, want, prec, f"edge {I.shape} n_bins={n_bins} alpha={alpha}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,n_sample", [("c3_batch", 150), ("c4_3d", 12), ("c5_stress", 60)])
def test_full_size_sampled(env, workloads, name, n_sample):
    from oracle import neighbourhood as nb
    nyx, ctx, dev = env
    w = workloads(name)
    say(f"case {name} full size neighbourhood features, sampled ROIs")
    rois, got = _run(nyx, device_images(w, dev), ctx, w.n_bins, 0, 0)
    n = rois.n_rois
    lab = rois.label.cpu().numpy()[:n].astype(np.int64) & 0xFFFFFFFF
    img = rois.image.cpu().numpy()[:n]
    bbox = rois.bbox.cpu().numpy()[:n]
    nvox = rois.n_vox.cpu().numpy()[:n]
    rng = np.random.default_rng(5)
    small = np.nonzero(nvox <= 50000)[0]           # the oracle loops over voxels in Python
    sample = sorted(set(rng.choice(small, size=min(n_sample, small.size), replace=False).tolist()) |
                    {int(small[np.argmax(nvox[small])])})
    want = [_roi_oracle(nb, w.intensity[img[r]], w.labels[img[r]], int(lab[r]), bbox[r], w.n_bins, 0)
            for r in sample]
    _check(nb, got[sample], np.array(want), 0, f"{name} sampled")
    assert np.all(np.isfinite(got[nvox >= 2][:, :18]))
