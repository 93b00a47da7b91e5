"""Checks that need no GPU: the library loads and exports every symbol
include/nyx.h declares; static tables agree with the oracle; device-free
calls; host copies of the kernels' index rules (tiling, work tickets, the
staged ring) against brute force; the benchmark's one-GPU contract."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "nyx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nyx_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def nyx():
    from paper_2603_12016_amd import nyx as m
    m.lib()
    return m


def test_header_declares_expected_entry_points():
    names = _header_functions()
    for required in ("nyx_bin_rois", "nyx_glcm_accumulate", "nyx_glcm_features", "nyx_extract_batch"):
        assert required in names


def test_library_exports_every_declared_symbol(nyx):
    lib = nyx.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name
    assert set(_header_functions()) == set(nyx.EXPORTS)


def test_feature_names_match_oracle(nyx, oracle_mod):
    assert nyx.nyx_feature_count() == 30
    assert [nyx.nyx_feature_name(f) for f in range(30)] == oracle_mod.feature_names()
    assert nyx.nyx_feature_name(30) is None and nyx.nyx_feature_name(-1) is None


def test_intensity_feature_names_match_oracle(nyx):
    from oracle import first_order as fo
    assert nyx.nyx_intensity_feature_count() == fo.NFO
    assert tuple(nyx.nyx_intensity_feature_name(f) for f in range(fo.NFO)) == fo.NAMES
    assert nyx.nyx_intensity_feature_name(fo.NFO) is None and nyx.nyx_intensity_feature_name(-1) is None


def test_neighbourhood_feature_names_match_oracle(nyx):
    from oracle import neighbourhood as nb
    assert nyx.nyx_neighbourhood_feature_count() == nb.NNF
    assert tuple(nyx.nyx_neighbourhood_feature_name(f) for f in range(nb.NNF)) == nb.NAMES
    assert nyx.nyx_neighbourhood_feature_name(nb.NNF) is None


@pytest.mark.parametrize("dims,dist", [(2, 1), (2, 3), (3, 1), (3, 2)])
def test_default_offsets_match_oracle(nyx, oracle_mod, dims, dist):
    assert np.array_equal(np.array(nyx.nyx_offsets_default(dims, dist), np.int32),
                          oracle_mod.default_offsets(dims, dist))


def test_default_offsets_cover_neighbourhood_once(nyx):
    # the 13 3D offsets and their negatives are exactly the 26 neighbours
    offs = nyx.nyx_offsets_default(3, 1)
    both = set(offs) | {(-a, -b, -c) for a, b, c in offs}
    assert len(both) == 26 and (0, 0, 0) not in both


def test_offsets_default_rejects_bad_arguments(nyx):
    with pytest.raises(nyx.NyxError) as e:
        nyx.nyx_offsets_default(4, 1)
    assert e.value.status == nyx.NYX_ERR_INVALID
    with pytest.raises(nyx.NyxError):
        nyx.nyx_offsets_default(2, 0)


def test_status_strings(nyx):
    assert nyx.nyx_status_string(0) == "ok"
    assert nyx.nyx_status_string(4) == "capacity too small"
    assert "unknown" in nyx.nyx_status_string(99)


def test_create_without_device_reports_device_error(nyx):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(nyx.NyxError) as e:
        nyx.nyx_create(0)
    assert e.value.status == nyx.NYX_ERR_DEVICE


@pytest.fixture(scope="module")
def rules():
    """The index rules of nyx_types.h compiled for the host by hipcc (the same
    inline functions the kernels instantiate), loaded with ctypes."""
    import ctypes
    import subprocess
    src = os.path.join(ROOT, "tests", "index_rules.hip")
    lib = os.path.join(ROOT, "tests", "libindex_rules.so")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
                           "-I" + os.path.join(ROOT, "paper_2603_12016_amd", "csrc"), "-o", tmp, src])
    os.replace(tmp, lib)
    L = ctypes.CDLL(lib)
    u32, P = ctypes.c_uint32, ctypes.c_void_p
    L.rules_tiles_for.argtypes = [u32, u32, u32, u32, u32, P, P]
    L.rules_tile_bounds.argtypes = [u32, u32, u32, u32, u32, P]
    L.rules_size_class.argtypes = [u32]
    L.rules_size_class.restype = u32
    L.rules_ticket_chunk.argtypes = [ctypes.c_int]
    L.rules_ticket_chunk.restype = u32
    L.rules_ticket_offsets.argtypes = [P, P]
    L.rules_ticket_offsets.restype = u32
    L.rules_ticket_range.argtypes = [u32, P, P, P, P, P]
    L.rules_label_entry.argtypes = [P, u32, u32, u32]
    L.rules_label_entry.restype = u32
    L.rules_fbn_levels.argtypes = [P, u32, u32, u32, u32, P]
    return L


def test_fbn_level_rule_exact(rules):
    # the compiled level rule (double reciprocal rounded up, no correction
    # step) against exact integer division, over every value of each range,
    # for ranges where the quotient lands exactly on integers often (powers
    # of two, multiples of ng) and random ones, and bin counts up to 8191
    rng = np.random.default_rng(2)
    cases = [(0, 0, 8), (5, 5, 64), (0, 1, 2), (0, 65535, 8191), (0, 65535, 64), (100, 164, 64), (7, 7 + 1024, 1024),
             (0, 4096, 8), (3, 3 + 63, 64), (1, 1 + 255, 256), (0, 30, 10), (0, 99, 100), (12, 12 + 8191, 8191)]
    cases += [(int(a), int(a + d), int(g)) for a, d, g in zip(rng.integers(0, 30000, 40), rng.integers(1, 35535, 40),
                                                            rng.integers(2, 8192, 40))]
    for vmin, vmax, ng in cases:
        I = np.arange(vmin, vmax + 1, dtype=np.uint32)
        out = np.zeros(I.size, np.uint32)
        rules.rules_fbn_levels(I.ctypes.data, I.size, vmin, vmax, ng, out.ctypes.data)
        D = vmax - vmin
        want = np.ones(I.size, np.int64) if D == 0 else \
            np.minimum(1 + (ng * (I.astype(np.int64) - vmin)) // D, ng)
        assert np.array_equal(out, want), (vmin, vmax, ng)


def test_label_entry_rule(rules):
    # the compiled label-to-entry rule: direct indexing up to max_label, else
    # 1 + rank in the sorted dictionary, 0 for background and absent labels
    for l in (0, 1, 7, 8, 9, 1000):
        assert rules.rules_label_entry(None, 0, 8, l) == (l if 0 < l <= 8 else 0)
    rng = np.random.default_rng(5)
    for n in (0, 1, 2, 3, 17, 256, 1001):
        d = np.unique(rng.integers(1, 2**32, size=n, dtype=np.uint64)).astype(np.uint32)
        d = np.concatenate([d, np.array([2**32 - 1], np.uint32)]) if n == 2 else d
        d = np.ascontiguousarray(np.unique(d))
        probes = np.concatenate([d, d - 1, d + 1, [0, 1, 2**32 - 1, 2**31]]).astype(np.uint32)
        pos = {int(v): k + 1 for k, v in enumerate(d)}
        for l in probes:
            want = pos.get(int(l), 0) if l != 0 else 0
            assert rules.rules_label_entry(d.ctypes.data if d.size else None, d.size, d.size, int(l)) == want


def test_split_rule_covers_rows_and_columns(rules):
    # the compiled tiling rule: the tiles of a split ROI partition its bbox
    from itertools import product
    rb, cb = np.zeros(1, np.uint32), np.zeros(1, np.uint32)
    b4 = np.zeros(4, np.uint32)
    for rows, width, n, tile in product([1, 3, 17, 100], [1, 5, 64, 300], [10, 1000, 30000], [7, 64, 1024]):
        rules.rules_tiles_for(n, rows, width, tile, tile, rb.ctypes.data, cb.ctypes.data)
        nt, tc = int(rb[0] * cb[0]), int(cb[0])
        assert 1 <= rb[0] <= rows and 1 <= cb[0] <= width
        if n > tile:
            assert nt >= min((n + tile - 1) // tile, rows) or cb[0] == width
        cover = np.zeros((rows, width), int)
        for t in range(nt):
            rules.rules_tile_bounds(rows, width, nt, tc, t, b4.ctypes.data)
            ra, rb_, ca, cb_ = (int(v) for v in b4)
            assert 0 <= ra <= rb_ <= rows and 0 <= ca <= cb_ <= width
            cover[ra:rb_, ca:cb_] += 1
        assert np.all(cover == 1), (rows, width, n, tile)


def test_size_class_is_floor_log2(rules):
    for v in [0, 1, 2, 3, 4, 7, 8, 1023, 1024, 65535, 65536, 2**31 - 1, 2**31, 2**32 - 1]:
        want = 0 if v <= 1 else v.bit_length() - 1
        assert rules.rules_size_class(v) == want, v


def test_ticket_scheme_hands_out_every_entry_once(rules):
    # the compiled work-queue rule: classes largest first, at most 8 entries
    # (about 8192 voxels) per ticket; tickets t = k * lanes + lane drawn from
    # `lanes` counters by the work-groups of each lane
    ncls = rules.rules_classes()
    for cl in range(ncls):
        assert rules.rules_ticket_chunk(cl) == max(1, min(8, 8192 >> cl)), cl
    rng = np.random.default_rng(5)
    first = np.zeros(ncls, np.uint32)
    c_cl, e0, e1 = np.zeros(1, np.int32), np.zeros(1, np.uint32), np.zeros(1, np.uint32)
    for trial in range(40):
        counts = (rng.integers(0, 30, ncls) * (rng.random(ncls) < 0.4)).astype(np.uint32)
        total = int(rules.rules_ticket_offsets(counts.ctypes.data, first.ctypes.data))
        assert total == sum(-(-int(counts[c]) // max(1, min(8, 8192 >> c))) for c in range(ncls))
        grid = int(rng.choice([1, 5, 32, 100, 1280]))
        lanes = min(32, grid)
        seen = []
        last_cl = ncls
        for t in range(total):
            rules.rules_ticket_range(t, counts.ctypes.data, first.ctypes.data, c_cl.ctypes.data, e0.ctypes.data,
                                     e1.ctypes.data)
            assert int(c_cl[0]) <= last_cl     # largest classes first
            last_cl = int(c_cl[0])
            assert e0[0] < e1[0] <= counts[c_cl[0]]
            seen += [(int(c_cl[0]), e) for e in range(int(e0[0]), int(e1[0]))]
        # every ticket index below total is claimed by exactly one lane counter
        claimed = sorted(k * lanes + ln for ln in range(lanes) for k in range(total) if k * lanes + ln < total)
        assert claimed == list(range(total))
        assert sorted(seen) == sorted((cl, e) for cl in range(ncls) for e in range(int(counts[cl]))), trial


def test_staged_ring_indexing_counts_every_pair_once():
    # a model of the staged accumulation's ring walk (it lives inside the
    # kernel, not in a host-callable rule; the GPU parity tests of volumes and
    # longer offsets cover the kernel itself) (rows staged once per
    # chunk into ring_rows x W bytes, neighbours read at slot + dz*H + dy,
    # offsets flipped forward) against brute force, over tile partitions
    def fwd(o):
        dz, dy, dx = o
        return (-dz, -dy, -dx) if dz < 0 or (dz == 0 and (dy < 0 or (dy == 0 and dx < 0))) else o

    def staged(lev, offs, ra, rb, ring_bytes, ts):
        D, H, W = lev.shape
        rows, ring_rows = D * H, ring_bytes // W
        reach = max([fz * H + fy for fz, fy, fx in map(fwd, offs) if abs(fy) < H and abs(fx) < W] + [0])
        if ring_rows < reach + 4:
            return None
        C, ring, cnt, staged_to, r0 = ring_rows - reach, np.full(ring_rows * W, -1), {}, ra, ra
        while r0 < rb:
            r1 = min(r0 + C, rb)
            for f in range(0, (r1 + reach - staged_to) * W):
                r, x = staged_to + f // W, f % W
                ring[((r - ra) % ring_rows) * W + x] = lev.reshape(rows, W)[r, x] if r < rows else 0
            staged_to = r1 + reach
            for f in range((r1 - r0) * W):
                r, x = r0 + f // W, f % W
                slot, y = (r - ra) % ring_rows, r % H
                lv = ring[slot * W + x]
                assert lv >= 0
                for d, o in enumerate(offs):
                    dz, dy, dx = fwd(o)
                    if lv and 0 <= y + dy < H and 0 <= x + dx < W:
                        s2 = slot + dz * H + dy
                        s2 -= ring_rows if s2 >= ring_rows else 0
                        lw = ring[s2 * W + x + dx]
                        assert lw >= 0
                        if lw:
                            k = (d, min(lv, lw), max(lv, lw))
                            cnt[k] = cnt.get(k, 0) + 1
            r0 += C
        return cnt

    rng = np.random.default_rng(12)
    off3 = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 1), (0, 1, -1), (1, 0, 1), (1, 0, -1), (1, 1, 0), (1, -1, 0),
            (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)]
    sets = [off3, [(-a, -b, -c) for a, b, c in off3[:7]], [(0, 0, 2), (0, -2, 2), (0, -2, 0), (0, -2, -2)]]
    checked = 0
    for trial in range(24):
        D, H, W = int(rng.integers(1, 5)), int(rng.integers(1, 8)), int(rng.integers(1, 10))
        offs = sets[trial % 3]
        lev = rng.integers(1, 5, (D, H, W)) * (rng.random((D, H, W)) < 0.7)
        want = {}
        for z, y, x in zip(*np.nonzero(lev)):
            for d, (dz, dy, dx) in enumerate(offs):
                zz, yy, xx = z + dz, y + dy, x + dx
                if 0 <= zz < D and 0 <= yy < H and 0 <= xx < W and lev[zz, yy, xx]:
                    a, b = lev[z, y, x], lev[zz, yy, xx]
                    want[(d, min(a, b), max(a, b))] = want.get((d, min(a, b), max(a, b)), 0) + 1
        cuts = sorted({0, D * H, *map(int, rng.integers(0, D * H + 1, 2))})
        for ring_bytes in (W * (H + 5), W * (2 * H + 3), 300):
            got, ok = {}, True
            for ra, rb in zip(cuts[:-1], cuts[1:]):
                part = staged(lev, offs, ra, rb, ring_bytes, 7) if ra < rb else {}
                if part is None:
                    ok = False
                    break
                for k, v in part.items():
                    got[k] = got.get(k, 0) + v
            if ok:
                assert got == want, (D, H, W, cuts, ring_bytes)
                checked += 1
    assert checked >= 20


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)
