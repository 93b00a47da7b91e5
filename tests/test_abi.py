"""C-ABI checks that need no GPU: the library loads and exports every symbol
include/nyx.h declares; static tables agree with the oracle; device-free calls."""
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


def test_split_rule_covers_rows_and_columns():
    # host copy of the tiling rule the device uses: tiles partition the bbox
    from itertools import product

    def tiles_for(n, rows, width, split, tile):
        if n <= split or tile == 0:
            return 1, 1
        nt = (n + tile - 1) // tile
        rb = min(nt, rows)
        cb = min((nt + rb - 1) // rb, width)
        return rb, max(cb, 1)

    def bounds(rows, width, nt, tc, t):
        nrb = nt // tc
        rpt = (rows + nrb - 1) // nrb
        cpt = (width + tc - 1) // tc
        r, c = divmod(t, tc)
        ra, ca = min(r * rpt, rows), min(c * cpt, width)
        return ra, min(ra + rpt, rows), ca, min(ca + cpt, width)

    for rows, width, n, tile in product([1, 3, 17, 100], [1, 5, 64, 300], [10, 1000, 30000], [7, 64, 1024]):
        rb, cb = tiles_for(n, rows, width, tile, tile)
        cover = np.zeros((rows, width), int)
        for t in range(rb * cb):
            ra, rb_, ca, cb_ = bounds(rows, width, rb * cb, cb, t)
            cover[ra:rb_, ca:cb_] += 1
        assert np.all(cover == 1), (rows, width, n, tile)
