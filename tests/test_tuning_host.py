"""Tuning cache files on the host (no GPU): write/read round trip, the arch
filter, range checks and malformed files."""
import os

import pytest

from paper_2007_07627_amd import binding as B


def _entries():
    return [B.make_entry(16, 16, B.ICP_P2P_WELSCH, B.ICP_NN_CLUSTER, 12.5, slice_min=8, list_margin=0.16,
                         grid_per_cu=32),
            B.make_entry(11, 12, B.ICP_P2PL_WELSCH, B.ICP_NN_BRUTE, 0.75, batch=1, brute_items=16384,
                         brute_clusters=16, grid_per_cu=8)]


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tuning_gfx950.json")
    src = _entries()
    B.icp_tuning_file_write(path, "gfx950", src)
    got = B.icp_tuning_file_read(path, "gfx950")
    assert [B.entry_dict(e) for e in got] == [B.entry_dict(e) for e in src]
    assert B.icp_tuning_file_read(path, None)  # any arch
    assert B.icp_tuning_file_read(path, "gfx942") == []  # another arch's table holds nothing for it
    assert "gfx950" in open(path).read()


def test_defaults_and_empty_table(tmp_path):
    d = B.icp_tuning_default()
    assert d == {"slice_min": 6, "list_margin": pytest.approx(0.08), "brute_clusters": 8,
                 "brute_items": 8192, "grid_per_cu": 16}
    path = str(tmp_path / "empty.json")
    B.icp_tuning_file_write(path, "gfx950", [])
    assert B.icp_tuning_file_read(path, "gfx950") == []


def test_malformed_and_out_of_range(tmp_path):
    rc, _ = B.icp_tuning_file_read(str(tmp_path / "missing.json"), "gfx950", raw=True)
    assert rc == B.ICP_ERR_INVALID_ARG
    bad = tmp_path / "bad.json"
    bad.write_text('{"arch": "gfx950", "entries": [{"m_bucket": 3, "n_bucket": 4}]}')
    assert B.icp_tuning_file_read(str(bad), "gfx950", raw=True)[0] == B.ICP_ERR_INVALID_ARG
    path = str(tmp_path / "range.json")
    e = _entries()
    e[0].tuning.slice_min = 0
    B.icp_tuning_file_write(path, "gfx950", e)
    assert B.icp_tuning_file_read(path, "gfx950", raw=True)[0] == B.ICP_ERR_INVALID_ARG
    assert B.icp_tuning_file_write(path, 'gf"x', _entries(), raw=True) == B.ICP_ERR_INVALID_ARG
