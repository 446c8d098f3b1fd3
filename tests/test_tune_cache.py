"""Persistent store of the CG launch-shape autotuner (host-only library
calls sdgp_tune_cache_get / sdgp_tune_cache_put; no GPU needed)."""
import json
import os

import pytest

from paper_2205_09070_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libsdgp.so not built")


def test_roundtrip_and_json(tmp_path):
    f = tmp_path / "sub" / "tune.json"
    k1 = "gfx950|ni16|ns1|b1|n19|r12|lr1|pc1"
    k2 = "gfx950|ni8|ns2|b2|n17|r8|lr0|pc1"
    assert _lib.tune_cache_get(f, k1) is None              # no file yet
    _lib.tune_cache_put(f, k1, (16384, 768, 1, 1))
    _lib.tune_cache_put(f, k2, (32768, 1536, 0, 0))
    assert _lib.tune_cache_get(f, k1) == (16384, 768, 1, 1)
    assert _lib.tune_cache_get(f, k2) == (32768, 1536, 0, 0)
    # overwrite
    _lib.tune_cache_put(f, k1, (65528, 2304, 0, 1))
    assert _lib.tune_cache_get(f, k1) == (65528, 2304, 0, 1)
    doc = json.load(open(f))
    assert set(doc) == {k1, k2}
    assert doc[k1]["spmm_blocks"] == 65528 and doc[k1]["update_blocks"] == 2304
    assert doc[k2]["union_spmm"] == 0 and doc[k2]["fw_mfma"] == 0
    assert not [p for p in os.listdir(f.parent) if ".tmp" in p]   # no temporary left behind


def test_entries_written_by_another_process_are_read(tmp_path):
    """The file is the interface: entries another writer left are read, and
    lines that do not parse (or hold invalid values) are ignored."""
    f = tmp_path / "tune.json"
    f.write_text('{\n'
                 'garbage line\n'
                 '"a|b": {"spmm_blocks": 8192, "update_blocks": 100, "union_spmm": -1, "fw_mfma": 1},\n'
                 '"bad|grid": {"spmm_blocks": 12, "update_blocks": 100, "union_spmm": 0, "fw_mfma": 0},\n'
                 '"bad|union": {"spmm_blocks": 64, "update_blocks": 100, "union_spmm": 3, "fw_mfma": 0},\n'
                 '"missing|field": {"spmm_blocks": 64, "union_spmm": 0, "fw_mfma": 0}\n'
                 '}\n')
    assert _lib.tune_cache_get(f, "a|b") == (8192, 100, -1, 1)
    for k in ("bad|grid", "bad|union", "missing|field", "nope"):
        assert _lib.tune_cache_get(f, k) is None
    _lib.tune_cache_put(f, "c|d", (64, 1, 0, 0))
    doc = json.load(open(f))            # rewritten as valid JSON, invalid lines dropped
    assert set(doc) == {"a|b", "c|d"}


@pytest.mark.parametrize("values", [(12, 100, 0, 0), (0, 100, 0, 0), (65536, 100, 0, 0), (64, 0, 0, 0),
                                    (64, 70000, 0, 0), (64, 100, 2, 0), (64, 100, 0, -2)])
def test_invalid_values_rejected(tmp_path, values):
    with pytest.raises(_lib.SdgpError):
        _lib.tune_cache_put(tmp_path / "t.json", "k", values)
    assert not (tmp_path / "t.json").exists()


def test_invalid_keys_rejected(tmp_path):
    for key in ('with"quote', "with\nnewline", ""):
        with pytest.raises(_lib.SdgpError):
            _lib.tune_cache_put(tmp_path / "t.json", key, (64, 1, 0, 0))


def test_unwritable_store_still_serves_the_process(tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    f = blocker / "tune.json"           # parent is a file: cannot be created
    with pytest.raises(_lib.SdgpError):
        _lib.tune_cache_put(f, "k|unwritable", (256, 8, 1, 0))
    assert _lib.tune_cache_get(f, "k|unwritable") == (256, 8, 1, 0)
