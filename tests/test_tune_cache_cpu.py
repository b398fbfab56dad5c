"""Tuning-cache file of the library (host code, no GPU): hit, miss, replace,
other entries kept, and corrupt or foreign files ignored then rewritten."""
import ctypes
import json
import os

import pytest

from paper_1507_02525_amd import _binding as B


def _lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1507_02525_amd.build import build
        build()
    return B.lib()


def lookup(path, key):
    v = [ctypes.c_int(-7) for _ in range(4)]
    r = _lib().mrdft_tune_cache_lookup(str(path).encode(), key.encode(), *[ctypes.byref(a) for a in v])
    return r, tuple(a.value for a in v)


def store(path, key, t, g, o, s):
    return _lib().mrdft_tune_cache_store(str(path).encode(), key.encode(), t, g, o, s)


def test_miss_on_missing_file(tmp_path):
    r, v = lookup(tmp_path / "none.json", "gfx950|c64")
    assert r == 0 and v == (-7, -7, -7, -7)          # outputs untouched on a miss


def test_store_then_hit_and_replace(tmp_path):
    p = tmp_path / "tune.json"
    assert store(p, "gfx950|c64|m18", 11, 0, 3, 1) == 0
    assert lookup(p, "gfx950|c64|m18") == (1, (11, 0, 3, 1))
    assert lookup(p, "gfx950|c64|m17")[0] == 0
    assert store(p, "gfx950|r32|m16", 12, 0, 2, 0) == 0
    assert store(p, "gfx950|c64|m18", 12, 256, 0, 0) == 0          # replace one entry
    assert lookup(p, "gfx950|c64|m18") == (1, (12, 256, 0, 0))
    assert lookup(p, "gfx950|r32|m16") == (1, (12, 0, 2, 0))       # the other kept
    doc = json.loads(p.read_text())                                  # a valid JSON document
    assert doc["format"] == "mrdft-tune" and doc["version"] == 1 and len(doc["entries"]) == 2


@pytest.mark.parametrize("text", [
    "", "{", "not json", "[]", '{"format": "mrdft-tune", "version": 1}',
    '{"format": "mrdft-tune", "version": 2, "entries": {}}',
    '{"format": "other", "version": 1, "entries": {}}',
    '{"format": "mrdft-tune", "version": 1, "entries": {"k": {"tile_log": 11}}}',
    '{"format": "mrdft-tune", "version": 1, "entries": {"k": {"tile_log": -1, "grid": 0, "order": 0, "serial": 0}}}',
    '{"format": "mrdft-tune", "version": 1, "entries": {"k": {"tile_log": 11, "grid": 0, "order": 0, "serial": 0}}} x',
    '{"format": "mrdft-tune", "version": 1, "entries": {"k": {"tile_log": 1.5, "grid": 0, "order": 0, "serial": 0}}}',
    '\x00\xff\xfe garbage',
])
def test_corrupt_or_foreign_file_is_ignored_and_rewritten(tmp_path, text):
    p = tmp_path / "tune.json"
    p.write_bytes(text.encode("latin-1"))
    assert lookup(p, "k")[0] == 0
    assert store(p, "k2", 11, 0, 3, 0) == 0
    assert lookup(p, "k2") == (1, (11, 0, 3, 0))
    assert json.loads(p.read_text())["version"] == 1


def test_entries_written_by_hand_are_read(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"format": "mrdft-tune", "version": 1,
                             "entries": {"a|b": {"serial": 1, "order": 2, "grid": 512, "tile_log": 11}}}, indent=3))
    assert lookup(p, "a|b") == (1, (11, 512, 2, 1))


@pytest.mark.parametrize("key", ["", 'a"b', "a\\b", "a\nb"])
def test_bad_keys_rejected(tmp_path, key):
    p = tmp_path / "tune.json"
    assert store(p, key, 11, 0, 0, 0) == B.MRDFT_E_INVALID_ARG
    assert lookup(p, key)[0] == -1
    assert not p.exists()


def test_negative_values_rejected(tmp_path):
    assert store(tmp_path / "t.json", "k", 11, -1, 0, 0) == B.MRDFT_E_INVALID_ARG


def test_unwritable_path_reports_alloc(tmp_path):
    assert store(tmp_path / "no_such_dir" / "t.json", "k", 11, 0, 0, 0) == B.MRDFT_E_ALLOC
