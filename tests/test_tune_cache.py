"""Host-side checks of the tuning table (no GPU): the text form round-trips,
malformed files are rejected as a whole, argument checks of the autotuner
fail before any device work, and without a device a loaded table never
changes the configuration ctv_tiling reports."""
import ctypes
import json
import os

import pytest

from paper_2109_05496_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libctv.so not built")

INVALID = -1
ENTRIES = [
    {"arch": "gfx950:sramecc+:xnack-/256cu", "key": "00000000000000aa", "fuse": 9, "tile_waves": 8,
     "tile_rows": 8, "ms": 2.5, "what": "plain 1i m=2048 n=2048"},
    {"arch": "gfx950:sramecc+:xnack-/256cu", "key": "123456789abcdef0", "fuse": 6, "tile_waves": 8,
     "tile_rows": 4, "ms": 0.125, "what": "batched count=3"},
    {"arch": "gfx942/304cu", "key": "00000000000000aa", "fuse": 7, "tile_waves": 16, "tile_rows": 4, "ms": 1.0,
     "what": "another device"},
]


@pytest.fixture(autouse=True)
def clean_table():
    _lib.lib().ctv_tune_cache_clear()
    yield
    _lib.lib().ctv_tune_cache_clear()


def write_lines(path, objs):
    with open(path, "w") as f:
        for o in objs:
            f.write(json.dumps(o) + "\n")


def test_table_round_trip(tmp_path):
    src, dst = tmp_path / "in.jsonl", tmp_path / "out.jsonl"
    write_lines(src, ENTRIES)
    _lib.call("ctv_tune_cache_load", str(src).encode())
    assert _lib.lib().ctv_tune_cache_size() == 3
    # loading again replaces entries with the same (arch, key)
    _lib.call("ctv_tune_cache_load", str(src).encode())
    assert _lib.lib().ctv_tune_cache_size() == 3
    _lib.call("ctv_tune_cache_save", str(dst).encode())
    got = [json.loads(line) for line in open(dst) if line.strip()]
    key = lambda o: (o["arch"], o["key"])
    assert sorted(got, key=key) == sorted(ENTRIES, key=key)
    _lib.call("ctv_tune_cache_clear")
    assert _lib.lib().ctv_tune_cache_size() == 0


@pytest.mark.parametrize("bad", [
    dict(fuse=0), dict(fuse=17), dict(fuse=2.5), dict(tile_waves=8, tile_rows=16), dict(tile_waves=-1),
    dict(tile_waves=4, tile_rows=4), dict(key="xyz"), dict(arch=""), dict(tile_waves=99999999999),
    dict(fuse=1e300), dict(tile_rows=-1e12),
])
def test_malformed_table_rejected_whole(tmp_path, bad):
    path = tmp_path / "bad.jsonl"
    write_lines(path, [ENTRIES[0], dict(ENTRIES[1], **bad)])
    assert _lib.lib().ctv_tune_cache_load(str(path).encode()) == INVALID
    assert "malformed" in _lib.lib().ctv_last_error().decode()
    assert _lib.lib().ctv_tune_cache_size() == 0


def test_missing_field_and_missing_file(tmp_path):
    path = tmp_path / "short.jsonl"
    e = dict(ENTRIES[0])
    del e["tile_rows"]
    write_lines(path, [e])
    assert _lib.lib().ctv_tune_cache_load(str(path).encode()) == INVALID
    assert _lib.lib().ctv_tune_cache_load(str(tmp_path / "none.jsonl").encode()) == INVALID
    assert _lib.lib().ctv_tune_cache_load(None) == INVALID
    assert _lib.lib().ctv_tune_cache_save(None) == INVALID


def test_autotune_argument_checks():
    L = _lib.lib()
    p = _lib.make_params("1i", iters=20)
    lam = (ctypes.c_float * 1)(0.1)
    d = ctypes.c_void_p(0x1000)
    res = (_lib.Tuning * 4)()
    cnt = ctypes.c_int32()

    def status(p=p, reps=3, results=res, max_results=4):
        return L.ctv_autotune(ctypes.byref(p), 1, 64, 64, d, lam, None, d, d, 1 << 30, reps, results,
                              max_results, ctypes.byref(cnt), None, None)

    assert status(reps=0) == INVALID
    assert status(reps=101) == INVALID
    assert status(results=None, max_results=4) == INVALID
    assert status(max_results=-1) == INVALID
    assert status(p=_lib.make_params("1i", iters=20, schedule="flow")) == INVALID
    bad = _lib.make_params("1i", iters=20)
    bad.struct_size = 4
    assert status(p=bad) == INVALID
    descs = (_lib.ImageDesc * 1)()
    descs[0].m, descs[0].n, descs[0].lam, descs[0].iters, descs[0].support_offset = 8, 8, 0.1, 10, -1
    assert L.ctv_batched_autotune(descs, 1, ctypes.byref(p), d, None, d, d, 1 << 30, 0, res, 4,
                                  ctypes.byref(cnt), None, None) == INVALID
    assert L.ctv_batched_autotune(descs, 0, ctypes.byref(p), d, None, d, d, 1 << 30, 3, res, 4,
                                  ctypes.byref(cnt), None, None) == INVALID


def test_table_without_device_keeps_default(tmp_path):
    path = tmp_path / "t.jsonl"
    write_lines(path, ENTRIES)
    _lib.call("ctv_tune_cache_load", str(path).encode())
    from paper_2109_05496_amd import api
    assert api.tiling(0, 200, 2048, 2048, detail=True) == (8, 64, 8, 8)
    found = ctypes.c_int32(7)
    p = _lib.make_params("1i", iters=200)
    _lib.call("ctv_tune_lookup", ctypes.byref(p), 1, 2048, 2048, ctypes.byref(found), None)
    assert found.value == 0
