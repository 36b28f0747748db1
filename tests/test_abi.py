"""The C-ABI library loads and exports every call its header declares; the
argument checks that need no device reject bad input.  No compute calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1603_08390_amd as genie

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genie.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(genie_[a-z0-9_]+)\s*\(", text)))


def test_library_is_built():
    assert os.path.exists(genie.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    lib = genie.load()
    names = _declared()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(genie.EXPORTED)


def test_binding_names_match_header():
    for name in _declared():
        if name in ("genie_last_error", "genie_free_index", "genie_index_info_get"):
            continue
        assert hasattr(genie, name), name


def test_argument_errors_without_device():
    lib = genie.load()
    out = ctypes.c_void_p()
    vals = np.zeros((4, 2), dtype=np.uint32)
    # null values / null out
    assert lib.genie_build_index(None, 4, 2, 3, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert lib.genie_build_index(vals.ctypes.data, 4, 2, 3, None) == genie.GENIE_EINVAL
    # zero sizes
    assert lib.genie_build_index(vals.ctypes.data, 0, 2, 3, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert lib.genie_build_index(vals.ctypes.data, 4, 0, 3, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert lib.genie_build_index(vals.ctypes.data, 4, 2, 0, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert b"bad sizes" in lib.genie_last_error()
    # value >= n_buckets is caught before any device call
    bad = np.array([[0, 5]], dtype=np.uint32)
    assert lib.genie_build_index(bad.ctypes.data, 1, 2, 3, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert b"n_buckets" in lib.genie_last_error()
    # tiles other than 2^15 - 1 or 2^16 - 1 objects are refused
    for lg in (0, 14, 17):
        assert lib.genie_build_index_tiled(vals.ctypes.data, 4, 2, 3, lg,
                                           ctypes.byref(out)) == genie.GENIE_EINVAL
        assert b"tile_log2" in lib.genie_last_error()
    # search on a null index, bad k
    ids = np.zeros(4, dtype=np.uint32)
    off = np.array([0, 0], dtype=np.uint64)
    assert lib.genie_search(None, off.ctypes.data, None, 1, 1, ids.ctypes.data,
                            ids.ctypes.data) == genie.GENIE_EINVAL
    assert lib.genie_search_workspace_size(None, 1, 1) == 0
    # LSH argument checks
    assert lib.genie_lsh_signatures(None, 10, 4, None, None, ctypes.c_float(1.0), 3, None, 13,
                                    None, None) == genie.GENIE_EINVAL
    # n = 0 is a no-op
    assert lib.genie_lsh_signatures(None, 0, 4, None, None, ctypes.c_float(1.0), 3, None, 13,
                                    None, None) == genie.GENIE_OK
    # schedule and row-count search on a null index
    assert lib.genie_index_set_scan_schedule(None, 0) == genie.GENIE_EINVAL
    assert lib.genie_index_set_scan_shape(None, 1024, 4) == genie.GENIE_EINVAL
    assert lib.genie_search_rows_async(None, None, None, 0, 4, None, 8, 10, None,
                                       ctypes.c_float(0.0), None, None, None, 0,
                                       None) == genie.GENIE_EINVAL


def test_sequence_and_keyword_set_argument_errors_without_device():
    lib = genie.load()
    out = ctypes.c_void_p()
    EINVAL, ERANGE = genie.GENIE_EINVAL, genie.GENIE_ERANGE
    chars = np.frombuffer(b"abcabc", np.uint8).copy()
    off = np.array([0, 3, 6], dtype=np.uint64)
    c, o = chars.ctypes.data, off.ctypes.data
    assert lib.genie_seq_build(c, None, 2, 3, 16, ctypes.byref(out)) == EINVAL
    assert lib.genie_seq_build(c, o, 2, 3, 16, None) == EINVAL
    assert lib.genie_seq_build(c, o, 0, 3, 16, ctypes.byref(out)) == EINVAL
    for gram in (0, 9):
        assert lib.genie_seq_build(c, o, 2, gram, 16, ctypes.byref(out)) == EINVAL
        assert b"gram" in lib.genie_last_error()
    assert lib.genie_seq_build(None, o, 2, 3, 16, ctypes.byref(out)) == EINVAL
    first = np.array([1, 3, 6], dtype=np.uint64)
    assert lib.genie_seq_build(c, first.ctypes.data, 2, 3, 16, ctypes.byref(out)) == EINVAL
    assert b"offsets[0]" in lib.genie_last_error()
    down = np.array([0, 4, 3], dtype=np.uint64)
    assert lib.genie_seq_build(c, down.ctypes.data, 2, 3, 16, ctypes.byref(out)) == EINVAL
    assert b"decrease" in lib.genie_last_error()
    # tiles are checked by the keyword-set builder before any device call
    assert lib.genie_seq_build(c, o, 2, 3, 14, ctypes.byref(out)) == EINVAL
    assert b"tile_log2" in lib.genie_last_error()
    # 256 byte values: 256^4 n-gram codes exceed the 2^24 table
    every = np.arange(256, dtype=np.uint8)
    eoff = np.array([0, 256], dtype=np.uint64)
    assert lib.genie_seq_build(every.ctypes.data, eoff.ctypes.data, 1, 4, 16,
                               ctypes.byref(out)) == ERANGE
    assert b"n-gram codes" in lib.genie_last_error()
    # calls on a null sequence index
    assert lib.genie_seq_info_get(None, None) == EINVAL
    assert lib.genie_seq_match_index(None) is None
    assert lib.genie_seq_workspace_size(None, 1, 1, 1) == 0
    assert lib.genie_seq_decompose_async(None, None, None, 0, 1, None, None) == EINVAL
    assert lib.genie_seq_verify_async(None, None, None, 0, 1, 40, None, None, 32, 1, None, None,
                                      None, None) == EINVAL
    assert lib.genie_seq_search_async(None, None, None, 0, 1, 40, 32, 1, None, None, None, None,
                                      0, None) == EINVAL
    lib.genie_seq_free(None)
    # keyword sets: null pointers, a key >= n_keys, decreasing offsets, tiles
    keys = np.array([0, 1, 4], dtype=np.uint32)
    ko = np.array([0, 2, 3], dtype=np.uint64)
    k_, ko_ = keys.ctypes.data, ko.ctypes.data
    assert lib.genie_build_index_sets(None, k_, 2, 5, 16, ctypes.byref(out)) == EINVAL
    assert lib.genie_build_index_sets(ko_, k_, 2, 5, 16, None) == EINVAL
    assert lib.genie_build_index_sets(ko_, k_, 2, 4, 16, ctypes.byref(out)) == EINVAL
    assert b"out of range" in lib.genie_last_error()
    kd = np.array([0, 3, 2], dtype=np.uint64)
    assert lib.genie_build_index_sets(kd.ctypes.data, k_, 2, 5, 16, ctypes.byref(out)) == EINVAL
    assert b"decrease" in lib.genie_last_error()
    assert lib.genie_build_index_sets(ko_, k_, 2, 5, 17, ctypes.byref(out)) == EINVAL
    assert lib.genie_build_index_sets(ko_, k_, 0, 5, 16, ctypes.byref(out)) == EINVAL


def test_header_limits_match_binding():
    text = open(HEADER).read()
    for name, val in (("GENIE_MAX_K", genie.GENIE_MAX_K), ("GENIE_MAX_ITEMS", genie.GENIE_MAX_ITEMS),
                      ("GENIE_TILE_OBJECTS", genie.GENIE_TILE_OBJECTS),
                      ("GENIE_EINVAL", genie.GENIE_EINVAL), ("GENIE_ERANGE", genie.GENIE_ERANGE)):
        m = re.search(r"#define\s+%s\s+\(?(-?\d+)" % name, text)
        assert m and int(m.group(1)) == val, name


def test_oracle_shares_no_code_with_library():
    """The oracle's sources name nothing from the GPU library and the
    library's sources name nothing from the oracle."""
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith((".c", ".py", ".h")):
            text = open(os.path.join(odir, f)).read()
            assert "genie.h" not in text and "paper_1603_08390_amd" not in text, f
            assert "csrc" not in text and "libgenie" not in text, f
    csrc = os.path.join(ROOT, "paper_1603_08390_amd", "csrc")
    for f in os.listdir(csrc):
        assert "oracle" not in open(os.path.join(csrc, f)).read().lower(), f
    assert "oracle" not in open(os.path.join(ROOT, "paper_1603_08390_amd", "__init__.py")).read()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_noalloc_argument_errors_without_device():
    lib = genie.load()
    # the held-workspace search on a null index
    assert lib.genie_search_noalloc_async(None, None, None, 0, 4, 8, 10, None, None,
                                          None) == genie.GENIE_EINVAL
    assert b"null index" in lib.genie_last_error()


def test_probe_argument_errors_without_device():
    lib = genie.load()
    # probes: bad mode, zero sizes, null outputs
    out = ctypes.c_double()
    assert lib.genie_probe_lds_atomics(4, 1, 1, None, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert lib.genie_probe_lds_atomics(0, 0, 1, None, ctypes.byref(out)) == genie.GENIE_EINVAL
    assert lib.genie_probe_hbm(None, None, 1 << 20, 1, None, ctypes.byref(out),
                               None) == genie.GENIE_EINVAL
    assert lib.genie_probe_hbm(None, None, 15, 1, None, None, None) == genie.GENIE_EINVAL


def test_hash_slots_argument_errors_without_device():
    lib = genie.load()
    assert lib.genie_index_set_hash_slots(None, 4) == genie.GENIE_EINVAL
    assert b"hash table slots" in lib.genie_last_error()
