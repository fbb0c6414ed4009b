"""Host-side checks of libnrlsh that need no GPU: the library loads, exports
every function include/nrlsh.h declares, and rejects bad arguments on the
host before any device work."""
import ctypes as C

import numpy as np
import pytest

import paper_1809_08782_amd as nr
from paper_1809_08782_amd import _lib

INVALID, NOT_FINITE = 1, 2


def test_library_exports_every_declared_symbol():
    L = nr.lib()
    declared = nr.header_symbols()
    assert "nrlsh_build" in declared and "nrlsh_query" in declared
    missing = [s for s in declared if not hasattr(L, s)]
    assert missing == []


def test_library_is_gfx950_code():
    with open(_lib.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"gfx950" in blob


def _build(items_ptr, n, d, m, L):
    h = C.c_void_p()
    st = nr.lib().nrlsh_build(items_ptr, n, d, m, L, 1, C.byref(h))
    return st, h


@pytest.mark.parametrize("n,d,m,L", [
    (0, 4, 1, 8),       # n < 1
    (10, 0, 1, 8),      # d < 1
    (10, 4, 0, 8),      # m < 1
    (10, 4, 11, 8),     # m > n
    (10, 4, 2, 0),      # L < 1
    (10, 4, 2, 65),     # L > 64
])
def test_build_rejects_bad_shapes(n, d, m, L):
    X = np.ones((max(n, 1), max(d, 1)), np.float32)
    st, h = _build(X.ctypes.data, n, d, m, L)
    assert st == INVALID
    assert not h.value
    assert nr.nrlsh_last_error()


def test_build_rejects_null_pointers():
    st, _ = _build(None, 10, 4, 2, 8)
    assert st == INVALID
    X = np.ones((10, 4), np.float32)
    assert nr.lib().nrlsh_build(X.ctypes.data, 10, 4, 2, 8, 1, None) == INVALID


def test_build_rejects_bad_eps():
    X = np.ones((10, 4), np.float32)
    h = C.c_void_p()
    for eps in (1.0, -0.1, float("nan")):
        opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 0, None, eps)
        assert nr.lib().nrlsh_build_ex(X.ctypes.data, 10, 4, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID


def test_build_rejects_misaligned_device_items():
    # rejected on the host before any device call: the pointer is never read
    h = C.c_void_p()
    opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 1, None, 0.0)
    for d, addr in ((8, 0x1008), (6, 0x1004), (5, 0x1002)):
        assert nr.lib().nrlsh_build_ex(C.c_void_p(addr), 10, d, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID
        assert "aligned" in nr.nrlsh_last_error()
        assert not h.value


def test_build_rejects_unknown_partition():
    X = np.ones((10, 4), np.float32)
    h = C.c_void_p()
    opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 0, None, 0.0, 0, 0, 0.0, 2)
    assert nr.lib().nrlsh_build_ex(X.ctypes.data, 10, 4, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID
    assert "partition" in nr.nrlsh_last_error()


def test_build_rejects_bad_projections():
    X = np.ones((10, 4), np.float32)
    h = C.c_void_p()
    opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 0, None, 0.0, 0, 0, 0.0, 0, 2)
    assert nr.lib().nrlsh_build_ex(X.ctypes.data, 10, 4, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID
    assert "projections" in nr.nrlsh_last_error()
    # per-subset projections exist only for the FP32 hash
    for storage in (1, 2):
        opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 0, None, 0.0, storage, 0, 0.0, 0, 1)
        assert nr.lib().nrlsh_build_ex(X.ctypes.data, 10, 4, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID
        assert "per-subset" in nr.nrlsh_last_error()


def test_bucket_table_options_rejected():
    X = np.ones((10, 4), np.float32)
    h = C.c_void_p()
    opts = _lib.BuildOpts(C.sizeof(_lib.BuildOpts), 0, None, 0.0, 0, 0, 0.0, 0, 0, 2)
    assert nr.lib().nrlsh_build_ex(X.ctypes.data, 10, 4, 2, 8, 1, C.byref(opts), C.byref(h)) == INVALID
    assert "bucket_tables" in nr.nrlsh_last_error()
    U = C.c_int64()
    assert nr.lib().nrlsh_get_bucket_table(None, C.byref(U), None, None, None, None) == INVALID
    Q = np.ones((2, 4), np.float32)
    ids = np.empty((2, 4), np.int64)
    ips = np.empty((2, 4), np.float32)
    fake = C.c_void_p(1)  # never dereferenced: the option check comes first
    qo = _lib.QueryOpts(C.sizeof(_lib.QueryOpts), 0, None, 0, 0, 7)
    assert nr.lib().nrlsh_query_ex(fake, Q.ctypes.data, 2, 4, 10, C.byref(qo), ids.ctypes.data,
                                   ips.ctypes.data) == INVALID
    assert "probe_mode" in nr.nrlsh_last_error()


def test_query_rejects_bad_arguments():
    L = nr.lib()
    Q = np.ones((2, 4), np.float32)
    ids = np.empty((2, 4), np.int64)
    ips = np.empty((2, 4), np.float32)
    assert L.nrlsh_query(None, Q.ctypes.data, 2, 4, 10, ids.ctypes.data, ips.ctypes.data) == INVALID
    fake = C.c_void_p(1)  # never dereferenced: argument checks come first
    assert L.nrlsh_query(fake, Q.ctypes.data, 2, 0, 10, ids.ctypes.data, ips.ctypes.data) == INVALID
    assert L.nrlsh_query(fake, Q.ctypes.data, 2, 1025, 10, ids.ctypes.data, ips.ctypes.data) == INVALID
    assert L.nrlsh_query(fake, Q.ctypes.data, 2, 4, 0, ids.ctypes.data, ips.ctypes.data) == INVALID
    assert L.nrlsh_query(fake, Q.ctypes.data, -1, 4, 10, ids.ctypes.data, ips.ctypes.data) == INVALID
    assert L.nrlsh_query(fake, None, 2, 4, 10, ids.ctypes.data, ips.ctypes.data) == INVALID
    assert L.nrlsh_query(fake, Q.ctypes.data, 2, 4, 10, None, ips.ctypes.data) == INVALID
    # nq = 0 is a no-op that never touches the device
    assert L.nrlsh_query(fake, None, 0, 4, 10, None, None) == 0


def test_query_rejects_unknown_rerank_mode():
    L = nr.lib()
    Q = np.ones((2, 4), np.float32)
    ids = np.empty((2, 4), np.int64)
    ips = np.empty((2, 4), np.float32)
    fake = C.c_void_p(1)  # never dereferenced: argument checks come first
    opts = _lib.QueryOpts(C.sizeof(_lib.QueryOpts), 0, None, 7)
    assert L.nrlsh_query_ex(fake, Q.ctypes.data, 2, 4, 10, C.byref(opts), ids.ctypes.data,
                            ips.ctypes.data) == INVALID


def test_free_null_and_profile_registry():
    nr.lib().nrlsh_free(None)
    nr.nrlsh_profile_reset()
    assert nr.nrlsh_profile_get("rerank") == (0.0, 0)
    with pytest.raises(nr.NrlshError):
        _lib._check(INVALID)


def test_inspection_rejects_null():
    L = nr.lib()
    assert L.nrlsh_get_projection(None, None) == INVALID
    assert L.nrlsh_get_codes(None, None) == INVALID
    assert L.nrlsh_get_build_stats(None, None) == INVALID
    assert L.nrlsh_query_codes(None, None, 1, None) == INVALID
    assert L.nrlsh_query_candidates(None, None, 1, 1, None) == INVALID


def _desc(index=1, queries=1, nq=2, T=10, ids=1, ips=1):
    return _lib.QueryDesc(index, queries, nq, T, ids, ips)


@pytest.mark.parametrize("field,bad", [("index", 0), ("nq", -1), ("T", 0), ("queries", 0),
                                       ("ids", 0), ("ips", 0)])
def test_multi_rejects_bad_descriptors(field, bad):
    """Descriptor checks run on the host before any index is touched (the
    index pointers here are never dereferenced)."""
    d = (_lib.QueryDesc * 1)(_desc(**{field: bad}))
    h = C.c_void_p()
    assert nr.lib().nrlsh_multi_plan_create(d, 1, 10, None, C.byref(h)) == INVALID
    assert not h.value
    assert nr.nrlsh_last_error()


def test_multi_rejects_bad_counts_k_and_options():
    L = nr.lib()
    d = (_lib.QueryDesc * 1)(_desc(index=0))
    h = C.c_void_p()
    assert L.nrlsh_multi_plan_create(None, 1, 10, None, C.byref(h)) == INVALID
    assert L.nrlsh_multi_plan_create(d, 0, 10, None, C.byref(h)) == INVALID
    assert L.nrlsh_multi_plan_create(d, 4097, 10, None, C.byref(h)) == INVALID
    assert L.nrlsh_multi_plan_create(d, 1, 0, None, C.byref(h)) == INVALID
    assert L.nrlsh_multi_plan_create(d, 1, 1025, None, C.byref(h)) == INVALID
    assert L.nrlsh_multi_plan_create(d, 1, 10, None, None) == INVALID
    # options are read first: the message names the option, not the descriptor
    for key, v, word in (("tune", 9, "tune"), ("chunk", 100, "chunk"), ("slice", -64, "slice"),
                         ("struct_size", 4, "struct_size"), ("persistent", 1, "persistent")):
        o = _lib.MultiOpts(C.sizeof(_lib.MultiOpts), 0, None, 1, 0, 0, 0)
        setattr(o, key, v)
        assert L.nrlsh_multi_plan_create(d, 1, 10, C.byref(o), C.byref(h)) == INVALID
        assert word in nr.nrlsh_last_error()
    assert L.nrlsh_multi_run(None, d, 1) == INVALID
    L.nrlsh_multi_plan_free(None)


def test_tune_table_lookup_on_empty_table():
    nr.nrlsh_tune_clear()
    assert nr.nrlsh_tune_lookup(128, 32, 100) is None
