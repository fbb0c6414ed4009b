"""ctypes binding of libnrlsh (argument marshalling only).

Names follow the C ABI of ``include/nrlsh.h``.  Host numpy arrays go through
the host-pointer entry points; CUDA/HIP torch tensors go through the ``_ex``
entry points with device pointers and torch's current stream.  There is no
fallback: if ``libnrlsh.so`` is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnrlsh.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "nrlsh.h")

NRLSH_OK = 0
STATUS_NAMES = {0: "NRLSH_OK", 1: "NRLSH_E_INVALID_ARG", 2: "NRLSH_E_NOT_FINITE",
                3: "NRLSH_E_OUT_OF_MEMORY", 4: "NRLSH_E_DEVICE", 5: "NRLSH_E_INTERNAL"}


class NrlshError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class BuildOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("device_ptrs", C.c_int32),
                ("stream", C.c_void_p), ("eps", C.c_double), ("hash_storage", C.c_int32),
                ("margin_mode", C.c_int32), ("margin_param", C.c_double),
                ("partition", C.c_int32), ("projections", C.c_int32),
                ("bucket_tables", C.c_int32), ("hash_tables", C.c_int32)]


PARTITIONS = {"percentile": 0, "uniform": 1}
PROJECTIONS = {"shared": 0, "per_subset": 1}


STORAGES = {"fp32": 0, "bf16": 1, "fp8": 2}


class QueryOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("device_ptrs", C.c_int32), ("stream", C.c_void_p),
                ("rerank_mode", C.c_int32), ("rerank_storage", C.c_int32),
                ("probe_mode", C.c_int32), ("scan_guess", C.c_int32), ("dense_head", C.c_int32)]


PROBES = {"scan": 0, "table": 1, "single": 2}


RERANK_MODES = {"auto": 0, "gather": 1, "screen": 2, "screen_fp32": 3, "screen_bf16x3": 4}


class BuildStats(C.Structure):
    _fields_ = [("recomputed_items", C.c_int64), ("recomputed_bits", C.c_int64),
                ("recompute_flips", C.c_int64), ("lowp_items", C.c_int64),
                ("lowp_bits", C.c_int64), ("lowp_changed", C.c_int64),
                ("recompute_flips_tiny", C.c_int64)]


class QueryStats(C.Structure):
    _fields_ = [("mode", C.c_int32), ("screen_passes", C.c_int32), ("kept_total", C.c_int64),
                ("kept_max", C.c_int64), ("theta_unset", C.c_int64), ("lp_kept_total", C.c_int64),
                ("lp_kept_max", C.c_int64), ("lp_fallbacks", C.c_int32), ("probe_mode", C.c_int32),
                ("table_lookups", C.c_int64), ("table_walked", C.c_int64),
                ("table_passes", C.c_int64), ("screen_pairs", C.c_int64), ("scan_pairs", C.c_int64),
                ("collect_fallbacks", C.c_int64), ("dense_head_items", C.c_int64),
                ("lp_gathered_total", C.c_int64), ("dense_head_pairs", C.c_int64)]


class QueryDesc(C.Structure):
    _fields_ = [("index", C.c_void_p), ("queries", C.c_void_p), ("nq", C.c_int64),
                ("probe_budget", C.c_int64), ("out_ids", C.c_void_p), ("out_ips", C.c_void_p)]


class MultiOpts(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("device_ptrs", C.c_int32), ("stream", C.c_void_p),
                ("use_graph", C.c_int32), ("tune", C.c_int32), ("chunk", C.c_int32),
                ("slice", C.c_int32), ("persistent", C.c_int32)]


class MultiInfo(C.Structure):
    _fields_ = [("grid", C.c_int32), ("graph", C.c_int32), ("items", C.c_int64 * 7),
                ("tuned_classes", C.c_int32), ("pad", C.c_int32), ("tune_ms", C.c_double)]


TUNE_MODES = {"table": 0, "missing": 1, "all": 2, "default": 3}
MULTI_PHASES = ("qhash", "hist", "threshold", "tie", "emit", "rerank", "merge")

_lib = None
P = C.c_void_p
I32, I64, U64, F64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double


def lib():
    """Load libnrlsh.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_1809_08782_amd.build`")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.nrlsh_build.argtypes = [P, I64, I32, I32, I32, U64, C.POINTER(P)]
        L.nrlsh_build.restype = st
        L.nrlsh_build_ex.argtypes = [P, I64, I32, I32, I32, U64, C.POINTER(BuildOpts), C.POINTER(P)]
        L.nrlsh_build_ex.restype = st
        L.nrlsh_free.argtypes = [P]
        L.nrlsh_free.restype = None
        L.nrlsh_query.argtypes = [P, P, I64, I32, I64, P, P]
        L.nrlsh_query.restype = st
        L.nrlsh_query_ex.argtypes = [P, P, I64, I32, I64, C.POINTER(QueryOpts), P, P]
        L.nrlsh_query_ex.restype = st
        L.nrlsh_query_noalloc.argtypes = [P, P, I64, I32, I64, P, P, P, P]
        L.nrlsh_query_noalloc.restype = st
        L.nrlsh_last_error.argtypes = []
        L.nrlsh_last_error.restype = C.c_char_p
        L.nrlsh_index_info.argtypes = [P, C.POINTER(I64), C.POINTER(I32), C.POINTER(I32),
                                       C.POINTER(I32), C.POINTER(I32)]
        L.nrlsh_index_info.restype = st
        for name in ("nrlsh_get_projection", "nrlsh_get_keys", "nrlsh_get_codes",
                     "nrlsh_get_rank_table"):
            f = getattr(L, name)
            f.argtypes = [P, P]
            f.restype = st
        L.nrlsh_get_partition.argtypes = [P, P, P, P]
        L.nrlsh_get_partition.restype = st
        L.nrlsh_get_projection_sets.argtypes = [P, C.POINTER(I32)]
        L.nrlsh_get_projection_sets.restype = st
        L.nrlsh_get_bucket_table.argtypes = [P, C.POINTER(I64), P, P, P, P]
        L.nrlsh_get_bucket_table.restype = st
        L.nrlsh_get_layout.argtypes = [P, P, P]
        L.nrlsh_get_layout.restype = st
        L.nrlsh_get_hash_copy.argtypes = [P, P, P, C.POINTER(I32)]
        L.nrlsh_get_hash_copy.restype = st
        L.nrlsh_get_build_stats.argtypes = [P, C.POINTER(BuildStats)]
        L.nrlsh_get_build_stats.restype = st
        L.nrlsh_query_codes.argtypes = [P, P, I64, P]
        L.nrlsh_query_codes.restype = st
        L.nrlsh_query_candidates.argtypes = [P, P, I64, I64, P]
        L.nrlsh_query_candidates.restype = st
        L.nrlsh_query_candidates_ex.argtypes = [P, P, I64, I64, I32, P, P]
        L.nrlsh_query_candidates_ex.restype = st
        L.nrlsh_query_candidates_levels.argtypes = [P, P, I64, I64, P, P]
        L.nrlsh_query_candidates_levels.restype = st
        L.nrlsh_get_hash_tables.argtypes = [P, C.POINTER(I32)]
        L.nrlsh_get_hash_tables.restype = st
        L.nrlsh_get_codes_table.argtypes = [P, I32, P]
        L.nrlsh_get_codes_table.restype = st
        L.nrlsh_get_query_stats.argtypes = [C.POINTER(QueryStats)]
        L.nrlsh_get_query_stats.restype = st
        L.nrlsh_multi_plan_create.argtypes = [C.POINTER(QueryDesc), I32, I32,
                                              C.POINTER(MultiOpts), C.POINTER(P)]
        L.nrlsh_multi_plan_create.restype = st
        L.nrlsh_multi_run.argtypes = [P, C.POINTER(QueryDesc), I32]
        L.nrlsh_multi_run.restype = st
        L.nrlsh_multi_plan_free.argtypes = [P]
        L.nrlsh_multi_plan_free.restype = None
        L.nrlsh_query_multi.argtypes = [C.POINTER(QueryDesc), I32, I32, C.POINTER(MultiOpts)]
        L.nrlsh_query_multi.restype = st
        L.nrlsh_multi_plan_info.argtypes = [P, C.POINTER(MultiInfo), P, P]
        L.nrlsh_multi_plan_info.restype = st
        L.nrlsh_tune_clear.argtypes = []
        L.nrlsh_tune_clear.restype = None
        L.nrlsh_tune_lookup.argtypes = [I32, I32, I64, C.POINTER(I32), C.POINTER(I32)]
        L.nrlsh_tune_lookup.restype = I32
        L.nrlsh_profile_enable.argtypes = [I32]
        L.nrlsh_profile_enable.restype = None
        L.nrlsh_profile_reset.argtypes = []
        L.nrlsh_profile_reset.restype = None
        L.nrlsh_profile_get.argtypes = [C.c_char_p, C.POINTER(F64), C.POINTER(I64)]
        L.nrlsh_profile_get.restype = st
        _lib = L
    return _lib


def header_symbols() -> list:
    """Function names declared in include/nrlsh.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    decl = r"^(?:nrlsh_status|void|int32_t|const char\s*\*)\s*\*?\s*(nrlsh_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, text, re.M)))


def _check(status: int):
    if status != NRLSH_OK:
        raise NrlshError(status, lib().nrlsh_last_error().decode(errors="replace"))


def _is_torch_device(t) -> bool:
    try:
        import torch
    except ImportError:  # pragma: no cover
        return False
    return isinstance(t, torch.Tensor) and t.is_cuda


def _torch_stream(t):
    import torch
    return P(torch.cuda.current_stream(t.device).cuda_stream)


def _host_f32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2:
        raise ValueError("expected a 2-D (rows x d) array")
    return a


class Index:
    """Owns an ``nrlsh_index*`` (Algorithm 1 output).  Free with close()."""

    def __init__(self, handle: int):
        self._h = P(handle)
        n, d, m, L, dp = I64(), I32(), I32(), I32(), I32()
        _check(lib().nrlsh_index_info(self._h, C.byref(n), C.byref(d), C.byref(m), C.byref(L),
                                      C.byref(dp)))
        self.n, self.d, self.m, self.L, self.dp = n.value, d.value, m.value, L.value, dp.value
        sets = I32()
        _check(lib().nrlsh_get_projection_sets(self._h, C.byref(sets)))
        self.qsets = sets.value  # 1: shared projections; m: one block per sub-dataset
        tabs = I32()
        _check(lib().nrlsh_get_hash_tables(self._h, C.byref(tabs)))
        self.tables = tabs.value  # independent hash tables

    @property
    def handle(self):
        if not self._h:
            raise ValueError("index is closed")
        return self._h

    def close(self):
        if self._h:
            lib().nrlsh_free(self._h)
            self._h = P()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------- inspection
    def projection(self) -> np.ndarray:
        """(tables qsets L) x (d+1); block tau qsets + j serves hash table tau
        and, when qsets = m, sub-dataset j."""
        A = np.empty((self.tables * self.qsets * self.L, self.d + 1), dtype=np.float32)
        _check(lib().nrlsh_get_projection(self.handle, A.ctypes.data))
        return A

    def keys(self) -> np.ndarray:
        k = np.empty(self.n, dtype=np.float64)
        _check(lib().nrlsh_get_keys(self.handle, k.ctypes.data))
        return k

    def partition(self):
        sid = np.empty(self.n, dtype=np.int32)
        keymax = np.empty(self.m, dtype=np.float64)
        U = np.empty(self.m, dtype=np.float64)
        _check(lib().nrlsh_get_partition(self.handle, sid.ctypes.data, keymax.ctypes.data,
                                         U.ctypes.data))
        return sid, keymax, U

    def layout(self):
        perm = np.empty(self.n, dtype=np.int32)
        off = np.empty(self.m + 1, dtype=np.int64)
        _check(lib().nrlsh_get_layout(self.handle, perm.ctypes.data, off.ctypes.data))
        return perm, off

    def codes(self, table: int = 0) -> np.ndarray:
        c = np.empty(self.n, dtype=np.uint64)
        if table == 0:
            _check(lib().nrlsh_get_codes(self.handle, c.ctypes.data))
        else:
            _check(lib().nrlsh_get_codes_table(self.handle, int(table), c.ctypes.data))
        return c

    def rank_table(self) -> np.ndarray:
        R = np.empty((self.m, self.L + 1), dtype=np.int32)
        _check(lib().nrlsh_get_rank_table(self.handle, R.ctypes.data))
        return R

    def build_stats(self) -> dict:
        st = BuildStats()
        _check(lib().nrlsh_get_build_stats(self.handle, C.byref(st)))
        return {"recomputed_items": st.recomputed_items, "recomputed_bits": st.recomputed_bits,
                "recompute_flips": st.recompute_flips, "lowp_items": st.lowp_items,
                "lowp_bits": st.lowp_bits, "lowp_changed": st.lowp_changed,
                "recompute_flips_tiny": st.recompute_flips_tiny}

    def hash_copy(self):
        """(storage name, copy in stored order n x dp, row scales or None)."""
        kind = I32()
        n, dp = self.n, self.dp
        # room for the widest element type, viewed as the storage kind afterwards
        buf = np.empty(n * dp * 4, dtype=np.uint8)
        sc = np.empty(n, dtype=np.float32)
        _check(lib().nrlsh_get_hash_copy(self.handle, buf.ctypes.data, sc.ctypes.data, C.byref(kind)))
        name = {0: "fp32", 1: "bf16", 2: "fp8"}[kind.value]
        if name == "fp32":
            return name, buf.view(np.float32).reshape(n, dp), None
        if name == "bf16":
            return name, buf[: n * dp * 2].view(np.uint16).reshape(n, dp), None
        return name, buf[: n * dp].reshape(n, dp), sc

    def query_codes(self, queries) -> np.ndarray:
        """(nq,) codes, or (nq, m) with a projection block per sub-dataset."""
        Q = _host_f32(queries)
        out = np.empty(Q.shape[0] * self.qsets, dtype=np.uint64)
        _check(lib().nrlsh_query_codes(self.handle, Q.ctypes.data, Q.shape[0], out.ctypes.data))
        return out if self.qsets == 1 else out.reshape(Q.shape[0], self.qsets)

    def bucket_table(self):
        """(ucode, ustart, uoff, titem) of an index built with bucket tables."""
        U = I64()
        _check(lib().nrlsh_get_bucket_table(self.handle, C.byref(U), None, None, None, None))
        ucode = np.empty(U.value, dtype=np.uint64)
        ustart = np.empty(U.value + 1, dtype=np.int64)
        uoff = np.empty(self.m + 1, dtype=np.int64)
        titem = np.empty(self.n, dtype=np.int32)
        _check(lib().nrlsh_get_bucket_table(self.handle, C.byref(U), ucode.ctypes.data,
                                            ustart.ctypes.data, uoff.ctypes.data, titem.ctypes.data))
        return ucode, ustart, uoff, titem

    def query_candidates(self, queries, probe_budget: int, probe: str = "scan"):
        """Probed ids per query: (nq, min(T, n)) for the scan; with probe="single"
        a list of per-query arrays (their lengths vary)."""
        Q = _host_f32(queries)
        Tq = min(int(probe_budget), self.n)
        out = np.empty((Q.shape[0], Tq), dtype=np.int64)
        if probe == "scan":
            _check(lib().nrlsh_query_candidates(self.handle, Q.ctypes.data, Q.shape[0],
                                                int(probe_budget), out.ctypes.data))
            return out
        counts = np.empty(Q.shape[0], dtype=np.int64)
        _check(lib().nrlsh_query_candidates_ex(self.handle, Q.ctypes.data, Q.shape[0], int(probe_budget),
                                               PROBES[probe], out.ctypes.data, counts.ctypes.data))
        return [out[i, :counts[i]].copy() for i in range(Q.shape[0])]

    def query_candidates_levels(self, queries, probe_budget: int):
        """Probed ids per query and each one's level l (equal code bits):
        two (nq, min(T, n)) arrays, int64 ids and int32 levels."""
        Q = _host_f32(queries)
        Tq = min(int(probe_budget), self.n)
        out = np.empty((Q.shape[0], Tq), dtype=np.int64)
        lv = np.empty((Q.shape[0], Tq), dtype=np.int32)
        _check(lib().nrlsh_query_candidates_levels(self.handle, Q.ctypes.data, Q.shape[0], int(probe_budget),
                                                   out.ctypes.data, lv.ctypes.data))
        return out, lv


# ------------------------------------------------------------------ C-ABI names
def nrlsh_build(items, m: int, L: int, seed: int, *, eps: float = 0.0, stream=None,
                hash_storage: str = "fp32", margin="rigorous", partition: str = "percentile",
                projections: str = "shared", bucket_tables: bool = False, hash_tables: int = 1) -> Index:
    """Algorithm 1.  ``items``: numpy (n, d) float32 on the host, or a CUDA torch
    tensor (n, d) float32 (device pointer, torch's current stream).
    ``hash_storage`` ("fp32", "bf16", "fp8") selects the precision form of the
    hash GEMM; ``margin`` is "rigorous" or a relative margin (float);
    ``partition`` is "percentile" (Algorithm 1) or "uniform" (Section 5);
    ``projections`` is "shared" (one matrix for all sub-datasets) or
    "per_subset" (an independent block per sub-dataset); ``bucket_tables``
    also builds the tables that probe="table" queries read; ``hash_tables``
    independent hash tables for probe="single" (multi-table single probe)."""
    h = P()
    st = STORAGES[hash_storage]
    part = PARTITIONS[partition]
    proj = PROJECTIONS[projections]
    tabs = 1 if bucket_tables else 0
    mmode, mparam = (0, 0.0) if margin == "rigorous" else (1, float(margin))
    if _is_torch_device(items):
        if items.dtype.__str__() != "torch.float32" or items.dim() != 2:
            raise ValueError("items must be a 2-D float32 tensor")
        items = items.contiguous()
        opts = BuildOpts(C.sizeof(BuildOpts), 1, stream or _torch_stream(items), float(eps), st,
                         mmode, mparam, part, proj, tabs, int(hash_tables))
        _check(lib().nrlsh_build_ex(P(items.data_ptr()), items.shape[0], items.shape[1], m, L,
                                    seed, C.byref(opts), C.byref(h)))
    else:
        X = _host_f32(items)
        if eps != 0.0 or stream is not None or st != 0 or part != 0 or proj != 0 or tabs or hash_tables != 1:
            opts = BuildOpts(C.sizeof(BuildOpts), 0, stream, float(eps), st, mmode, mparam, part,
                             proj, tabs, int(hash_tables))
            _check(lib().nrlsh_build_ex(X.ctypes.data, X.shape[0], X.shape[1], m, L, seed,
                                        C.byref(opts), C.byref(h)))
        else:
            _check(lib().nrlsh_build(X.ctypes.data, X.shape[0], X.shape[1], m, L, seed,
                                     C.byref(h)))
    return Index(h.value)


def nrlsh_query(ix: Index, queries, k: int, probe_budget: int, *, out=None, stream=None,
                rerank: str = "auto", rerank_storage: str = "fp32", probe: str = "scan",
                scan_guess: int = 0, dense_head: int = 0):
    """Multi-probe query with exact re-rank.  Returns (ids int64, ips float32),
    numpy for host queries, torch tensors for CUDA torch queries.  ``rerank``
    selects the re-rank mode ("auto", "gather", "screen", ...), ``probe`` how
    the probed items are found ("scan" or "table"), ``scan_guess`` how the scan
    finds them (0 default, -1 two passes only, g > 0 the collecting scan with a
    guess of g/16 T items), ``dense_head`` which sub-datasets the bfloat16
    re-rank screens whole (0 default, -1 none, g > 0 those expected to have at
    least g/256 of their items probed); all give the same result."""
    mode = RERANK_MODES[rerank]
    rst = STORAGES[rerank_storage]
    prb = PROBES[probe]
    if _is_torch_device(queries):
        import torch
        Q = queries.contiguous()
        nq = Q.shape[0]
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
            ips = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        else:
            ids, ips = out
        opts = QueryOpts(C.sizeof(QueryOpts), 1, stream or _torch_stream(Q), mode, rst, prb, int(scan_guess),
                         int(dense_head))
        _check(lib().nrlsh_query_ex(ix.handle, P(Q.data_ptr()), nq, k, int(probe_budget),
                                    C.byref(opts), P(ids.data_ptr()), P(ips.data_ptr())))
        return ids, ips
    Q = _host_f32(queries)
    nq = Q.shape[0]
    ids = np.empty((nq, k), dtype=np.int64)
    ips = np.empty((nq, k), dtype=np.float32)
    if mode or rst or prb or scan_guess or dense_head or stream is not None:
        opts = QueryOpts(C.sizeof(QueryOpts), 0, stream, mode, rst, prb, int(scan_guess), int(dense_head))
        _check(lib().nrlsh_query_ex(ix.handle, Q.ctypes.data, nq, k, int(probe_budget),
                                    C.byref(opts), ids.ctypes.data, ips.ctypes.data))
    else:
        _check(lib().nrlsh_query(ix.handle, Q.ctypes.data, nq, k, int(probe_budget),
                                 ids.ctypes.data, ips.ctypes.data))
    return ids, ips


def nrlsh_query_noalloc(ix: Index, queries, k: int, probe_budget: int, out, nonfinite, stream=None):
    """The query of nrlsh_query with every temporary buffer taken from the
    library's device scratch (no allocation, no copy, no synchronisation).
    ``queries``: CUDA torch tensor (nq, d) float32; ``out``: (ids int64,
    ips float32) CUDA tensors (nq, k); ``nonfinite``: a CUDA int32 tensor of one
    element, set nonzero when a query holds NaN or Inf.  Work is queued on
    ``stream`` (default: torch's current stream) and the call returns."""
    if not _is_torch_device(queries):
        raise ValueError("queries must be a CUDA tensor (device pointers only)")
    Q = queries.contiguous()
    ids, ips = out
    _check(lib().nrlsh_query_noalloc(ix.handle, P(Q.data_ptr()), Q.shape[0], k, int(probe_budget),
                                     stream or _torch_stream(Q), P(ids.data_ptr()), P(ips.data_ptr()),
                                     P(nonfinite.data_ptr())))


class MultiPlan:
    """Owns an ``nrlsh_multi_plan*``: the batching form for a fixed set of
    (index, query batch, probe budget) pairs, served by one graph of phase launches.

    ``pairs`` is a list of (Index, queries, probe_budget); the queries are all
    CUDA torch tensors (device pointers, torch's current stream) or all host
    arrays.  The plan owns one (ids, ips) output pair per entry; run() fills
    them and returns the list."""

    def __init__(self, pairs, k: int, *, use_graph: bool = True, tune: str = "table",
                 chunk: int = 0, slice: int = 0, stream=None, persistent: bool = False):
        self.k = k
        self._h = P()
        dev = [_is_torch_device(q) for _, q, _ in pairs]
        if any(dev) and not all(dev):
            raise ValueError("queries must be all device tensors or all host arrays")
        self.device = bool(dev) and all(dev)
        self._index = [ix for ix, _, _ in pairs]
        self._budget = [int(T) for _, _, T in pairs]
        self.outputs = []
        for ix, q, _ in pairs:
            nq = q.shape[0]
            if self.device:
                import torch
                self.outputs.append((torch.empty((nq, k), dtype=torch.int64, device=q.device),
                                     torch.empty((nq, k), dtype=torch.float32, device=q.device)))
            else:
                self.outputs.append((np.empty((nq, k), np.int64), np.empty((nq, k), np.float32)))
        self._descs, self._keep = self._make_descs([q for _, q, _ in pairs])
        if stream is None and self.device:
            stream = _torch_stream(pairs[0][1])
        opts = MultiOpts(C.sizeof(MultiOpts), 1 if self.device else 0, stream,
                         1 if use_graph else 0, TUNE_MODES[tune], int(chunk), int(slice),
                         1 if persistent else 0)
        _check(lib().nrlsh_multi_plan_create(self._descs, len(pairs), k, C.byref(opts),
                                             C.byref(self._h)))

    def _make_descs(self, queries):
        if len(queries) != len(self._index):
            raise ValueError(f"expected {len(self._index)} query batches, got {len(queries)}")
        arr = (QueryDesc * len(queries))()
        keep = []
        for i, (ix, q, T, (ids, ips)) in enumerate(zip(self._index, queries, self._budget,
                                                         self.outputs)):
            if self.device:
                q = q.contiguous()
                qp, ip, pp = q.data_ptr(), ids.data_ptr(), ips.data_ptr()
            else:
                q = _host_f32(q)
                qp, ip, pp = q.ctypes.data, ids.ctypes.data, ips.ctypes.data
            keep.append(q)
            if q.shape[0] and q.shape[1] != ix.d:
                raise ValueError(f"pair {i}: queries have {q.shape[1]} columns, index d = {ix.d}")
            arr[i] = QueryDesc(ix.handle.value, qp, q.shape[0], T, ip, pp)
        return arr, keep

    def run(self, queries=None):
        """Runs the plan (with new query batches of the same shapes if given)."""
        if queries is None:
            _check(lib().nrlsh_multi_run(self._h, self._descs, len(self._index)))
            return self.outputs
        descs, keep = self._make_descs(queries)
        _check(lib().nrlsh_multi_run(self._h, descs, len(self._index)))
        self._descs, self._keep = descs, keep
        return self.outputs

    def info(self) -> dict:
        inf = MultiInfo()
        n = len(self._index)
        chunk = np.zeros(n, np.int32)
        sl = np.zeros(n, np.int32)
        _check(lib().nrlsh_multi_plan_info(self._h, C.byref(inf), chunk.ctypes.data, sl.ctypes.data))
        return {"grid": inf.grid, "graph": bool(inf.graph),
                "items": dict(zip(MULTI_PHASES, list(inf.items))),
                "tuned_classes": inf.tuned_classes, "tune_ms": inf.tune_ms,
                "chunk": chunk.tolist(), "slice": sl.tolist()}

    def close(self):
        if self._h:
            lib().nrlsh_multi_plan_free(self._h)
            self._h = P()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass


def nrlsh_query_multi(pairs, k: int, **kw):
    """Batching form in one call (plan, run, free).  Returns [(ids, ips), ...]."""
    with MultiPlan(pairs, k, **kw) as plan:
        return plan.run()


def nrlsh_tune_clear():
    lib().nrlsh_tune_clear()


def nrlsh_tune_lookup(d: int, L: int, nq: int):
    """(chunk, slice) of the autotuner's table for class (d, L, nq), or None."""
    c, s = I32(), I32()
    if lib().nrlsh_tune_lookup(d, L, nq, C.byref(c), C.byref(s)):
        return c.value, s.value
    return None


def nrlsh_free(ix: Index):
    ix.close()


def nrlsh_last_error() -> str:
    return lib().nrlsh_last_error().decode(errors="replace")


def nrlsh_get_query_stats() -> dict:
    """Re-rank statistics of this thread's last query call."""
    st = QueryStats()
    _check(lib().nrlsh_get_query_stats(C.byref(st)))
    return {"mode": {1: "gather", 2: "screen", 3: "screen_fp32", 4: "screen_bf16x3"}.get(st.mode, "none"),
            "screen_passes": st.screen_passes, "kept_total": st.kept_total,
            "kept_max": st.kept_max, "theta_unset": st.theta_unset,
            "lp_kept_total": st.lp_kept_total, "lp_kept_max": st.lp_kept_max,
            "lp_fallbacks": st.lp_fallbacks, "probe": {1: "table"}.get(st.probe_mode, "scan"),
            "table_lookups": st.table_lookups, "table_walked": st.table_walked,
            "table_passes": st.table_passes, "screen_pairs": st.screen_pairs,
            "scan_pairs": st.scan_pairs, "collect_fallbacks": st.collect_fallbacks,
            "dense_head_items": st.dense_head_items, "lp_gathered_total": st.lp_gathered_total,
            "dense_head_pairs": st.dense_head_pairs}


def nrlsh_profile_enable(on: bool = True):
    lib().nrlsh_profile_enable(1 if on else 0)


def nrlsh_profile_reset():
    lib().nrlsh_profile_reset()


def nrlsh_profile_get(name: str):
    ms, n = F64(), I64()
    _check(lib().nrlsh_profile_get(name.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value
