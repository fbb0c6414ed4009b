"""ctypes wrapper around the plain-C FP64 oracle (``nrlsh_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the product library.  Every function is a
thin marshalling layer; the arithmetic lives in the C file, whose header
lists the readings of the paper that it takes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nrlsh_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-D_GNU_SOURCE"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I32, I64, U64, F64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double


def _declare(L):
    L.orc_keys.argtypes = [P, I64, I32, P]
    L.orc_rank.argtypes = [P, I64, P]
    L.orc_rank.restype = C.c_int
    L.orc_splitmix64_at.argtypes = [U64, U64]
    L.orc_splitmix64_at.restype = U64
    L.orc_box_muller.argtypes = [U64, U64]
    L.orc_box_muller.restype = F64
    L.orc_projection.argtypes = [U64, I32, I32, P]
    L.orc_partition.argtypes = [P, P, I64, I32, P, P, P]
    L.orc_transform.argtypes = [P, I32, F64, F64, F64, P]
    L.orc_hash_vec.argtypes = [P, I32, I32, P]
    L.orc_hash_vec.restype = U64
    L.orc_item_codes.argtypes = [P, I64, I64, I32, I32, P, P, P, P, P, P]
    L.orc_item_codes2.argtypes = [P, I64, I64, I32, I32, P, I32, P, P, P, P, P]
    L.orc_query_code.argtypes = [P, I32, I32, P]
    L.orc_query_code.restype = U64
    L.orc_same_bits.argtypes = [U64, U64, I32]
    L.orc_same_bits.restype = I32
    L.orc_cos_level.argtypes = [I32, I32, F64]
    L.orc_cos_level.restype = F64
    L.orc_rank_table.argtypes = [P, I32, I32, F64, P, P]
    L.orc_rank_table.restype = C.c_int
    L.orc_candidates.argtypes = [P, P, I64, I32, P, U64, I64, P, P]
    L.orc_candidates.restype = I64
    L.orc_candidates2.argtypes = [P, P, I64, I32, P, P, I32, I64, P, P]
    L.orc_candidates2.restype = I64
    L.orc_ip.argtypes = [P, P, I32]
    L.orc_ip.restype = F64
    L.orc_topk.argtypes = [P, I32, P, P, I64, I32, P, P]
    L.orc_topk.restype = C.c_int
    L.orc_build.argtypes = [P, I64, I32, I32, I32, U64, F64, I32]
    L.orc_build.restype = P
    L.orc_build2.argtypes = [P, I64, I32, I32, I32, U64, F64, I32, I32]
    L.orc_build2.restype = P
    L.orc_build3.argtypes = [P, I64, I32, I32, I32, U64, F64, I32, I32, I32]
    L.orc_build3.restype = P
    L.orc_build4.argtypes = [P, I64, I32, I32, I32, U64, F64, I32, I32, I32, I32]
    L.orc_build4.restype = P
    L.orc_candidates_mt.argtypes = [P, P, I64, I32, I32, P, I32, I64, P]
    L.orc_candidates_mt.restype = I64
    L.orc_query2.argtypes = [P, P, I64, I32, I64, I32, I32, P, P]
    L.orc_query2.restype = C.c_int
    L.orc_free.argtypes = [P]
    L.orc_index_arrays.argtypes = [P] + [C.POINTER(P)] * 8
    L.orc_query.argtypes = [P, P, I64, I32, I64, I32, P, P]
    L.orc_query.restype = C.c_int
    L.orc_bruteforce.argtypes = [P, I64, I32, P, I64, I32, I32, P, P]
    L.orc_bruteforce.restype = C.c_int


def _p(a: np.ndarray):
    return a.ctypes.data_as(P)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------- pieces
def keys(X) -> np.ndarray:
    X = _f32(X)
    n, d = X.shape
    out = np.empty(n, dtype=np.float64)
    lib().orc_keys(_p(X), n, d, _p(out))
    return out


def ranks(key) -> np.ndarray:
    key = np.ascontiguousarray(key, dtype=np.float64)
    out = np.empty(key.shape[0], dtype=np.int64)
    if lib().orc_rank(_p(key), key.shape[0], _p(out)) != 0:
        raise MemoryError("oracle rank")
    return out


def splitmix64_at(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64_at(seed, k))


def box_muller(h1: int, h2: int) -> float:
    return float(lib().orc_box_muller(h1, h2))


def projection(seed: int, L: int, d: int) -> np.ndarray:
    A = np.empty((L, d + 1), dtype=np.float32)
    lib().orc_projection(seed, L, d, _p(A))
    return A


def partition(key, rank, m: int):
    key = np.ascontiguousarray(key, dtype=np.float64)
    rank = np.ascontiguousarray(rank, dtype=np.int64)
    n = key.shape[0]
    sid = np.empty(n, dtype=np.int32)
    keymax = np.empty(m, dtype=np.float64)
    U = np.empty(m, dtype=np.float64)
    lib().orc_partition(_p(key), _p(rank), n, m, _p(sid), _p(keymax), _p(U))
    return sid, keymax, U


def transform(x, key: float, keymax: float, Uj: float) -> np.ndarray:
    x = _f32(x)
    v = np.empty(x.shape[0] + 1, dtype=np.float64)
    lib().orc_transform(_p(x), x.shape[0], key, keymax, Uj, _p(v))
    return v


def hash_vec(A, v) -> int:
    A = _f32(A)
    v = np.ascontiguousarray(v, dtype=np.float64)
    L, d1 = A.shape
    return int(lib().orc_hash_vec(_p(A), L, d1 - 1, _p(v)))


def item_codes(X, A, key, sid, keymax, U, per_subset: bool = False) -> np.ndarray:
    """Codes of all items.  per_subset: A holds m L rows and an item of
    sub-dataset j hashes with rows j L .. j L + L - 1."""
    X = _f32(X)
    A = _f32(A)
    n, d = X.shape
    m = np.asarray(U).shape[0]
    L = A.shape[0] // m if per_subset else A.shape[0]
    key = np.ascontiguousarray(key, dtype=np.float64)
    sid = np.ascontiguousarray(sid, dtype=np.int32)
    keymax = np.ascontiguousarray(keymax, dtype=np.float64)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty(n, dtype=np.uint64)
    lib().orc_item_codes2(_p(X), 0, n, d, L, _p(A), int(per_subset), _p(key), _p(sid),
                          _p(keymax), _p(U), _p(out))
    return out


def query_code(A, q) -> int:
    A = _f32(A)
    q = _f32(q)
    return int(lib().orc_query_code(_p(A), A.shape[0], A.shape[1] - 1, _p(q)))


def query_codes(A, Q) -> np.ndarray:
    Q = _f32(Q)
    return np.array([query_code(A, Q[i]) for i in range(Q.shape[0])], dtype=np.uint64)


def same_bits(a: int, b: int, L: int) -> int:
    return int(lib().orc_same_bits(a, b, L))


def cos_level(l: int, L: int, eps: float = 0.0) -> float:
    return float(lib().orc_cos_level(l, L, eps))


def rank_table(U, L: int, eps: float = 0.0):
    U = np.ascontiguousarray(U, dtype=np.float64)
    m = U.shape[0]
    R = np.empty((m, L + 1), dtype=np.int32)
    shat = np.empty((m, L + 1), dtype=np.float64)
    if lib().orc_rank_table(_p(U), m, L, eps, _p(R), _p(shat)) != 0:
        raise MemoryError("oracle rank table")
    return R, shat


def candidates(codes, sid, L: int, R, qcode, T: int):
    """First min(T, n) items by (rank of (sub-dataset, same bits), index).
    qcode: one query code, or an array of one code per sub-dataset (for
    independent projections per sub-dataset)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    sid = np.ascontiguousarray(sid, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.int32)
    n = codes.shape[0]
    Tq = min(T, n)
    cand = np.empty(max(Tq, 1), dtype=np.int64)
    ls = np.empty(max(Tq, 1), dtype=np.int32)
    if np.ndim(qcode) == 0:
        got = lib().orc_candidates(_p(codes), _p(sid), n, L, _p(R), int(qcode), T, _p(cand), _p(ls))
    else:
        qc = np.ascontiguousarray(qcode, dtype=np.uint64)
        got = lib().orc_candidates2(_p(codes), _p(sid), n, L, _p(R), _p(qc), 1, T, _p(cand), _p(ls))
    if got < 0:
        raise MemoryError("oracle candidates")
    return cand[:got], ls[:got]


def ip(q, x) -> float:
    q = _f32(q)
    x = _f32(x)
    return float(lib().orc_ip(_p(q), _p(x), q.shape[0]))


def topk(X, q, cand, k: int):
    X = _f32(X)
    q = _f32(q)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    ids = np.empty(k, dtype=np.int64)
    ips = np.empty(k, dtype=np.float64)
    if lib().orc_topk(_p(X), X.shape[1], _p(q), _p(cand), cand.shape[0], k, _p(ids), _p(ips)):
        raise MemoryError("oracle topk")
    return ids, ips


def bruteforce(X, Q, k: int, threads: int = 1):
    X = _f32(X)
    Q = _f32(Q)
    nq = Q.shape[0]
    ids = np.empty((nq, k), dtype=np.int64)
    ips = np.empty((nq, k), dtype=np.float64)
    if lib().orc_bruteforce(_p(X), X.shape[0], X.shape[1], _p(Q), nq, k, threads, _p(ids), _p(ips)):
        raise MemoryError("oracle brute force")
    return ids, ips


# ---------------------------------------------------------------- whole method
class OracleIndex:
    """Index built by the oracle (Algorithm 1).  Keeps a reference to X."""

    PARTITIONS = {"percentile": 0, "uniform": 1}
    PROJECTIONS = {"shared": 0, "per_subset": 1}

    def __init__(self, X, m: int, L: int, seed: int, eps: float = 0.0, threads: int = 1,
                 partition: str = "percentile", projections: str = "shared", tables: int = 1):
        self.X = _f32(X)
        self.n, self.d = self.X.shape
        self.m, self.L, self.seed, self.eps = m, L, seed, eps
        self.partition = partition
        self.projections = projections
        self.per_subset = self.PROJECTIONS[projections] == 1
        self.tables = tables
        self._h = lib().orc_build4(_p(self.X), self.n, self.d, m, L, seed, eps,
                                   self.PARTITIONS[partition], int(self.per_subset), tables, threads)
        if not self._h:
            raise MemoryError("oracle build")
        ptrs = [P() for _ in range(8)]
        lib().orc_index_arrays(self._h, *[C.byref(p) for p in ptrs])

        def view(p, ct, count, dt):
            buf = (ct * count).from_address(p.value)
            return np.ctypeslib.as_array(buf).view(dt).copy()

        n, d, L_ = self.n, self.d, L
        rows = (m * L_ if self.per_subset else L_) * tables
        self.A = view(ptrs[0], C.c_float, rows * (d + 1), np.float32).reshape(rows, d + 1)
        self.key = view(ptrs[1], C.c_double, n, np.float64)
        self.rank = view(ptrs[2], C.c_int64, n, np.int64)
        self.sid = view(ptrs[3], C.c_int32, n, np.int32)
        self.keymax = view(ptrs[4], C.c_double, m, np.float64)
        self.U = view(ptrs[5], C.c_double, m, np.float64)
        self.codes_t = view(ptrs[6], C.c_uint64, n * tables, np.uint64).reshape(tables, n)
        self.codes = self.codes_t[0].copy()
        self.R = view(ptrs[7], C.c_int32, m * (L_ + 1), np.int32).reshape(m, L_ + 1)

    def query(self, Q, k: int, T: int, threads: int = 1):
        Q = _f32(Q)
        nq = Q.shape[0]
        ids = np.empty((nq, k), dtype=np.int64)
        ips = np.empty((nq, k), dtype=np.float64)
        if lib().orc_query(self._h, _p(Q), nq, k, T, threads, _p(ids), _p(ips)):
            raise MemoryError("oracle query")
        return ids, ips

    def query_code(self, q, table: int = 0):
        """The query code of one table; with per-subset projections, one code
        per sub-dataset."""
        L = self.L
        P = self.m if self.per_subset else 1
        blocks = [query_code(self.A[(table * P + b) * L:(table * P + b + 1) * L], q) for b in range(P)]
        if not self.per_subset:
            return blocks[0]
        return np.array(blocks, dtype=np.uint64)

    def query_codes_all(self, q) -> np.ndarray:
        """Every table's codes, tables x P (P = m with per-subset projections, else 1)."""
        P = self.m if self.per_subset else 1
        return np.array([query_code(self.A[b * self.L:(b + 1) * self.L], q)
                         for b in range(self.tables * P)], dtype=np.uint64).reshape(self.tables, P)

    def candidates_single_probe(self, q, T: int) -> np.ndarray:
        """Multi-table single probe: the probed items of query q, in probing order."""
        qc = np.ascontiguousarray(self.query_codes_all(q).reshape(-1))
        cand = np.empty(self.n, dtype=np.int64)
        codes = np.ascontiguousarray(self.codes_t)
        nc = lib().orc_candidates_mt(_p(codes), _p(self.sid), self.n, self.m, self.tables, _p(qc),
                                     int(self.per_subset), T, _p(cand))
        if nc < 0:
            raise MemoryError("oracle candidates")
        return cand[:nc]

    def query_single_probe(self, Q, k: int, T: int, threads: int = 1):
        Q = _f32(Q)
        nq = Q.shape[0]
        ids = np.empty((nq, k), dtype=np.int64)
        ips = np.empty((nq, k), dtype=np.float64)
        if lib().orc_query2(self._h, _p(Q), nq, k, T, 1, threads, _p(ids), _p(ips)):
            raise MemoryError("oracle query")
        return ids, ips

    def candidates(self, q, T: int):
        return candidates(self.codes, self.sid, self.L, self.R, self.query_code(q), T)

    def close(self):
        if self._h:
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
