"""Precision form of the hash GEMM (BF16 / FP8 E4M3 storage on the matrix
cores): rounding of the stored copies, sign parity with the FP64 oracle under
the rigorous margin, and the flips left by a scaled margin."""
import math

import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ definitions
def e4m3_value(code: int) -> float:
    """OCP E4M3: sign, 4-bit exponent (bias 7), 3-bit mantissa; subnormals
    m 2^-9; 0x7F / 0xFF are NaN."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 7
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def bf16_value(code: int) -> float:
    return float(np.array([code << 16], dtype=np.uint32).view(np.float32)[0])


def _stored_rows(ix, X):
    perm, _ = ix.layout()
    name, copy, scales = ix.hash_copy()
    out = np.empty_like(copy[:, : X.shape[1]])
    out[perm] = copy[:, : X.shape[1]]
    sc = None
    if scales is not None:
        sc = np.empty_like(scales)
        sc[perm] = scales
    return name, out, sc


def test_fp8_copy_rounds_to_nearest_even():
    """Every finite E4M3 value maps to its own code and midpoints between
    neighbours go to the even code (the row scale max|x| / 448 is fixed at 1 by
    a 448 in every row, so values above 448 cannot occur)."""
    say("case fp8 rounding")
    finite = [c for c in range(256) if (c & 0x7F) != 0x7F]
    vals, want = [], []
    for c in finite:
        vals.append(e4m3_value(c))
        want.append(c)
    pos = sorted(c for c in finite if c < 0x80)
    for a, b in zip(pos[:-1], pos[1:]):  # midpoints of adjacent positive codes
        mid = (e4m3_value(a) + e4m3_value(b)) / 2.0
        even = a if (a & 1) == 0 else b
        vals += [mid, -mid]
        want += [even, even | 0x80]
    d = 64
    nrow = -(-len(vals) // (d - 1))
    X = np.zeros((nrow, d), np.float32)
    flat = np.zeros(nrow * (d - 1), np.float32)
    flat[: len(vals)] = vals
    X[:, 1:] = flat.reshape(nrow, d - 1)
    X[:, 0] = 448.0
    with nr.nrlsh_build(X, 1, 8, 1, hash_storage="fp8") as ix:
        name, q, sc = _stored_rows(ix, X)
    assert name == "fp8"
    assert np.all(sc == 1.0)
    got = q[:, 1:].reshape(-1)[: len(vals)]
    bad = [(v, w, g) for v, w, g in zip(vals, want, got) if w != g and not (v == 0.0 and w & 0x7F == 0 and g & 0x7F == 0)]
    assert bad == [], bad[:10]


def test_bf16_copy_rounds_to_nearest_even():
    say("case bf16 rounding")
    rng = np.random.default_rng(1)
    codes = rng.integers(0, 0x7F7F, size=4000).astype(np.int64)
    lo = np.array([bf16_value(int(c)) for c in codes])
    hi = np.array([bf16_value(int(c) + 1) for c in codes])
    mids = ((lo + hi) / 2).astype(np.float32)           # exact ties -> even code
    want_mid = np.where(codes % 2 == 0, codes, codes + 1)
    near = (lo + (hi - lo) * 0.3).astype(np.float32)   # below the tie -> lower code
    vals = np.concatenate([mids, near, -mids])
    want = np.concatenate([want_mid, codes, want_mid | 0x8000])
    d = 80
    nrow = -(-len(vals) // d)
    flat = np.zeros(nrow * d, np.float32)
    flat[: len(vals)] = vals
    X = flat.reshape(nrow, d)
    with nr.nrlsh_build(X, 1, 8, 1, hash_storage="bf16") as ix:
        name, q, _ = _stored_rows(ix, X)
    assert name == "bf16"
    got = q.reshape(-1)[: len(vals)].astype(np.int64)
    assert np.array_equal(got, want)


SHAPES = [
    (3000, 75, 7, 32),
    (5000, 150, 16, 64),
    (2000, 33, 3, 16),
    (1024, 128, 8, 63),
    (700, 8, 1, 20),
]


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_d%d_m%d_L%d" % s)
def test_rigorous_margin_matches_fp64_signs(storage, shape):
    n, d, m, L = shape
    say(f"case rigorous {storage} n={n} d={d} m={m} L={L}")
    X = make_items("pareto", n, d, seed=n + d, alpha=2.5)
    Q = make_queries(40, d, seed=n + 1)
    oix = orc.OracleIndex(X, m, L, seed=29, threads=8)
    with nr.nrlsh_build(X, m, L, 29, hash_storage=storage) as gix:
        codes = gix.codes()
        st = gix.build_stats()
        say(f"  {storage}: bits in margin {st['lowp_bits']}/{n * L}; items re-hashed whole "
            f"{st['lowp_items']}/{n} ({st['lowp_changed']} bits changed); bits recomputed in FP64 "
            f"{st['recomputed_bits']} on {st['recomputed_items']} items ({st['recompute_flips']} flips)")
        assert np.array_equal(codes, oix.codes)
        # every in-margin bit went through an exact recheck: either its item
        # was re-hashed whole, or the bit itself was recomputed in FP64
        assert st["lowp_bits"] > 0
        assert st["lowp_items"] * L + st["recomputed_bits"] >= st["lowp_bits"]
        ids, ips = nr.nrlsh_query(gix, Q, 10, max(50, n // 20))
        oids, oips = oix.query(Q, 10, max(50, n // 20))
        assert np.array_equal(ids, oids)
        assert np.array_equal(ips, oips.astype(np.float32))


def _qrel(storage, d):
    gd = d * 2.0 ** -24 / (1 - d * 2.0 ** -24)
    if storage == "fp8":
        return (2 ** -3 + 2 ** -8 + 2 ** -20 + 2 ** -21 + 2 ** -10 * 2.2 * math.sqrt(d) / 448
                + 2 ** -20 * d / 448 ** 2 + 2.2 * gd)
    return 2 ** -7 + 2 ** -16 + 2 ** -21 + 2.2 * gd


@pytest.mark.parametrize("storage,margin", [("bf16", 1e-3), ("fp8", 1e-3), ("bf16", 1.5e-2), ("fp8", 0.25)])
def test_scaled_margin_flips_stay_within_quantisation_bound(storage, margin):
    """A scaled margin may leave sign flips against FP64; each must be a bit
    whose exact scaled projection lies within the worst-case quantisation
    error (the rigorous margin), i.e. the rounding analysis holds."""
    n, d, m, L = 6000, 150, 16, 64
    say(f"case scaled {storage} margin={margin}")
    X = make_items("pareto", n, d, seed=77, alpha=2.5)
    oix = orc.OracleIndex(X, m, L, seed=31, threads=8)
    with nr.nrlsh_build(X, m, L, 31, hash_storage=storage, margin=margin) as gix:
        codes = gix.codes()
        st = gix.build_stats()
    diff = codes ^ oix.codes
    items = np.flatnonzero(diff)
    nflip = int(sum(bin(int(v)).count("1") for v in diff[items]))
    say(f"  {storage} margin {margin}: {nflip} flipped bits of {n * L} ({nflip / (n * L):.2e}), "
        f"re-hashed items {st['lowp_items']}, bits in margin {st['lowp_bits']}")
    A = oix.A.astype(np.float64)
    anorm = np.sqrt((A[:, :d] ** 2).sum(axis=1))
    a_all = np.sqrt((A ** 2).sum(axis=1))
    q = _qrel(storage, d) * (1 + 2 ** -10)
    tau = 2 * ((d + 3) * 2.0 ** -24 / (1 - (d + 3) * 2.0 ** -24)) * a_all
    for i in items:
        s = oix.sid[i]
        v = orc.transform(X[i], oix.key[i], oix.keymax[s], oix.U[s])
        for r in range(L):
            if (int(diff[i]) >> r) & 1:
                p = oix.U[s] * float(A[r] @ v)
                bound = q * anorm[r] * math.sqrt(oix.key[i]) + tau[r] * oix.U[s]
                assert abs(p) <= bound * 1.01, (i, r, p, bound)
    assert nflip <= 0.05 * n * L


@pytest.mark.parametrize("k,T", [(10, 3000), (100, 2500), (10, 9000)])
def test_bf16_rerank_copy_gives_exact_topk(k, T):
    """Gather re-rank from the bfloat16 copy with bounds, then an exact FP64
    re-rank of the items that may still reach the top-k: the oracle's result."""
    n, d = 9000, 128
    say(f"case bf16 rerank k={k} T={T}")
    X = make_items("lognormal", n, d, seed=91, sigma=1.0)
    Q = make_queries(150, d, seed=92)
    oix = orc.OracleIndex(X, 16, 64, seed=33, threads=8)
    oids, oips = oix.query(Q, k, T, threads=8)
    with nr.nrlsh_build(X, 16, 64, 33) as gix:
        ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage="bf16")
        st = nr.nrlsh_get_query_stats()
        say(f"  exact re-rank lists: total {st['lp_kept_total']} max {st['lp_kept_max']} "
            f"fallbacks {st['lp_fallbacks']}")
        assert np.array_equal(ids, oids)
        assert np.array_equal(ips, oips.astype(np.float32))
        assert st["lp_kept_total"] > 0 and st["lp_fallbacks"] == 0


def test_bf16_rerank_overflow_is_remembered_per_index():
    """Nearly equal rows keep every item inside the bfloat16 bound, so the
    short lists overflow: the batch falls back to the FP32 rows, later calls
    with at least that k and budget skip the bfloat16 pass, smaller budgets
    still take it; every call returns the oracle's result."""
    say("case bf16 rerank overflow hint")
    rng = np.random.default_rng(5)
    n, d = 20000, 16
    X = (1.0 + 1e-4 * rng.standard_normal((n, d))).astype(np.float32)
    Q = make_queries(30, d, seed=6)
    oix = orc.OracleIndex(X, 4, 16, seed=7, threads=8)
    with nr.nrlsh_build(X, 4, 16, 7) as gix:
        for T, expect in ((n, "fallback"), (n, "skipped"), (4096, "bf16")):
            oids, oips = oix.query(Q, 10, T, threads=8)
            ids, ips = nr.nrlsh_query(gix, Q, 10, T, rerank="gather", rerank_storage="bf16")
            st = nr.nrlsh_get_query_stats()
            say(f"  T={T}: kept {st['lp_kept_total']} fallbacks {st['lp_fallbacks']}")
            assert np.array_equal(ids, oids), T
            assert np.array_equal(ips, oips.astype(np.float32)), T
            if expect == "fallback":
                assert st["lp_fallbacks"] >= 1
            elif expect == "skipped":
                assert st["lp_fallbacks"] == 0 and st["lp_kept_total"] == 0
            else:
                assert st["lp_fallbacks"] == 0 and st["lp_kept_total"] > 0
