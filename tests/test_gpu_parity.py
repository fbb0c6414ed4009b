"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle,
step by step, on seeded inputs spanning several tiles and ragged tails, plus
the degenerate cases of the method."""
import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import check_build, check_query, say
from workloads import make_items, make_queries, tiny

pytestmark = pytest.mark.gpu

# (n, d, m, L, nq, k, T): tiles of 64 rows / 16 hash bits / 32 coordinates,
# with ragged tails in every dimension; m = 1 (SimpleLSH), m = n, n = 1, d = 1
SHAPES = [
    (1000, 16, 4, 16, 70, 10, 100),
    (3001, 33, 7, 31, 65, 10, 257),
    (4097, 64, 8, 32, 130, 7, 1000),
    (2500, 130, 16, 33, 64, 10, 300),
    (5000, 75, 13, 64, 100, 100, 700),
    (777, 8, 1, 17, 33, 5, 50),
    (64, 5, 64, 8, 10, 3, 20),
    (1, 3, 1, 5, 4, 2, 1),
    (300, 1, 3, 12, 20, 4, 30),
    (2049, 300, 32, 32, 65, 10, 200),
    (999, 150, 9, 1, 40, 10, 99),
    (1500, 40, 6, 63, 40, 64, 1500),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_d%d_m%d_L%d" % s[:4])
def test_parity_shapes(shape):
    n, d, m, L, nq, k, T = shape
    say(f"case n={n} d={d} m={m} L={L} nq={nq} k={k} T={T}")
    X = make_items("lognormal", n, d, seed=n + d, sigma=0.9)
    Q = make_queries(nq, d, seed=n + 7)
    oix = orc.OracleIndex(X, m, L, seed=1234 + L, threads=8)
    with nr.nrlsh_build(X, m, L, 1234 + L) as gix:
        check_build(gix, oix, f"n{n}")
        check_query(gix, oix, Q, k, T, f"n{n}")
        # budgets around the edges: smaller than k, exactly n, above n
        for TT in (1, max(1, k - 1), n, n + 5):
            ids, _ = nr.nrlsh_query(gix, Q[:8], k, TT)
            oids, _ = oix.query(Q[:8], k, TT)
            assert np.array_equal(ids, oids), f"T={TT}"


@pytest.mark.parametrize("k", [10, 100])
def test_parity_large_budget_split_rerank(k):
    """Budgets above 1024 with few queries split each probed list across waves."""
    say(f"case split rerank k={k}")
    n, d = 20000, 40
    X = make_items("lognormal", n, d, seed=51, sigma=1.0)
    Q = make_queries(9, d, seed=52)
    oix = orc.OracleIndex(X, 16, 32, seed=13, threads=8)
    with nr.nrlsh_build(X, 16, 32, 13) as gix:
        for T in (3000, 17777, n):
            ids, ips = nr.nrlsh_query(gix, Q, k, T)
            oids, oips = oix.query(Q, k, T)
            assert np.array_equal(ids, oids), f"T={T}"
            assert np.array_equal(ips, oips.astype(np.float32)), f"T={T}"


SCREEN_CASES = [
    # (n, d, m, L, nq, k, T)
    (20000, 64, 8, 32, 150, 10, 20000),     # T = n: every item probed
    (30011, 75, 16, 32, 130, 10, 4000),     # T < n: predicate with a cut bucket
    (25000, 128, 32, 64, 64, 100, 25000),   # L = 64, k = 100
    (12000, 300, 13, 17, 200, 16, 5000),    # d = 300, ragged L
    (9000, 33, 1, 20, 70, 10, 3000),        # m = 1
    (7000, 8, 4, 16, 65, 64, 6999),         # small d, T = n - 1
    (15000, 260, 12, 32, 300, 10, 15000),   # d_p >= 256, T = n: 128-query tiles, last one ragged
]


@pytest.mark.parametrize("case", SCREEN_CASES, ids=lambda c: "n%d_d%d_m%d_L%d_T%d" % (c[0], c[1], c[2], c[3], c[6]))
def test_parity_screen_rerank(case):
    """Every query-tiled matrix-core screen (bf16, FP32, bf16x3) followed by the
    FP64 re-rank gives the oracle's top-k; T = n takes the all-probed path."""
    n, d, m, L, nq, k, T = case
    say(f"case screen n={n} d={d} m={m} L={L} nq={nq} k={k} T={T}")
    X = make_items("lognormal", n, d, seed=n + 3, sigma=0.9)
    Q = make_queries(nq, d, seed=n + 4)
    oix = orc.OracleIndex(X, m, L, seed=17, threads=8)
    with nr.nrlsh_build(X, m, L, 17) as gix:
        oids, oips = oix.query(Q, k, T, threads=8)
        for mode in ("screen", "screen_fp32", "screen_bf16x3", "gather"):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank=mode)
            st = nr.nrlsh_get_query_stats()
            assert st["mode"] == mode, st
            assert np.array_equal(ids, oids), mode
            assert np.array_equal(ips, oips.astype(np.float32)), mode


def test_screen_with_duplicates_and_zero_rows():
    say("case screen duplicates")
    n, d = 8000, 24
    X = make_items("lognormal", n, d, seed=71, sigma=0.7)
    X[100:900] = 0.0
    X[2000:2100] = X[5000]
    Q = make_queries(80, d, seed=72)
    Q[5] = X[5000] / np.linalg.norm(X[5000])
    Q[6] = 0.0
    oix = orc.OracleIndex(X, 10, 32, seed=5, threads=8)
    with nr.nrlsh_build(X, 10, 32, 5) as gix:
        for T in (3000, n):
            oids, oips = oix.query(Q, 10, T, threads=8)
            for mode in ("screen", "screen_fp32", "screen_bf16x3"):
                ids, ips = nr.nrlsh_query(gix, Q, 10, T, rerank=mode)
                assert np.array_equal(ids, oids), f"T={T} {mode}"
                assert np.array_equal(ips, oips.astype(np.float32)), f"T={T} {mode}"


# dimensions around the norm keys' 32-column chunks (taken in pairs, so an
# odd chunk count ends with a chunk wholly past d) and the hash's 16-coordinate
# steps (also paired; d_p = d rounded up to 8), for each load width the keys
# use (d % 4 == 0, d % 2 == 0, odd)
CHUNK_DIMS = [1, 2, 3, 4, 6, 8, 24, 31, 32, 33, 62, 63, 64, 65, 96, 98, 120, 136, 161]


@pytest.mark.parametrize("d", CHUNK_DIMS)
def test_build_chunk_boundaries(d):
    n = 333
    say(f"case build chunk boundaries n={n} d={d}")
    X = make_items("lognormal", n, d, seed=1000 + d, sigma=0.8)
    oix = orc.OracleIndex(X, 5, 20, seed=31 + d, threads=8)
    with nr.nrlsh_build(X, 5, 20, 31 + d) as gix:
        check_build(gix, oix, f"d{d}")


def test_parity_tiny_config():
    """The small recipe end to end: n = 1e4, d = 64, m = 8, L = 16, 100 queries,
    top-10, budget 500."""
    w = tiny()
    say("case tiny config")
    X, Q = w.items(), w.queries()
    oix = orc.OracleIndex(X, w.m, w.L, seed=w.index_seed, threads=8)
    with nr.nrlsh_build(X, w.m, w.L, w.index_seed) as gix:
        check_build(gix, oix, "tiny")
        check_query(gix, oix, Q, w.k, w.budgets[0], "tiny")


def test_edge_duplicates_zero_rows_zero_query():
    say("case duplicates / zero rows / zero query")
    n, d = 1200, 24
    X = make_items("lognormal", n, d, seed=5, sigma=0.7)
    X[100:400] = 0.0            # all-zero rows: the lowest sub-datasets get U_j = 0
    X[500:520] = X[600]         # duplicate rows (equal keys, ties broken by index)
    X[700] = X[701] = X[702] = X[900]
    Q = make_queries(20, d, seed=6)
    Q[3] = 0.0                  # zero query: all-zero code, all inner products 0
    Q[4] = X[600] / np.linalg.norm(X[600])
    oix = orc.OracleIndex(X, 10, 32, seed=77, threads=8)
    assert oix.U[0] == 0.0
    with nr.nrlsh_build(X, 10, 32, 77) as gix:
        check_build(gix, oix, "edge")
        check_query(gix, oix, Q, 10, 150, "edge")
        check_query(gix, oix, Q, 10, n, "edge-full")


def test_edge_extreme_magnitudes():
    """Sub-datasets with U_j far below 2^-60 or above 2^60 take the FP64 path."""
    say("case extreme magnitudes")
    n, d = 900, 12
    X = make_items("lognormal", n, d, seed=9, sigma=0.5)
    X[:300] *= np.float32(1e-25)
    X[600:] *= np.float32(1e25)
    Q = make_queries(16, d, seed=10)
    oix = orc.OracleIndex(X, 3, 20, seed=3, threads=8)
    with nr.nrlsh_build(X, 3, 20, 3) as gix:
        st = check_build(gix, oix, "extreme")
        assert st["recomputed_items"] >= 600
        check_query(gix, oix, Q, 10, 100, "extreme")


def test_all_equal_norms():
    """Equal norms: every sub-dataset has the same U_j (Section 3.2 remark)."""
    say("case equal norms")
    rng = np.random.default_rng(3)
    base = np.array([3, -1, 2, 0, 5, -4, 1, 1], dtype=np.float32)
    X = np.stack([rng.permutation(base) * rng.choice([-1, 1], size=8) for _ in range(640)])
    X = X.astype(np.float32)
    Q = make_queries(12, 8, seed=4)
    oix = orc.OracleIndex(X, 8, 16, seed=8, threads=8)
    with nr.nrlsh_build(X, 8, 16, 8) as gix:
        check_build(gix, oix, "equal")
        check_query(gix, oix, Q, 10, 64, "equal")


@pytest.mark.parametrize("eps", [0.1, 0.25])
def test_adjusted_metric(eps):
    """Adjusted similarity metric with eps > 0 (Section 3.3)."""
    say(f"case eps={eps}")
    X = make_items("lognormal", 4000, 32, seed=21, sigma=0.8)
    Q = make_queries(70, 32, seed=22)
    oix = orc.OracleIndex(X, 8, 16, seed=5, eps=eps, threads=8)
    with nr.nrlsh_build(X, 8, 16, 5, eps=eps) as gix:
        check_build(gix, oix, f"eps{eps}")
        check_query(gix, oix, Q, 10, 400, f"eps{eps}")


def test_non_finite_inputs_rejected():
    say("case non-finite")
    X = make_items("lognormal", 100, 4, seed=1)
    X[17, 2] = np.nan
    with pytest.raises(nr.NrlshError) as e:
        nr.nrlsh_build(X, 2, 8, 1)
    assert e.value.status == 2
    X[17, 2] = 1.0
    with nr.nrlsh_build(X, 2, 8, 1) as gix:
        Q = make_queries(3, 4, seed=2)
        Q[1, 0] = np.inf
        with pytest.raises(nr.NrlshError) as e:
            nr.nrlsh_query(gix, Q, 3, 10)
        assert e.value.status == 2
        # a budget covering every item skips the query hash: the other
        # query passes must still catch it, in every re-rank mode
        for mode in ("screen", "screen_fp32", "screen_bf16x3", "gather"):
            with pytest.raises(nr.NrlshError) as e:
                nr.nrlsh_query(gix, Q, 3, 100, rerank=mode)
            assert e.value.status == 2, mode


def test_deterministic_and_batch_independent():
    say("case determinism")
    X = make_items("lognormal", 6000, 48, seed=31, sigma=1.0)
    Q = make_queries(300, 48, seed=32)
    with nr.nrlsh_build(X, 12, 32, 9) as a, nr.nrlsh_build(X, 12, 32, 9) as b:
        assert np.array_equal(a.codes(), b.codes())
        i1, p1 = nr.nrlsh_query(a, Q, 10, 600)
        i2, p2 = nr.nrlsh_query(b, Q, 10, 600)
        assert np.array_equal(i1, i2) and np.array_equal(p1, p2)
        parts = [nr.nrlsh_query(a, Q[s:e], 10, 600) for s, e in ((0, 1), (1, 64), (64, 199), (199, 300))]
        assert np.array_equal(np.concatenate([p[0] for p in parts]), i1)
        assert np.array_equal(np.concatenate([p[1] for p in parts]), p1)


def test_device_pointer_path_matches_host_path():
    """The _ex entry points on torch device tensors give the host-path results."""
    import torch
    say("case device pointers")
    X = make_items("lognormal", 5000, 64, seed=41, sigma=0.6)
    Q = make_queries(200, 64, seed=42)
    with nr.nrlsh_build(X, 8, 32, 11) as h:
        ih, ph = nr.nrlsh_query(h, Q, 10, 500)
        hc = h.codes()
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    with nr.nrlsh_build(Xd, 8, 32, 11) as g:
        assert np.array_equal(g.codes(), hc)
        idd, ipd = nr.nrlsh_query(g, Qd, 10, 500)
        torch.cuda.synchronize()
        assert np.array_equal(idd.cpu().numpy(), ih)
        assert np.array_equal(ipd.cpu().numpy(), ph)


def test_build_returns_before_its_last_kernels():
    """nrlsh_build returns once the caller's items are read: the items may be
    overwritten at once on another stream, and a query on a third stream, the
    build counters and the inspection calls all see the finished index."""
    import torch
    say("case asynchronous build end")
    X = make_items("lognormal", 20000, 96, seed=43, sigma=0.8)
    Q = make_queries(300, 96, seed=44)
    with nr.nrlsh_build(X, 16, 32, 17) as h:
        ih, ph = nr.nrlsh_query(h, Q, 10, 2000)
        hc = h.codes()
        hst = h.build_stats()
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    sa, sb, sc = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(2):
        Xc = Xd.clone()
        torch.cuda.synchronize()
        g = nr.nrlsh_build(Xc, 16, 32, 17, stream=sa.cuda_stream)
        with torch.cuda.stream(sb):
            Xc.fill_(float("nan"))  # the caller reuses its items right away
        with torch.cuda.stream(sc):
            idd, ipd = nr.nrlsh_query(g, Qd, 10, 2000, stream=sc.cuda_stream)
        sc.synchronize()
        assert np.array_equal(idd.cpu().numpy(), ih), f"rep {rep}"
        assert np.array_equal(ipd.cpu().numpy(), ph), f"rep {rep}"
        assert g.build_stats() == hst
        assert np.array_equal(g.codes(), hc)
        g.close()
    torch.cuda.synchronize()


UNIFORM_CASES = [
    # (n, d, m, L, kind, T)
    (6000, 40, 16, 32, "lognormal", 600),
    (5000, 64, 32, 64, "pareto", 5000),   # heavy tail: many empty ranges
    (3000, 17, 1, 20, "lognormal", 300),
    (4096, 128, 7, 31, "lowrank", 1000),
]


@pytest.mark.parametrize("case", UNIFORM_CASES, ids=lambda c: "n%d_d%d_m%d_L%d_%s" % c[:5])
def test_parity_uniform_partition(case):
    """Section 5's uniform norm ranges: partition (including empty ranges),
    codes, rank table and query results equal the oracle's."""
    n, d, m, L, kind, T = case
    say(f"case uniform n={n} d={d} m={m} L={L} {kind}")
    kw = {"alpha": 2.5} if kind == "pareto" else {"sigma": 1.0} if kind == "lognormal" else {}
    X = make_items(kind, n, d, seed=n + m, **kw)
    Q = make_queries(90, d, seed=n + 1)
    oix = orc.OracleIndex(X, m, L, seed=23, threads=8, partition="uniform")
    with nr.nrlsh_build(X, m, L, 23, partition="uniform") as gix:
        sid, keymax, U = gix.partition()
        say(f"  empty ranges: {int((np.bincount(oix.sid, minlength=m) == 0).sum())} of {m}")
        check_build(gix, oix, "uniform")
        check_query(gix, oix, Q, 10, T, "uniform")
        for mode in ("screen", "gather"):
            ids, ips = nr.nrlsh_query(gix, Q, 10, n, rerank=mode)
            oids, oips = oix.query(Q, 10, n, threads=8)
            assert np.array_equal(ids, oids), mode


def test_uniform_partition_equal_norms():
    """Every item has the same norm: all of them fall in the last range."""
    say("case uniform equal norms")
    X = make_queries(500, 12, seed=3) * 2.0  # unit rows scaled by 2
    oix = orc.OracleIndex(X, 5, 16, 9, threads=4, partition="uniform")
    with nr.nrlsh_build(X, 5, 16, 9, partition="uniform") as gix:
        check_build(gix, oix, "equal norms")
        check_query(gix, oix, make_queries(20, 12, seed=4), 5, 100, "equal norms")


@pytest.mark.parametrize("n,d,m,L,nq,k,T", [
    (30011, 75, 4, 32, 70, 10, 3001),     # 2 tiles x 4 sub-datasets: chunked scans
    (40000, 33, 2, 48, 5, 100, 17777),    # W = 2, one tile, threshold bucket cut across chunks
    (25000, 64, 3, 16, 130, 10, 25000),   # T = n
])
def test_parity_small_batch_chunked_scan(n, d, m, L, nq, k, T):
    """Small batches over large sub-datasets take the chunked scans (appends
    in any order, threshold bucket cut by stored position); the probed set
    and the results equal the oracle's, also with the bfloat16 re-rank copy."""
    say(f"case chunked scan n={n} d={d} m={m} L={L} nq={nq} k={k} T={T}")
    X = make_items("lognormal", n, d, seed=n + 11, sigma=0.9)
    Q = make_queries(nq, d, seed=n + 12)
    oix = orc.OracleIndex(X, m, L, seed=41, threads=8)
    oids, oips = oix.query(Q, k, T, threads=8)
    with nr.nrlsh_build(X, m, L, 41) as gix:
        for storage in ("fp32", "bf16"):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage=storage)
            assert np.array_equal(ids, oids), storage
            assert np.array_equal(ips, oips.astype(np.float32)), storage
            if storage == "bf16":
                st = nr.nrlsh_get_query_stats()
                say(f"  bf16 lists: total {st['lp_kept_total']} max {st['lp_kept_max']} "
                    f"fallbacks {st['lp_fallbacks']}")


PER_SUBSET_CASES = [
    # (n, d, m, L, kind, T, partition)
    (6000, 40, 16, 32, "lognormal", 600, "percentile"),
    (5000, 64, 8, 64, "pareto", 5000, "percentile"),     # W = 2, T = n
    (3000, 17, 1, 20, "lognormal", 300, "percentile"),   # one sub-dataset: the shared index
    (4100, 128, 7, 31, "lowrank", 1000, "percentile"),   # sub-datasets cut hash blocks raggedly
    (5000, 64, 32, 48, "pareto", 2000, "uniform"),       # empty sub-datasets own no hash block
]


@pytest.mark.parametrize("case", PER_SUBSET_CASES, ids=lambda c: "n%d_d%d_m%d_L%d_%s_T%d_%s" % c)
def test_parity_per_subset_projections(case):
    """Independent projections per sub-dataset: projection blocks, item codes
    (each sub-dataset hashed with its own rows), the m query codes, probed sets
    and results equal the oracle's, for every re-rank mode."""
    n, d, m, L, kind, T, part = case
    say(f"case per-subset projections n={n} d={d} m={m} L={L} {kind} T={T} {part}")
    kw = {"alpha": 2.5} if kind == "pareto" else {"sigma": 1.0} if kind == "lognormal" else {}
    X = make_items(kind, n, d, seed=n + 3 * m, **kw)
    Q = make_queries(70, d, seed=n + 5)
    oix = orc.OracleIndex(X, m, L, seed=29, threads=8, partition=part, projections="per_subset")
    with nr.nrlsh_build(X, m, L, 29, partition=part, projections="per_subset") as gix:
        assert gix.qsets == m
        check_build(gix, oix, "per-subset")
        check_query(gix, oix, Q, 10, T, "per-subset")
        oids, oips = oix.query(Q, 10, n, threads=8)
        for mode in ("gather", "screen", "screen_fp32", "screen_bf16x3"):
            ids, ips = nr.nrlsh_query(gix, Q, 10, n, rerank=mode)
            assert np.array_equal(ids, oids), mode
            assert np.array_equal(ips, oips.astype(np.float32)), mode


def test_parity_per_subset_small_batch_chunked_scan():
    """Per-subset query codes through the chunked scans and the tie cut."""
    n, d, m, L, nq, k, T = 30011, 75, 4, 32, 70, 10, 3001
    say(f"case per-subset chunked scan n={n} d={d} m={m} L={L} nq={nq} T={T}")
    X = make_items("lognormal", n, d, seed=n + 13, sigma=0.9)
    Q = make_queries(nq, d, seed=n + 14)
    oix = orc.OracleIndex(X, m, L, seed=43, threads=8, projections="per_subset")
    oids, oips = oix.query(Q, k, T, threads=8)
    with nr.nrlsh_build(X, m, L, 43, projections="per_subset") as gix:
        cand = gix.query_candidates(Q[:8], T)
        for qi in range(8):
            assert np.array_equal(np.sort(cand[qi]), np.sort(oix.candidates(Q[qi], T)[0])), qi
        for storage in ("fp32", "bf16"):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage=storage)
            assert np.array_equal(ids, oids), storage
            assert np.array_equal(ips, oips.astype(np.float32)), storage


def test_per_subset_index_rejected_by_batching_form():
    X = make_items("lognormal", 2000, 16, seed=5, sigma=0.5)
    Q = make_queries(4, 16, seed=6)
    with nr.nrlsh_build(X, 4, 16, 7, projections="per_subset") as gix:
        with pytest.raises(nr.NrlshError, match="per-subset"):
            nr.nrlsh_query_multi([(gix, Q, 100)], 10)


@pytest.mark.parametrize("mode", ["screen", "screen_bf16x3"])
def test_screen_norm_pruning_keeps_exact_result(mode):
    """Heavy-tailed norms: the keep pass skips every chunk whose sub-dataset's
    largest norm cannot reach any tile query's theta (Cauchy-Schwarz), yet the
    result equals the oracle's exact top-k at T = n and at a smaller budget."""
    n, d, m, L = 30000, 64, 16, 32
    say(f"case screen norm pruning {mode}")
    X = make_items("pareto", n, d, seed=71, alpha=2.0)
    Q = make_queries(200, d, seed=72)
    oix = orc.OracleIndex(X, m, L, seed=73, threads=8)
    with nr.nrlsh_build(X, m, L, 73) as gix:
        for T in (n, 3000):
            oids, oips = oix.query(Q, 10, T, threads=8)
            ids, ips = nr.nrlsh_query(gix, Q, 10, T, rerank=mode)
            st = nr.nrlsh_get_query_stats()
            say(f"  T={T}: pairs evaluated {st['screen_pairs']} of {Q.shape[0] * n}")
            assert np.array_equal(ids, oids), T
            assert np.array_equal(ips, oips.astype(np.float32)), T
            if T == n:
                assert 0 < st["screen_pairs"] < Q.shape[0] * n


def _midpoint_case():
    """Two items whose bfloat16 roundings move their inner products with the
    query in opposite directions by the full unit roundoff of both operands:
    the query's first 32 coordinates lie just below a rounding midpoint
    (rounded down by almost 2^-8), its last 32 just above one (rounded up),
    item A sits on the first group and item B on the second.  A's exact inner
    product is the larger (by about 1e-3), B's bfloat16 one the larger (by
    about 0.5): a bound that counted only one operand's rounding would place
    B's lower bound above A's upper bound and return B."""
    d = 64
    lo = np.float32(1 + 2 ** -8 - 2 ** -20)  # bfloat16 rounds it down to 1
    hi = np.float32(1 + 2 ** -8 + 2 ** -20)  # bfloat16 rounds it up to 1 + 2^-7
    q = np.concatenate([np.full(32, lo), np.full(32, hi)]).astype(np.float32)
    a = np.concatenate([np.full(32, lo), np.zeros(32)]).astype(np.float32)
    b = np.concatenate([np.zeros(32), np.full(32, hi)]).astype(np.float32)
    ip_a = float(np.dot(q.astype(np.float64), a.astype(np.float64)))
    rest = float(np.dot(q[32:63].astype(np.float64), b[32:63].astype(np.float64)))
    b[63] = np.float32((ip_a - rest) / float(hi) - 1e-3)
    filler = make_items("lognormal", 998, d, seed=91, sigma=0.3) * np.float32(0.05)
    X = np.concatenate([filler[:500], a[None], filler[500:], b[None]]).astype(np.float32)
    Q = np.stack([q, q * np.float32(0.5), q * np.float32(4.0)]).astype(np.float32)
    return X, Q, 500, X.shape[0] - 1


def test_screen_bound_at_bf16_rounding_midpoints():
    X, Q, ia, ib = _midpoint_case()
    X64 = X.astype(np.float64)
    ip = X64 @ Q[0].astype(np.float64)
    assert np.argmax(ip) == ia and ip[ia] - ip[ib] > 0 and ip[ia] - ip[ib] < 2e-3
    n = X.shape[0]
    say("case bf16 midpoints")
    oix = orc.OracleIndex(X, 4, 16, seed=3, threads=4)
    with nr.nrlsh_build(X, 4, 16, 3) as gix:
        for k in (1, 2):
            oids, oips = oix.query(Q, k, n)
            assert np.all(oids[:, 0] == ia)
            for mode in ("screen", "screen_bf16x3", "screen_fp32", "gather"):
                ids, ips = nr.nrlsh_query(gix, Q, k, n, rerank=mode)
                assert np.array_equal(ids, oids), f"k={k} {mode}: {ids[:, 0]}"
                assert np.array_equal(ips, oips.astype(np.float32)), f"k={k} {mode}"
            # the bfloat16 first pass of the gather re-rank bounds each row's
            # own rounding error
            ids, ips = nr.nrlsh_query(gix, Q, k, n, rerank="gather", rerank_storage="bf16")
            assert np.array_equal(ids, oids), f"k={k} bf16 rows: {ids[:, 0]}"
            assert np.array_equal(ips, oips.astype(np.float32)), f"k={k} bf16 rows"


STAGED_CASES = [
    # (n, d, m, L, nq, k, T, sigma, early): long-tailed norms, so that a small
    # budget is met inside the top sub-datasets and the tiles stop early; a
    # budget of a third of the items needs every sub-dataset
    (60000, 32, 64, 32, 130, 10, 600, 1.0, True),
    (40000, 48, 128, 64, 70, 100, 2000, 1.0, True),
    (30000, 16, 16, 20, 200, 10, 50, 0.8, True),
    (20000, 24, 40, 33, 65, 10, 7000, 1.2, False),
]


@pytest.mark.parametrize("case", STAGED_CASES, ids=lambda c: "n%d_m%d_L%d_T%d" % (c[0], c[2], c[3], c[6]))
def test_staged_scan_early_exit(case):
    """The first scan pass visits sub-datasets in descending U_j and stops a
    tile once every query's threshold bucket is known: probed sets, top-k ids
    and inner products still equal the oracle's, and fewer pairs are counted
    than nq x n."""
    n, d, m, L, nq, k, T, sigma, early = case
    say(f"case staged scan n={n} d={d} m={m} L={L} nq={nq} k={k} T={T}")
    X = make_items("lognormal", n, d, seed=n + 11, sigma=sigma)
    Q = make_queries(nq, d, seed=n + 12)
    oix = orc.OracleIndex(X, m, L, seed=29, threads=8)
    with nr.nrlsh_build(X, m, L, 29) as gix:
        check_query(gix, oix, Q, k, T, f"staged n{n}")
        oids, oips = oix.query(Q, k, T, threads=8)
        for mode in ("gather", "screen"):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank=mode)
            st = nr.nrlsh_get_query_stats()
            say(f"  {mode}: pass-1 pairs {st['scan_pairs']} of {nq * n}")
            assert np.array_equal(ids, oids), mode
            assert np.array_equal(ips, oips.astype(np.float32)), mode
            assert 0 < st["scan_pairs"] <= nq * n, st["scan_pairs"]
            if early:
                assert st["scan_pairs"] < nq * n, st["scan_pairs"]


@pytest.mark.parametrize("proj", ["shared", "per_subset"])
def test_candidates_with_levels(proj):
    """The probed set with each item's level l (equal code bits) against the
    oracle's probing order: the same (id, l) pairs, as sets."""
    say(f"case candidates with levels {proj}")
    n, d, m, L, nq, T = 20000, 16, 8, 24, 24, 3000
    X = make_items("lognormal", n, d, seed=105, sigma=1.0)
    Q = make_queries(nq, d, seed=106)
    oix = orc.OracleIndex(X, m, L, seed=33, projections=proj)
    with nr.nrlsh_build(X, m, L, 33, projections=proj) as gix:
        ids, lv = gix.query_candidates_levels(Q, T)
        assert ids.shape == (nq, T) and lv.shape == (nq, T)
        # the same set as the ids-only call (the order of a probed list is
        # that of its appends, which varies from call to call)
        assert np.array_equal(np.sort(ids, axis=1), np.sort(gix.query_candidates(Q, T), axis=1))
        for i in range(nq):
            oc, ol = oix.candidates(Q[i], T)
            assert sorted(zip(ids[i].tolist(), lv[i].tolist())) == sorted(zip(oc.tolist(), ol.tolist())), i
