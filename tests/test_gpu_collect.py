"""The collecting scan (one scan behind a sampled guess of each query's cut,
then the threshold pass and a filter of the collected keys) against the FP64
oracle: probed sets, top-k ids and inner products, the default and the forced
fallback to the two exact passes, ties in the threshold bucket."""
import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import check_query, say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu

# (n, d, m, L, nq, k, T, projections): budgets of 6400 and more below 2n/3
# take the collecting scan by default; 1, 2 and 3 tiles with ragged tails
CASES = [
    (60000, 40, 16, 32, 130, 10, 8000, "shared"),
    (80000, 24, 32, 64, 70, 100, 12000, "shared"),
    (50000, 20, 8, 16, 64, 10, 9000, "per_subset"),
    (45000, 9, 5, 63, 200, 16, 20000, "shared"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_m%d_L%d_T%d_%s" % (c[0], c[2], c[3], c[6], c[7]))
def test_collect_matches_oracle(case):
    n, d, m, L, nq, k, T, proj = case
    say(f"case collect n={n} d={d} m={m} L={L} nq={nq} k={k} T={T} {proj}")
    X = make_items("lognormal", n, d, seed=n + 3, sigma=1.0)
    Q = make_queries(nq, d, seed=n + 4)
    oix = orc.OracleIndex(X, m, L, seed=77 + L, threads=8, projections=proj)
    with nr.nrlsh_build(X, m, L, 77 + L, projections=proj) as gix:
        # probed sets (the candidates call takes the scan probe), then the
        # top-k of every re-rank mode
        check_query(gix, oix, Q, k, T, f"collect n{n}")
        oids, oips = oix.query(Q, k, T)
        for storage in ("fp32", "bf16"):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage=storage)
            st = nr.nrlsh_get_query_stats()
            assert st["scan_pairs"] > 0 and st["collect_fallbacks"] == 0, st
            assert np.array_equal(ids, oids), storage
            assert np.array_equal(ips, oips.astype(np.float32)), storage
        # the two passes alone give the same answer
        ids2, ips2 = nr.nrlsh_query(gix, Q, k, T, rerank="gather", scan_guess=-1)
        assert np.array_equal(ids2, oids) and np.array_equal(ips2, oips.astype(np.float32))


@pytest.mark.parametrize("guess", [1, 4096])
def test_collect_guess_that_misses_falls_back(guess):
    """A guess of T/16 items tends to collect too few (the cut bucket may
    still bring enough), one of 256 T too many for the key room (every item
    is collected): such batches are probed again by the two passes, with the
    same result."""
    say(f"case collect fallback guess={guess}")
    n, d, m, L = 40000, 32, 8, 32
    X = make_items("lognormal", n, d, seed=91, sigma=0.8)
    Q = make_queries(100, d, seed=92)
    oix = orc.OracleIndex(X, m, L, seed=5, threads=8)
    fallbacks = []
    with nr.nrlsh_build(X, m, L, 5) as gix:
        for T in (500, 7000):
            ids, ips = nr.nrlsh_query(gix, Q, 10, T, rerank="gather", scan_guess=guess)
            fallbacks.append(nr.nrlsh_get_query_stats()["collect_fallbacks"])
            oids, oips = oix.query(Q, 10, T)
            assert np.array_equal(ids, oids), T
            assert np.array_equal(ips, oips.astype(np.float32)), T
    say(f"  fallbacks per budget {fallbacks}")
    assert fallbacks[0] >= 1
    if guess == 4096:  # every item collected: more than the key room
        assert min(fallbacks) >= 1


def test_collect_small_budget_and_tied_buckets():
    """The collecting scan forced on small budgets (the sample is every group)
    over items repeated many times, so that threshold buckets hold long runs of
    equal codes cut by stored position."""
    say("case collect ties")
    base = make_items("lognormal", 700, 16, seed=93, sigma=0.7)
    X = np.ascontiguousarray(np.repeat(base, 12, axis=0)[:8000])
    Q = make_queries(90, 16, seed=94)
    oix = orc.OracleIndex(X, 6, 24, seed=9, threads=8)
    with nr.nrlsh_build(X, 6, 24, 9) as gix:
        for T, g in ((333, 16), (1000, 20), (2500, 40)):
            ids, ips = nr.nrlsh_query(gix, Q, 12, T, rerank="gather", scan_guess=g)
            oids, oips = oix.query(Q, 12, T)
            assert np.array_equal(ids, oids), (T, g)
            assert np.array_equal(ips, oips.astype(np.float32)), (T, g)


def test_dense_head_matches_oracle():
    """The bfloat16 re-rank with its dense head (sub-datasets screened whole on
    the matrix cores, seeded theta for the gather of the others): none, the
    default range, the widest (probed fraction 1/256) and the narrowest (1/4),
    on three batches with a ragged tail."""
    say("case dense head")
    n, d, m, L, nq, k, T = 120000, 32, 16, 32, 150, 20, 9000
    X = make_items("lognormal", n, d, seed=95, sigma=1.0)
    Q = make_queries(nq, d, seed=96)
    oix = orc.OracleIndex(X, m, L, seed=13, threads=8)
    oids, oips = oix.query(Q, k, T)
    items = {}
    with nr.nrlsh_build(X, m, L, 13) as gix:
        for dense_head in (-1, 0, 1, 64):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage="bf16",
                                      dense_head=dense_head)
            st = nr.nrlsh_get_query_stats()
            say(f"  dense_head {dense_head}: stats {st}")
            assert st["collect_fallbacks"] == 0 and st["lp_fallbacks"] == 0, st
            items[dense_head] = st["dense_head_items"]
            # the keep pass evaluates at most every (query, head item) pair
            assert 0 <= st["dense_head_pairs"] <= nq * st["dense_head_items"], st
            assert (st["dense_head_pairs"] > 0) == (st["dense_head_items"] > 0), st
            assert np.array_equal(ids, oids), dense_head
            assert np.array_equal(ips, oips.astype(np.float32)), dense_head
    assert items[-1] == 0, items
    assert items[1] >= items[0] >= items[64] and items[1] > 0, items


@pytest.mark.parametrize("m", [6, 2])
def test_dense_head_tied_buckets(m):
    """Dense head over every sub-dataset with threshold buckets holding long
    runs of equal codes, cut by stored position inside the screened range;
    with m = 2 each sub-dataset holds more items than its witnesses, whose
    selection by norm then meets long runs of equal keys."""
    say(f"case dense head ties m={m}")
    base = make_items("lognormal", 900, 16, seed=97, sigma=0.7)
    X = np.ascontiguousarray(np.repeat(base, 14, axis=0)[:12000])
    Q = make_queries(80, 16, seed=98)
    oix = orc.OracleIndex(X, m, 24, seed=21, threads=8)
    with nr.nrlsh_build(X, m, 24, 21) as gix:
        for T, g in ((1500, 20), (4000, 18), (7000, 24)):
            ids, ips = nr.nrlsh_query(gix, Q, 12, T, rerank="gather", rerank_storage="bf16", scan_guess=g,
                                      dense_head=1)
            st = nr.nrlsh_get_query_stats()
            assert st["dense_head_items"] > 0 and st["collect_fallbacks"] == 0, (T, st)
            oids, oips = oix.query(Q, 12, T)
            assert np.array_equal(ids, oids), (T, g)
            assert np.array_equal(ips, oips.astype(np.float32)), (T, g)


def test_dense_head_overflow_reruns_without_head():
    """Items alike to within the bfloat16 bounds: the screen keeps every probed
    pair of the head, the lists overflow, and the batch runs again without the
    head (then the FP32 re-rank), with the same result."""
    say("case dense head overflow")
    n, d, m, L, k, T = 30000, 16, 4, 16, 10, 19000
    rng = np.random.default_rng(99)
    v = rng.standard_normal(d).astype(np.float32)
    X = np.ascontiguousarray((v[None, :] * (1.0 + 1e-4 * rng.standard_normal((n, 1)))
                              + 1e-5 * rng.standard_normal((n, d))).astype(np.float32))
    Q = make_queries(64, d, seed=100)
    oix = orc.OracleIndex(X, m, L, seed=23, threads=8)
    oids, oips = oix.query(Q, k, T)
    with nr.nrlsh_build(X, m, L, 23) as gix:
        ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage="bf16", dense_head=1)
        st = nr.nrlsh_get_query_stats()
        say(f"  stats {st}")
        assert st["lp_fallbacks"] >= 1, st
        assert np.array_equal(ids, oids)
        assert np.array_equal(ips, oips.astype(np.float32))


def test_probing_order_too_long_for_lds():
    """m (L + 1) buckets beyond what the threshold pass stages in LDS (12,288):
    it then reads the probing order from memory; the two-pass scan (small
    budget) and the collecting scan (large budget) against the oracle."""
    say("case threshold order in memory")
    n, d, m, L, k = 48000, 12, 400, 32, 10
    X = make_items("lognormal", n, d, seed=101, sigma=1.0)
    Q = make_queries(70, d, seed=102)
    oix = orc.OracleIndex(X, m, L, seed=31, threads=8)
    with nr.nrlsh_build(X, m, L, 31) as gix:
        for T in (3000, 12000):
            ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather")
            oids, oips = oix.query(Q, k, T)
            assert np.array_equal(ids, oids), T
            assert np.array_equal(ips, oips.astype(np.float32)), T
        assert nr.nrlsh_get_query_stats()["scan_pairs"] > 0


@pytest.mark.parametrize("T", [6500, 7000])
def test_dense_head_every_pair_a_candidate(T):
    """Items alike to within the bfloat16 bounds and a budget below the kept
    lists' room: every evaluated pair of the head reaches theta, so the keep
    pass's candidate queue fills and empties many times per iteration, and
    the kept lists (every probed pair of the head) are used, not run again."""
    say(f"case dense head every pair a candidate T={T}")
    n, d, m, L, k = 30000, 16, 4, 16, 10
    rng = np.random.default_rng(103)
    v = rng.standard_normal(d).astype(np.float32)
    X = np.ascontiguousarray((v[None, :] * (1.0 + 1e-4 * rng.standard_normal((n, 1)))
                              + 1e-5 * rng.standard_normal((n, d))).astype(np.float32))
    Q = make_queries(64, d, seed=104)
    oix = orc.OracleIndex(X, m, L, seed=29, threads=8)
    oids, oips = oix.query(Q, k, T)
    with nr.nrlsh_build(X, m, L, 29) as gix:
        ids, ips = nr.nrlsh_query(gix, Q, k, T, rerank="gather", rerank_storage="bf16", dense_head=1)
        st = nr.nrlsh_get_query_stats()
        say(f"  stats {st}")
        assert st["dense_head_items"] > 0 and st["lp_fallbacks"] == 0 and st["collect_fallbacks"] == 0, st
        assert np.array_equal(ids, oids)
        assert np.array_equal(ips, oips.astype(np.float32))
