"""Bucket-table probe (the hash lookup of Section 3.3): the table built on the
GPU equals the distinct codes of each sub-dataset, and queries through it
probe exactly the oracle's set and return the oracle's top-k, whether buckets
are found by Hamming-ball lookups or by whole-sub-dataset passes."""
import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu


def _expected_table(codes, sid, m):
    """Distinct codes of each sub-dataset from the oracle's codes (numpy)."""
    n = codes.shape[0]
    # stored order: sub-dataset major, index ascending; then stable by code
    perm = np.lexsort((np.arange(n), sid))
    pos_of = np.empty(n, np.int64)
    pos_of[perm] = np.arange(n)
    order = np.lexsort((pos_of, codes, sid))
    titem = pos_of[order].astype(np.int32)
    sc, cc = sid[order], codes[order]
    start = np.ones(n, bool)
    start[1:] = (sc[1:] != sc[:-1]) | (cc[1:] != cc[:-1])
    ustart = np.concatenate([np.flatnonzero(start), [n]]).astype(np.int64)
    ucode = cc[start]
    usid = sc[start]
    uoff = np.searchsorted(usid, np.arange(m + 1), side="left").astype(np.int64)
    return ucode, ustart, uoff, titem


CASES = [
    # (n, d, m, L, kind, partition, projections, budgets)
    (6000, 40, 16, 32, "lognormal", "percentile", "shared", (1, 37, 600, 6000)),
    (5000, 64, 8, 64, "pareto", "percentile", "shared", (500, 5000)),
    (20000, 24, 8, 12, "lognormal", "percentile", "shared", (1, 100, 1000, 20000)),  # short codes
    (3000, 17, 1, 20, "lognormal", "percentile", "shared", (64, 3000)),
    (5000, 64, 32, 16, "pareto", "uniform", "per_subset", (300, 5000)),  # empty sub-datasets
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_d%d_m%d_L%d_%s_%s_%s" % c[:7])
def test_table_probe_matches_oracle(case):
    n, d, m, L, kind, part, proj, budgets = case
    say(f"case table n={n} d={d} m={m} L={L} {kind} {part} {proj}")
    kw = {"alpha": 2.5} if kind == "pareto" else {"sigma": 1.0}
    X = make_items(kind, n, d, seed=n + L, **kw)
    Q = make_queries(70, d, seed=n + 7)
    oix = orc.OracleIndex(X, m, L, seed=31, threads=8, partition=part, projections=proj)
    with nr.nrlsh_build(X, m, L, 31, partition=part, projections=proj, bucket_tables=True) as gix:
        ucode, ustart, uoff, titem = gix.bucket_table()
        eu, es, eo, et = _expected_table(oix.codes, oix.sid, m)
        say(f"  distinct codes {ucode.shape[0]} of {n}")
        assert np.array_equal(ucode, eu) and np.array_equal(ustart, es)
        assert np.array_equal(uoff, eo) and np.array_equal(titem, et)
        for T in budgets:
            oids, oips = oix.query(Q, 10, T, threads=8)
            ids, ips = nr.nrlsh_query(gix, Q, 10, T, probe="table")
            st = nr.nrlsh_get_query_stats()
            say(f"  T={T}: lookups {st['table_lookups']} walked {st['table_walked']} "
                f"passes {st['table_passes']}")
            assert st["probe"] == "table"
            assert np.array_equal(ids, oids), f"T={T} ids"
            assert np.array_equal(ips, oips.astype(np.float32)), f"T={T} ips"
            if T <= 1024:  # k = T: the whole probed set, ordered
                kk = min(T, n)
                ids_all, _ = nr.nrlsh_query(gix, Q[:12], kk, T, probe="table")
                oall, _ = oix.query(Q[:12], kk, T, threads=8)
                assert np.array_equal(ids_all, oall), f"T={T} probed set"


def test_table_probe_duplicates_and_bf16_rows():
    """Many equal rows (long runs per code), the BF16 re-rank copy, and both
    lookup kinds in one batch."""
    say("case table duplicates")
    base = make_items("lognormal", 400, 16, seed=3, sigma=0.7)
    X = np.repeat(base, 10, axis=0)
    Q = make_queries(40, 16, seed=4)
    oix = orc.OracleIndex(X, 4, 10, seed=5, threads=8)
    with nr.nrlsh_build(X, 4, 10, 5, bucket_tables=True) as gix:
        for T in (5, 333, 4000):
            oids, oips = oix.query(Q, 20, T, threads=8)
            for storage in ("fp32", "bf16"):
                ids, ips = nr.nrlsh_query(gix, Q, 20, T, probe="table", rerank_storage=storage)
                assert np.array_equal(ids, oids), (T, storage)
                assert np.array_equal(ips, oips.astype(np.float32)), (T, storage)
        st = nr.nrlsh_get_query_stats()
        assert st["table_walked"] > 0


def test_table_probe_device_queries_and_rejections():
    import torch
    X = make_items("lognormal", 3000, 32, seed=8, sigma=0.8)
    Q = make_queries(130, 32, seed=9)
    oix = orc.OracleIndex(X, 6, 16, seed=10, threads=8)
    oids, _ = oix.query(Q, 10, 250, threads=8)
    with nr.nrlsh_build(torch.from_numpy(X).cuda(), 6, 16, 10, bucket_tables=True) as gix:
        ids, _ = nr.nrlsh_query(gix, torch.from_numpy(Q).cuda(), 10, 250, probe="table")
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), oids)
        with pytest.raises(nr.NrlshError, match="GATHER"):
            nr.nrlsh_query(gix, Q, 10, 250, probe="table", rerank="screen")
    with nr.nrlsh_build(X, 6, 16, 10) as plain:
        with pytest.raises(nr.NrlshError, match="bucket_tables"):
            nr.nrlsh_query(plain, Q, 10, 250, probe="table")
        with pytest.raises(nr.NrlshError, match="bucket tables"):
            plain.bucket_table()
