"""GPU parity of the multi-table single probe (the alternative to the
single-table multi-probe that Section 4 names): each table's projection
block and codes, the probed sets (tables in order until the budget, the
table where it runs out cut higher-norm sub-datasets first and by index),
top-k ids and inner products, against the FP64 oracle."""
import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu

CASES = [
    # (n, d, m, L, tables, projections, nq, k, budgets)
    (6000, 24, 8, 8, 3, "shared", 70, 10, (1, 40, 500, 6000)),
    (9000, 40, 16, 12, 8, "shared", 130, 10, (100, 2000, 9000)),
    (5000, 17, 6, 16, 4, "per_subset", 65, 5, (20, 300, 5000)),
    (4000, 64, 4, 40, 2, "shared", 64, 16, (10, 4000)),
    (3000, 30, 5, 6, 1, "shared", 50, 10, (30, 3000)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_m%d_L%d_t%d_%s" % (c[0], c[2], c[3], c[4], c[5]))
def test_single_probe_matches_oracle(case):
    n, d, m, L, t, proj, nq, k, budgets = case
    say(f"case single probe n={n} d={d} m={m} L={L} tables={t} {proj}")
    X = make_items("lognormal", n, d, seed=n + 61, sigma=0.9)
    Q = make_queries(nq, d, seed=n + 62)
    oix = orc.OracleIndex(X, m, L, seed=71, threads=8, projections=proj, tables=t)
    with nr.nrlsh_build(X, m, L, 71, projections=proj, hash_tables=t) as gix:
        assert gix.tables == t
        A = gix.projection()
        assert np.array_equal(A.view(np.uint32), oix.A.view(np.uint32))
        for tb in range(t):
            assert np.array_equal(gix.codes(tb), oix.codes_t[tb]), f"codes of table {tb}"
        for T in budgets:
            cands = gix.query_candidates(Q, T, probe="single")
            sizes = []
            for qi in range(nq):
                oc = oix.candidates_single_probe(Q[qi], T)
                sizes.append(len(oc))
                assert np.array_equal(np.sort(cands[qi]), np.sort(oc)), f"T={T} probed set of query {qi}"
            ids, ips = nr.nrlsh_query(gix, Q, k, T, probe="single")
            oids, oips = oix.query_single_probe(Q, k, T, threads=8)
            say(f"  T={T}: probed per query {min(sizes)}..{max(sizes)}")
            assert np.array_equal(ids, oids), f"T={T} ids"
            assert np.array_equal(ips, oips.astype(np.float32)), f"T={T} ips"
        # the multi-probe query still reads table 0 only
        ids, _ = nr.nrlsh_query(gix, Q[:8], k, 300)
        o1 = orc.OracleIndex(X, m, L, seed=71, threads=8, projections=proj)
        oids, _ = o1.query(Q[:8], k, 300)
        assert np.array_equal(ids, oids)


def test_single_probe_device_pointers_and_rejections():
    import torch
    X = make_items("lognormal", 3000, 16, seed=7, sigma=0.8)
    Q = make_queries(20, 16, seed=8)
    oix = orc.OracleIndex(X, 4, 10, seed=9, tables=3)
    with nr.nrlsh_build(torch.from_numpy(X).cuda(), 4, 10, 9, hash_tables=3) as gix:
        ids, ips = nr.nrlsh_query(gix, torch.from_numpy(Q).cuda(), 5, 200, probe="single")
        torch.cuda.synchronize()
        oids, oips = oix.query_single_probe(Q, 5, 200)
        assert np.array_equal(ids.cpu().numpy(), oids)
        assert np.array_equal(ips.cpu().numpy(), oips.astype(np.float32))
        with pytest.raises(nr.NrlshError, match="GATHER"):
            nr.nrlsh_query(gix, Q, 5, 200, probe="single", rerank="screen")
    with pytest.raises(nr.NrlshError, match="hash_tables"):
        nr.nrlsh_build(X, 4, 10, 9, hash_tables=9)
    with pytest.raises(nr.NrlshError, match="FP32"):
        nr.nrlsh_build(X, 4, 10, 9, hash_tables=2, hash_storage="bf16")
