"""The query entry point that allocates nothing (nrlsh_query_noalloc, every
temporary buffer in the library's device scratch) against nrlsh_query_ex on
the same index and queries: two calls in a row, the second with a smaller
input, bit-identical ids and inner products."""
import numpy as np
import pytest
import torch

import paper_1809_08782_amd as nr
from parity_util import say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu


def _noalloc(ix, Qd, k, T):
    nq = Qd.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    ips = torch.full((nq, k), 7.0, dtype=torch.float32, device="cuda")
    flag = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    nr.nrlsh_query_noalloc(ix, Qd, k, T, (ids, ips), flag)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), ips.cpu().numpy(), int(flag.item())


def test_noalloc_matches_query_ex_two_calls():
    torch.cuda.set_device(0)
    n, d, m, L = 50000, 40, 64, 64
    X = make_items("lognormal", n, d, seed=81, sigma=1.0)
    Qa = make_queries(300, d, seed=82)
    Qb = make_queries(70, d, seed=83)
    Xd = torch.from_numpy(X).cuda()
    with nr.nrlsh_build(Xd, m, L, 84) as ix:
        # first call: 300 queries (five batches of 64 and a ragged one at most)
        for Q, k, T in ((Qa, 10, 3000), (Qb, 7, 500)):
            say(f"case noalloc nq={Q.shape[0]} k={k} T={T}")
            Qd = torch.from_numpy(Q).cuda()
            ids, ips, flag = _noalloc(ix, Qd, k, T)
            rids, rips = nr.nrlsh_query(ix, Qd, k, T, rerank="gather")
            torch.cuda.synchronize()
            assert flag == 0
            assert np.array_equal(ids, rids.cpu().numpy()), f"ids differ at nq={Q.shape[0]}"
            assert np.array_equal(ips, rips.cpu().numpy()), f"ips differ at nq={Q.shape[0]}"


def test_noalloc_flags_nonfinite_and_rejects_oversize():
    torch.cuda.set_device(0)
    n, d, m, L = 300000, 4, 8, 16
    X = make_items("lognormal", n, d, seed=91, sigma=0.5)
    Q = make_queries(5, d, seed=92)
    Q[3, 1] = np.nan
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    with nr.nrlsh_build(Xd, m, L, 93) as ix:
        _, _, flag = _noalloc(ix, Qd, 3, 100)
        assert flag != 0
        # 64 lists of 280,000 entries do not fit the 64 MiB scratch
        with pytest.raises(nr.NrlshError, match="scratch"):
            _noalloc(ix, Qd[:2], 3, 280000)
