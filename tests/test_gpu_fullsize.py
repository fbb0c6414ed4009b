"""Parity at the largest single-GPU workload: n = 1e7 items of d = 128 with
LogNormal(0, 1) norms, m = 128, L = 64, top-100 at budget 5e4, one batch of
4096 queries (the launch configuration the benchmark times), in the plain
FP32 form and in the precision form (FP8 hash copy under the rigorous margin,
bfloat16 re-rank copy).  The whole index is compared with the oracle's (keys,
partition, layout, projection, rank table, every item code), and 32 of the
batch's queries, spread over its tiles, element by element."""
import numpy as np
import pytest

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import check_build, say
from workloads.synthetic import large_shaped

pytestmark = pytest.mark.gpu


def test_full_size_index_and_sampled_queries():
    import torch

    torch.cuda.set_device(0)
    w = large_shaped()
    T = w.budgets[0]
    say(f"case full size n={w.n} d={w.d} m={w.m} L={w.L} k={w.k} T={T}: generating inputs")
    X = w.items()
    Q = w.queries(4096)
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    sample = np.linspace(0, Q.shape[0] - 1, 32).astype(np.int64)
    say("oracle build")
    oix = orc.OracleIndex(X, w.m, w.L, w.index_seed, threads=16)
    oids, oips = oix.query(Q[sample], w.k, T, threads=16)
    for hash_storage, rerank_storage in (("fp32", "fp32"), ("fp8", "bf16")):
        say(f"form hash={hash_storage} rerank={rerank_storage}")
        with nr.nrlsh_build(Xd, w.m, w.L, w.index_seed, hash_storage=hash_storage) as gix:
            check_build(gix, oix, f"full {hash_storage}")
            ids, ips = nr.nrlsh_query(gix, Qd, w.k, T, rerank="gather", rerank_storage=rerank_storage)
            st = nr.nrlsh_get_query_stats()
            say(f"  query stats {st}")
            ids = ids.cpu().numpy()[sample]
            ips = ips.cpu().numpy()[sample]
            assert np.array_equal(ids, oids), f"{hash_storage}: top-k ids"
            assert np.array_equal(ips, oips.astype(np.float32)), f"{hash_storage}: inner products"
    oix.close()
