"""Shared helpers of the GPU parity tests: run the HIP library and the CPU
oracle on the same seeded inputs and compare every step."""
import sys

import numpy as np

import oracle.oracle as orc
import paper_1809_08782_amd as nr


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected_layout(sid, m):
    """Stored order: sub-dataset major, ascending original index inside."""
    perm = np.lexsort((np.arange(sid.shape[0]), sid)).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(np.bincount(sid, minlength=m))]).astype(np.int64)
    return perm, off


def check_build(gix, oix, label=""):
    """Index parity: keys, partition, layout, projection, codes, rank table."""
    assert gix.n == oix.n and gix.d == oix.d and gix.m == oix.m and gix.L == oix.L
    A = gix.projection()
    assert np.array_equal(A.view(np.uint32), oix.A.view(np.uint32)), f"{label}: projection"
    key = gix.keys()
    assert np.array_equal(key.view(np.uint64), oix.key.view(np.uint64)), f"{label}: keys"
    sid, keymax, U = gix.partition()
    assert np.array_equal(sid, oix.sid), f"{label}: sub-dataset ids"
    assert np.array_equal(keymax.view(np.uint64), oix.keymax.view(np.uint64)), f"{label}: keymax"
    assert np.array_equal(U.view(np.uint64), oix.U.view(np.uint64)), f"{label}: U"
    perm, off = gix.layout()
    eperm, eoff = expected_layout(oix.sid, oix.m)
    assert np.array_equal(perm, eperm), f"{label}: layout"
    assert np.array_equal(off, eoff), f"{label}: offsets"
    R = gix.rank_table()
    assert np.array_equal(R, oix.R), f"{label}: rank table"
    codes = gix.codes()
    diff = codes ^ oix.codes
    nbad = int(np.count_nonzero(diff))
    st = gix.build_stats()
    say(f"  [{label}] code mismatches {nbad}/{gix.n}, recomputed items "
        f"{st['recomputed_items']} bits {st['recomputed_bits']} fp32 flips {st['recompute_flips']}")
    assert nbad == 0, f"{label}: {nbad} item codes differ"
    assert 0 <= st["recompute_flips_tiny"] <= st["recompute_flips"] <= st["recomputed_bits"], st
    return st


def check_query(gix, oix, Q, k, T, label=""):
    """Query parity: query codes, probed sets, top-k ids and inner products."""
    qc = gix.query_codes(Q)
    if getattr(oix, "per_subset", False):  # one code per (query, sub-dataset)
        oqc = np.stack([oix.query_code(q) for q in Q]).reshape(Q.shape[0], oix.m)
    else:
        oqc = orc.query_codes(oix.A, Q)
    nq = Q.shape[0]
    assert np.array_equal(qc.reshape(nq, -1), oqc.reshape(nq, -1)), f"{label}: query codes"
    cand = gix.query_candidates(Q, T)
    Tq = min(T, oix.n)
    assert cand.shape == (Q.shape[0], Tq)
    for qi in range(Q.shape[0]):
        oc, _ = oix.candidates(Q[qi], T)
        assert np.array_equal(np.sort(cand[qi]), np.sort(oc)), f"{label}: probed set of query {qi}"
    ids, ips = nr.nrlsh_query(gix, Q, k, T)
    oids, oips = oix.query(Q, k, T)
    assert np.array_equal(ids, oids), f"{label}: top-k ids"
    # inner products: FP64 rounded to FP32 on both sides.  The bar is 1e-5
    # relative error against the FP64 value; the design makes them identical.
    fin = np.isfinite(oips)
    rel = np.abs(ips[fin].astype(np.float64) - oips[fin]) / np.maximum(np.abs(oips[fin]), 1e-30)
    assert rel.size == 0 or rel.max() <= 1e-5, f"{label}: ip relative error {rel.max()}"
    assert np.array_equal(ips, oips.astype(np.float32)), f"{label}: ips not bit-identical"
    assert np.all(np.isneginf(ips[~fin])) and np.all(ids[~fin] == -1)
    return ids, ips
