"""Batching form: many indexes of uneven n, d, L and m, each with its own query
batch, served by one launch per phase over all pairs (replayed from a
captured hipGraph).  Each pair must get exactly what the CPU
oracle gives for that index and batch (same probed set, same top-k, same FP64
inner products), whatever the tile shapes, graph replay or autotuning."""
import numpy as np
import pytest
import torch

import oracle.oracle as orc
import paper_1809_08782_amd as nr
from parity_util import say
from workloads import make_items, make_queries

pytestmark = pytest.mark.gpu

# (n, d, m, L, nq, T, items kind, seed): ragged tails everywhere, W = 1 and 2,
# a single query, tiles with 6 and 64 queries, T >= n, T < k
SET = [
    (3000, 64, 8, 32, 70, 300, "lognormal", 11),
    (1500, 33, 3, 16, 1, 1500, "lognormal", 12),
    (5000, 128, 16, 64, 130, 700, "pareto", 13),
    (800, 20, 1, 48, 64, 9, "lognormal", 14),
    (4100, 256, 16, 32, 5, 2000, "lowrank", 15),
    (2200, 100, 7, 63, 200, 4000, "pareto", 16),
]

_cache = {}


def _set_state():
    """Indexes, queries and oracle results of SET (built once per process)."""
    if "set" in _cache:
        return _cache["set"]
    state = []
    for (n, d, m, L, nq, T, kind, seed) in SET:
        kw = {"alpha": 2.5} if kind == "pareto" else {"sigma": 0.8} if kind == "lognormal" else {}
        X = make_items(kind, n, d, seed=seed, **kw)
        Q = make_queries(nq, d, seed=seed + 100)
        oix = orc.OracleIndex(X, m, L, seed=seed + 200, threads=8)
        gix = nr.nrlsh_build(X, m, L, seed + 200)
        state.append({"X": X, "Q": Q, "T": T, "oix": oix, "gix": gix})
    _cache["set"] = state
    return state


def _expected(state, k):
    key = ("exp", k)
    if key not in _cache:
        _cache[key] = [st["oix"].query(st["Q"], k, st["T"], threads=8) for st in state]
    return _cache[key]


def _check(outs, exp, label):
    for i, ((ids, ips), (oids, oips)) in enumerate(zip(outs, exp)):
        if isinstance(ids, torch.Tensor):
            ids, ips = ids.cpu().numpy(), ips.cpu().numpy()
        assert np.array_equal(ids, oids), f"{label}: pair {i} ids"
        assert np.array_equal(ips, oips.astype(np.float32)), f"{label}: pair {i} ips"


def _pairs(state, device):
    out = []
    for st in state:
        q = torch.from_numpy(st["Q"]).cuda() if device else st["Q"]
        out.append((st["gix"], q, st["T"]))
    return out


def test_multi_host_pointers_and_direct_launch():
    say("case multi host pointers, no graph")
    state = _set_state()
    outs = nr.nrlsh_query_multi(_pairs(state, False), 10, use_graph=False)
    _check(outs, _expected(state, 10), "host")


@pytest.mark.parametrize("k", [10, 100])
def test_multi_matches_oracle_device_pointers(k):
    say(f"case multi device k={k}")
    state = _set_state()
    with nr.MultiPlan(_pairs(state, True), k) as plan:
        info = plan.info()
        say(f"  grid {info['grid']} graph {info['graph']} items {info['items']}")
        assert info["graph"]
        outs = plan.run()
        torch.cuda.synchronize()
        _check(outs, _expected(state, k), f"k={k}")


@pytest.mark.parametrize("chunk,slice", [(64, 64), (128, 192), (4096, 512), (65536, 4096)])
def test_multi_any_tile_shape_same_result(chunk, slice):
    """Tiny chunks (many pass-1 / pass-2 items per sub-dataset, the threshold
    bucket cut across chunks) and tiny slices (many re-rank items and a merge)."""
    say(f"case multi chunk={chunk} slice={slice}")
    state = _set_state()
    with nr.MultiPlan(_pairs(state, True), 10, chunk=chunk, slice=slice) as plan:
        assert set(plan.info()["chunk"]) == {chunk}
        outs = plan.run()
        torch.cuda.synchronize()
        _check(outs, _expected(state, 10), f"chunk={chunk} slice={slice}")


def test_multi_graph_replays_with_new_queries():
    """Replays of one captured graph, with new query contents between them and
    eager single-index queries interleaved: every replay matches the oracle."""
    say("case multi replays")
    state = _set_state()
    pairs = _pairs(state, True)
    with nr.MultiPlan(pairs, 10) as plan:
        for rep in range(3):
            qs = []
            for i, st in enumerate(state):
                Q = make_queries(st["Q"].shape[0], st["Q"].shape[1], seed=500 + 10 * rep + i)
                qs.append(torch.from_numpy(Q).cuda())
            outs = plan.run(qs)
            torch.cuda.synchronize()
            exp = [st["oix"].query(q.cpu().numpy(), 10, st["T"], threads=8) for st, q in zip(state, qs)]
            _check(outs, exp, f"replay {rep}")
            # eager work between replays
            ids, _ = nr.nrlsh_query(state[0]["gix"], qs[0], 10, state[0]["T"])
            assert np.array_equal(ids.cpu().numpy(), exp[0][0])


def test_multi_autotune_fills_table_and_keeps_results():
    say("case multi autotune")
    state = _set_state()
    nr.nrlsh_tune_clear()
    with nr.MultiPlan(_pairs(state, True), 10, tune="missing") as plan:
        info = plan.info()
        say(f"  tuned {info['tuned_classes']} classes in {info['tune_ms']:.1f} ms: "
            f"chunk {info['chunk']} slice {info['slice']}")
        assert info["tuned_classes"] >= 1
        for st, c, s in zip(state, info["chunk"], info["slice"]):
            got = nr.nrlsh_tune_lookup(st["gix"].d, st["gix"].L, st["Q"].shape[0])
            assert got == (c, s)
        outs = plan.run()
        torch.cuda.synchronize()
        _check(outs, _expected(state, 10), "tuned")
    # a second plan takes the shapes from the table without timing anything
    with nr.MultiPlan(_pairs(state, True), 10, tune="missing") as plan:
        assert plan.info()["tuned_classes"] == 0


def test_multi_skips_empty_batches_and_rejects_nonfinite():
    say("case multi empty batch and non-finite query")
    state = _set_state()
    pairs = _pairs(state, True)
    d0 = state[0]["Q"].shape[1]
    pairs.insert(2, (state[0]["gix"], torch.empty((0, d0), device="cuda"), 50))
    with nr.MultiPlan(pairs, 10) as plan:
        outs = plan.run()
        torch.cuda.synchronize()
        exp = list(_expected(state, 10))
        exp.insert(2, (np.empty((0, 10), np.int64), np.empty((0, 10), np.float32)))
        _check(outs, exp, "with empty")
        bad = [q.clone() for _, q, _ in pairs]
        bad[0][3, 5] = float("nan")
        with pytest.raises(nr.NrlshError, match="NOT_FINITE"):
            plan.run(bad)
        # the plan keeps working after the rejected batch
        outs = plan.run([q for _, q, _ in pairs])
        torch.cuda.synchronize()
        _check(outs, exp, "after non-finite")


def test_multi_rejects_shape_mismatch():
    state = _set_state()
    pairs = _pairs(state, True)
    with nr.MultiPlan(pairs, 10) as plan:
        qs = [q for _, q, _ in pairs]
        qs[1] = torch.cat([qs[1], qs[1]])
        with pytest.raises(nr.NrlshError, match="shape"):
            plan.run(qs)


def test_multi_persistent_form_is_rejected():
    """The single persistent launch is disabled: asking for it fails on the host."""
    state = _set_state()
    with pytest.raises(nr.NrlshError, match="persistent"):
        nr.MultiPlan(_pairs(state, True), 10, persistent=True)


@pytest.mark.skip(reason="the single persistent launch is disabled: its launches did not "
                         "complete (two runs ended by the 120 s test time-out); the cause is "
                         "not yet shown, so it stays off the GPU")
def test_multi_persistent_launch_matches_oracle():
    state = _set_state()
    with nr.MultiPlan(_pairs(state, True), 10, persistent=True) as plan:
        outs = plan.run()
        torch.cuda.synchronize()
        _check(outs, _expected(state, 10), "persistent")
