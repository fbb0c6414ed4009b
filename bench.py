#!/usr/bin/env python3
"""Throughput of the norm-ranging LSH hot path on one MI355X.

One step = the whole path on one batch of synthetic input already resident in
HBM: index build (norm keys, radix sort, percentile partition, SimpleLSH
transform + SRP hash, rank table) over all n items, then the multi-probe query
(query hash, staged popcount scan, threshold, emission, re-rank, top-k) of all
nq queries at probe budget T.  value = nq / query-phase time, measured with
HIP events on the library's stream; the build is timed apart in the same steps
and reported as items/s.

Default workload: n = 1e7 items of d = 128 with LogNormal(0, 1) norms,
m = 128, L = 64, k = 100, T = 5e4 (0.5 % of n), 1e5 queries in batches of
4096.  Forms: FP8 E4M3 hash + bfloat16 first-pass re-rank (exact FP64
re-check) as the headline, the plain FP32 form on the same inputs for
comparison; every form returns the same top-k.  The recall curve over
power-of-two budgets shows where recall@10 >= 0.9 is first reached.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_MFMA_PEAK_TFS = 157.3  # MI355X dense FP32 matrix
BF16_MFMA_PEAK_TFS = 2500.0  # MI355X dense bf16 matrix


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def ground_truth(Xd, Qs, k):
    """Exact top-k by FP64 inner products on the GPU (torch, independent of libnrlsh)."""
    import torch
    X64 = Xd.double()
    out = []
    for s in range(0, Qs.shape[0], 50):
        qT = Qs[s:s + 50].double().T.contiguous()
        sc = X64 @ qT                      # (n, chunk)
        out.append(torch.topk(sc, k, dim=0).indices.T.cpu())
    del X64
    return torch.cat(out).numpy()


def traffic_record(kernel, workload, T, timer=None, tag="traffic_record"):
    """HBM bytes per query of a launch of `kernel` from a committed counter
    summary (profiles/*.md, a line "traffic_record: {json}"), provided the
    sources it names still hash to what they were when the counters were taken.
    A record that names the timer it belongs to (one kernel can serve two
    steps, as the FP32 re-rank does) matches that timer only.  tag
    "sq_record" reads the instruction counts of the same summaries."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            lines = [ln for ln in f if ln.startswith(tag + ": ")]
        for ln in lines:
            rec = json.loads(ln[len(tag) + 2:])
            if rec.get("kernel") != kernel or rec.get("workload") != workload or rec.get("T") != T:
                continue
            if timer is not None and rec.get("timer", timer) != timer:
                continue
            same = True
            for src, digest in rec.get("sources", {}).items():
                fp = os.path.join(ROOT, src)
                if not os.path.exists(fp):
                    same = False
                    break
                with open(fp, "rb") as f:
                    same &= hashlib.sha256(f.read()).hexdigest() == digest
            if same:
                rec["file"] = os.path.relpath(path, ROOT)
                return rec
    return None


def recall(ids, gt):
    k = gt.shape[1]
    hit = 0
    for a, b in zip(ids, gt):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (k * gt.shape[0])


def run_batching(args):
    """Batching form: 64 indexes (n log-uniform in [1e4, 2e6], d in {64, 128,
    256}, m = 16, L = 32), a query batch of 1..4096 per index, T = max(500,
    1% of n), top-10.  One step = every pair's query batch through one plan
    (a replay of the captured graph of phase launches).  The same pairs are
    also run one index at a time through nrlsh_query for comparison."""
    import numpy as np
    import torch

    import paper_1809_08782_amd as nr
    from workloads.synthetic import batching_set

    torch.cuda.set_device(0)
    ws = batching_set(64)
    k = ws[0].k
    nq_total = sum(w.nq for w in ws)
    log(f"batching: {len(ws)} indexes, sum n = {sum(w.n for w in ws)}, sum nq = {nq_total}")
    pairs, build_s = [], 0.0
    for i, w in enumerate(ws):
        X = torch.from_numpy(w.items()).cuda()
        Q = torch.from_numpy(w.queries()).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ix = nr.nrlsh_build(X, w.m, w.L, w.index_seed)
        torch.cuda.synchronize()
        build_s += time.perf_counter() - t
        del X
        pairs.append((ix, Q, w.budgets[0]))
        if i % 16 == 15:
            log(f"  built {i + 1} indexes")
    t = time.perf_counter()
    plan = nr.MultiPlan(pairs, k, tune="missing")
    plan_s = time.perf_counter() - t
    info = plan.info()
    log(f"plan: {plan_s:.2f}s (tuning {info['tune_ms']:.0f} ms, {info['tuned_classes']} classes), "
        f"items {info['items']}")
    for i in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    nr.nrlsh_profile_reset()
    t = time.perf_counter()
    for i in range(args.steps):
        plan.run()
        log(f"  step {i + 1}/{args.steps} done ({time.perf_counter() - t:.3f}s)")
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t) / args.steps
    nr.nrlsh_profile_enable(True)
    plan.run()
    nr.nrlsh_profile_enable(False)
    multi_ms, _ = nr.nrlsh_profile_get("multi")
    outs = [(a.clone(), b.clone()) for a, b in plan.outputs]

    # the same pairs one index at a time
    def sequential():
        return [nr.nrlsh_query(ix, Q, k, T) for ix, Q, T in pairs]
    sequential()
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq_steps = max(1, args.steps // 2)
    for _ in range(seq_steps):
        seq = sequential()
    torch.cuda.synchronize()
    seq_s = (time.perf_counter() - t) / seq_steps
    same = all(torch.equal(a, c) and torch.equal(b, d) for (a, b), (c, d) in zip(outs, seq))
    log(f"batched {step_s * 1e3:.2f} ms/step, sequential {seq_s * 1e3:.2f} ms, identical={same}")

    # recall@k on up to 64 queries of each pair against exact MIPS (torch FP64)
    hit = tot = 0
    for w, (ix, Q, T), (ids, _) in zip(ws, pairs, outs):
        X = torch.from_numpy(w.items()).cuda().double()
        s = min(64, w.nq)
        gt = torch.topk(X @ Q[:s].double().T, k, dim=0).indices.T.cpu().numpy()
        got = ids[:s].cpu().numpy()
        hit += sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(got, gt))
        tot += s * k
        del X
    rec = hit / tot

    # algorithmic bytes of one step: both scan passes read every code once per
    # 64-query tile; the re-rank reads T rows (4d bytes + 8 for position and id)
    scan_b = sum(2 * math.ceil(w.nq / 64) * w.n * 4 for w in ws)
    rr_b = sum(w.nq * min(w.budgets[0], w.n) * (4 * w.d + 8) for w in ws)
    achieved = (scan_b + rr_b) / (multi_ms * 1e-3) / 1e9
    out = {
        "metric": "queries/sec at recall@10>=0.9 (plain FP32 vs BF16/FP8); scan+rerank HBM GB/s",
        "value": nq_total / step_s, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_s * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "arith": {"scan": "u32", "rerank": "f64"}, "data": "synthetic",
        "config": {"workload": "batching64", "indexes": len(ws), "sum_n": sum(w.n for w in ws),
                   "sum_nq": nq_total, "m": 16, "L": 32, "k": k, "T": "max(500, ceil(0.01 n))",
                   "parallelism": "single GPU"},
        "recall_sampled": rec,
        "sequential_ms_per_step": seq_s * 1e3, "speedup_vs_sequential": seq_s / step_s,
        "identical_to_sequential": bool(same), "build_s_all_indexes": build_s,
        "plan_s": plan_s, "plan": info,
        "roofline": {"kernel": "graph of phase launches", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": scan_b + rr_b,
                     "graph_ms": multi_ms},
        "cpu_baseline": None,
    }
    plan.close()
    for ix, _, _ in pairs:
        ix.close()
    print(json.dumps(out), flush=True)


# Forms of the path timed on the same inputs.  Every form returns the same
# top-k (the re-rank is exact in all of them); they differ in the precision of
# the hash operands and of the rows the re-rank reads first.
FORMS = {
    "fp32": {"hash_storage": "fp32", "rerank_storage": "fp32",
             "arith": {"hash": "fp32 mfma + fp64 sign fix-up", "scan": "u32 xor/popcount",
                       "rerank": "fp64 (exact products of fp32 rows)"}},
    "fp8_bf16": {"hash_storage": "fp8", "rerank_storage": "bf16",
                 "arith": {"hash": "fp8 e4m3 mfma (fp32 accumulate), margin re-check in fp32 + fp64",
                           "scan": "u32 xor/popcount",
                           "rerank": "fp64 sums of bf16 rows (bounded), exact fp64 re-check from fp32 rows"}},
    "bf16_hash": {"hash_storage": "bf16", "rerank_storage": "fp32",
                  "arith": {"hash": "bf16 mfma (fp32 accumulate), margin re-check in fp32 + fp64",
                            "scan": "u32 xor/popcount", "rerank": "fp64 (exact products of fp32 rows)"}},
    "fp8_hash": {"hash_storage": "fp8", "rerank_storage": "fp32",
                 "arith": {"hash": "fp8 e4m3 mfma (fp32 accumulate), margin re-check in fp32 + fp64",
                           "scan": "u32 xor/popcount", "rerank": "fp64 (exact products of fp32 rows)"}},
}
# headline form first, then the forms it is compared with
DEFAULT_FORMS = {"large": "fp8_bf16,fp32", "precision": "fp32,bf16_hash,fp8_hash", "mf": "fp32",
                 "tiny": "fp32"}
KERNELS = ["keys", "sort", "layout", "quant", "hash", "hash_rehash", "hash_fixup", "table", "qhash",
           "scan_sample", "guess", "scan_collect", "filter",
           "scan_hist", "threshold", "tie_locate", "scan_emit", "table_count", "table_emit",
           "order", "rerank", "head_theta", "head_screen", "rerank_lp", "screen_max", "screen", "rerank_exact"]
BUILD_KERNELS = {"keys", "sort", "layout", "quant", "hash", "hash_rehash", "hash_fixup", "table"}
INT_VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes per clock x 2.4 GHz
INT8_MFMA_PEAK_TOPS = 5000.0                    # dense int8 matrix-core peak, TOP/s
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4            # wave-wide vector instructions per second


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["tiny", "mf", "precision", "large", "batching"])
    ap.add_argument("--forms", default=None,
                    help="comma list of forms to time, headline first (" + ", ".join(FORMS) + ")")
    ap.add_argument("--budget", type=int, default=None,
                    help="probe budget T of the timed steps (default: the workload's stated budget)")
    ap.add_argument("--query-batch", type=int, default=None,
                    help="queries per nrlsh_query call (default 4096 for large, else all at once)")
    ap.add_argument("--extra-batches", default=None,
                    help="comma list of other batch sizes timed for the headline form (large: 1024,256)")
    ap.add_argument("--recall-queries", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="queries the oracle baseline times (default 64 for large, 256 otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the labelled T = n (exact MIPS) timing")
    ap.add_argument("--rerank", default="auto", choices=["auto", "gather", "screen", "screen_fp32", "screen_bf16x3"],
                    help="re-rank mode (all give identical results)")
    ap.add_argument("--margin", default="rigorous",
                    help="'rigorous' or a relative margin for the low-precision hash")
    ap.add_argument("--nq", type=int, default=None, help="override the number of queries")
    ap.add_argument("--variants", default="",
                    help="labelled variants timed after the headline, each at its own recall-0.9 "
                         "budget: eps:E (adjusted metric), uniform (norm ranges), bits (paper's "
                         "code-bit accounting), m:M (sub-datasets), per_subset (independent "
                         "projections per sub-dataset); combine with '+'")
    ap.add_argument("--probe", default="scan", choices=["scan", "table"],
                    help="how the timed steps find the probed items: linear scan of the codes, "
                         "or the bucket tables (hash lookup, Section 3.3)")
    ap.add_argument("--probe-sweep", default="", metavar="L,...",
                    help="time query batches of 1, 16 and 256 queries at budgets 100, 1000, 10000 "
                         "with both probes, on indexes of these code lengths")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a MIB-MiB buffer 3 times before the steps (a kernel of known "
                         "traffic that scales hardware byte counters)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the untimed recall sweep; used under a profiler so that only "
                         "timed-step kernels are launched")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1809_08782_amd as nr
    from workloads import PRESETS

    if args.workload == "batching":
        run_batching(args)
        return

    w = PRESETS[args.workload]()
    if args.nq is not None:
        w.nq = args.nq
    large = args.workload == "large"
    forms = [f.strip() for f in (args.forms or DEFAULT_FORMS[args.workload]).split(",") if f.strip()]
    for f in forms:
        if f not in FORMS:
            ap.error(f"unknown form {f}")
    qb = args.query_batch or (4096 if large else w.nq)
    extra_batches = [int(v) for v in (args.extra_batches if args.extra_batches is not None
                                      else ("1024,256" if large else "")).split(",") if v.strip()]
    cpu_sample = args.cpu_sample or (64 if large else 256)
    margin = args.margin if args.margin == "rigorous" else float(args.margin)
    T_op = args.budget or w.budgets[0]
    Tq = min(T_op, w.n)
    torch.cuda.set_device(0)
    log(f"workload {w.name}: n={w.n} d={w.d} m={w.m} L={w.L} nq={w.nq} k={w.k} T={T_op} "
        f"batch={qb} forms={forms}")
    t0 = time.perf_counter()
    X = w.items()
    Q = w.queries()
    log(f"generated inputs in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    ids_buf = torch.empty((w.nq, w.k), dtype=torch.int64, device="cuda")
    ips_buf = torch.empty((w.nq, w.k), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    norms = torch.linalg.vector_norm(Xd, dim=1).double()
    med = float(norms.median())
    norm_stats = {"max_over_median": float(norms.max()) / med,
                  "p999_over_median": float(torch.quantile(norms[:1_000_000].float(), 0.999)) / med}
    del norms

    # ------------------------------------------------------------ recall curve
    # every form returns the same top-k, so one (plain) index serves the curve;
    # recall@k against exact MIPS on the first `recall_queries` queries
    nrec = min(args.recall_queries, w.nq)
    curve, curve10 = {}, {}
    gt = None
    T_09 = None
    if not args.no_sweep:
        gt = ground_truth(Xd, Qd[:nrec], w.k)
        sweep = sorted({*(1 << e for e in range(8, 21) if (1 << e) < w.n), w.n, *w.budgets, T_op})
        with nr.nrlsh_build(Xd, w.m, w.L, w.index_seed) as ix:
            for T in sweep:
                ids, _ = nr.nrlsh_query(ix, Qd[:nrec], w.k, T, rerank=args.rerank)
                got = ids.cpu().numpy()
                curve[T] = recall(got, gt)
                curve10[T] = recall(got[:, :10], gt[:, :10])
                log(f"recall@{w.k} T={T}: {curve[T]:.4f} (recall@10 {curve10[T]:.4f})")
                if T_09 is None and curve10[T] >= 0.9:
                    T_09 = T

    if args.copy_calibration > 0:
        # an elementwise copy (reads B, writes B) of B = MIB MiB: a kernel of
        # known traffic for the byte counters
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: fill + 3 elementwise copies of {args.copy_calibration} MiB")
        del src, dst

    # ------------------------------------------------------------ timed steps
    # one step = the whole path: index build over all n items, then every
    # query in batches of qb at budget T.  HIP events on the library's stream
    # (torch's current stream, which the library is given) split the step
    # into the build and the query phase.
    stream = torch.cuda.current_stream()

    def one_step(form, T, batch, nq):
        cfg = FORMS[form]
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        ix = nr.nrlsh_build(Xd, w.m, w.L, w.index_seed, hash_storage=cfg["hash_storage"], margin=margin,
                            bucket_tables=args.probe == "table")
        e1.record(stream)
        for b0 in range(0, nq, batch):
            b1 = min(nq, b0 + batch)
            nr.nrlsh_query(ix, Qd[b0:b1], w.k, T, out=(ids_buf[b0:b1], ips_buf[b0:b1]), rerank=args.rerank,
                           rerank_storage=cfg["rerank_storage"], probe=args.probe)
        e2.record(stream)
        torch.cuda.synchronize()
        bst = ix.build_stats()
        ix.close()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), bst

    def timed(form, T, batch, nq, steps, warmup, profile=False):
        for i in range(warmup):
            one_step(form, T, batch, nq)
            log(f"  [{form}] T={T} batch={batch} warmup {i + 1}/{warmup} done")
        nr.nrlsh_profile_reset()
        nr.nrlsh_profile_enable(profile)
        b_ms, q_ms, walls = [], [], []
        bst = None
        for i in range(steps):
            t = time.perf_counter()
            b, q, bst = one_step(form, T, batch, nq)
            walls.append(time.perf_counter() - t)
            b_ms.append(b)
            q_ms.append(q)
            log(f"  [{form}] T={T} batch={batch} step {i + 1}/{steps}: build {b:.2f} ms, query {q:.2f} ms")
        nr.nrlsh_profile_enable(False)
        kern = {}
        if profile:
            for nm in KERNELS:
                ms, cnt = nr.nrlsh_profile_get(nm)
                if cnt:
                    kern[nm] = {"avg_ms": ms / cnt, "launches_per_step": cnt / steps,
                                "ms_per_step": ms / steps}
        return {"build_ms": sum(b_ms) / steps, "query_ms": sum(q_ms) / steps,
                "wall_ms": sum(walls) / steps * 1e3, "qps": nq / (sum(q_ms) / steps * 1e-3),
                "build_stats": bst, "kernels": kern, "query_stats": nr.nrlsh_get_query_stats()}

    results = {}
    head = forms[0]
    for form in forms:
        r = timed(form, T_op, qb, w.nq, args.steps, args.warmup)
        if form == head:
            ids_op = ids_buf.clone()
            ips_op = ips_buf.clone()
        else:
            same = bool(torch.equal(ids_buf, ids_op) and torch.equal(ips_buf, ips_op))
            r["identical_to_" + head] = same
            log(f"[{form}] identical top-k to {head}: {same}")
        # per-kernel split from a separate profiled run (event pairs per launch)
        pr = timed(form, T_op, qb, w.nq, max(1, args.steps // 2), 0, profile=True)
        r["kernels"] = pr["kernels"]
        r["hashed_items_per_s"] = (w.n / (pr["kernels"]["hash"]["avg_ms"] * 1e-3)
                                   if "hash" in pr["kernels"] else None)
        r["built_items_per_s"] = w.n / (r["build_ms"] * 1e-3)
        results[form] = r
        log(f"[{form}] T={T_op}: query {r['query_ms']:.2f} ms ({r['qps']:.4g} q/s), build "
            f"{r['build_ms']:.2f} ms; kernels {json.dumps({k: round(v['ms_per_step'], 3) for k, v in r['kernels'].items()})}")
    hr = results[head]

    batches = []
    for b in extra_batches:
        r = timed(head, T_op, b, w.nq, 1, 1)
        batches.append({"batch": b, "query_ms": r["query_ms"], "qps": r["qps"]})
        log(f"[{head}] batch {b}: {r['qps']:.4g} q/s")

    # exact MIPS: a budget covering every item (the path then skips the scan)
    exact = None
    if not args.no_exact and T_op < w.n:
        ne = min(w.nq, 16384)
        r = timed("fp32", w.n, min(qb, ne) if large else ne, ne, 1, 1)
        exact = {"T": w.n, "nq": ne, "query_ms": r["query_ms"], "qps": r["qps"], "recall@k": 1.0,
                 "label": "exact MIPS (T = n probes every item), plain FP32 index"}
        log(f"exact MIPS T=n: {r['qps']:.4g} q/s")

    # ------------------------------------------------------------ labelled variants
    variants = run_variants(args, w, Xd, Qd, gt, nrec, margin, ids_buf, ips_buf) if args.variants else []
    probe_sweep = run_probe_sweep(args, w, Xd, Qd) if args.probe_sweep else []

    # ------------------------------------------------------------ roofline
    kern = hr["kernels"]
    qkern = {k: v for k, v in kern.items() if k not in BUILD_KERNELS}
    dom = max(qkern, key=lambda nm: qkern[nm]["ms_per_step"]) if qkern else None
    roof, roofs = roofline(dom, kern, w, Tq, qb, hr["query_stats"])
    scan = None
    scan_kernel = "scan_collect" if "scan_collect" in kern else ("scan_hist" if "scan_hist" in kern else None)
    if scan_kernel:
        W = (w.L + 31) // 32
        st = hr["query_stats"]
        pairs = st.get("scan_pairs") or 0
        # the stats are the last query call's: the last batch, of nq - (calls - 1) qb queries
        last_nq = w.nq - (-(-w.nq // qb) - 1) * qb
        frac = pairs / (last_nq * w.n)
        per = kern[scan_kernel]
        step_pairs = frac * w.nq * w.n  # scanned pairs of the whole step, at the last batch's fraction
        # the two passes: XOR + popcount per code word and the histogram
        # address (1 op) per pair, on the vector ALUs; the collecting scan:
        # 32 W int8 multiply-adds per pair on the matrix cores (2 ops each)
        collect = scan_kernel == "scan_collect"
        ops = 64 * W if collect else 2 * W + 1
        scan = {"kernel": scan_kernel,
                "pairs_scanned_last_batch": pairs,
                "last_batch_queries": last_nq,
                "pairs_all_last_batch": last_nq * w.n,
                "scanned_fraction": frac,
                "scan_ms_per_step": per["ms_per_step"],
                "pairs_per_s": step_pairs / (per["ms_per_step"] * 1e-3) if pairs else None,
                "int_ops_per_pair": ops,
                "other_ms_per_step": {nm: kern[nm]["ms_per_step"] for nm in
                                      ("scan_sample", "guess", "threshold", "tie_locate", "filter",
                                       "scan_hist", "scan_emit") if nm in kern and nm != scan_kernel}}
        if scan["pairs_per_s"] and collect:
            scan["int8_mfma_tops"] = scan["pairs_per_s"] * ops / 1e12
            scan["int8_mfma_frac"] = scan["int8_mfma_tops"] / INT8_MFMA_PEAK_TOPS
        elif scan["pairs_per_s"]:
            scan["int_valu_tops"] = scan["pairs_per_s"] * ops / 1e12
            scan["int_valu_frac"] = scan["int_valu_tops"] / INT_VALU_PEAK_TOPS

    # ------------------------------------------------------------ CPU oracle baseline
    cpu = None
    if not args.no_cpu_baseline:
        import oracle.oracle as orc
        threads = max(1, min(16, os.cpu_count() or 1))
        S = min(cpu_sample, w.nq)
        t = time.perf_counter()
        oix = orc.OracleIndex(X, w.m, w.L, w.index_seed, threads=threads)
        tb = time.perf_counter() - t
        t = time.perf_counter()
        oids, oips = oix.query(Q[:S], w.k, T_op, threads=threads)
        tq = time.perf_counter() - t
        oix.close()
        gpu_ids = ids_op[:S].cpu().numpy()
        gpu_ips = ips_op[:S].cpu().numpy()
        cpu = {"value": S / tq, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"{S} of {w.nq} queries at T={T_op} on {threads} threads ({tq:.1f}s), "
                         f"after a full oracle build of the {w.n} items ({tb:.1f}s, not counted)",
               "build_s": tb, "build_items_per_s": w.n / tb, "query_s_per_query": tq / S,
               "gpu_topk_equals_oracle_on_sample": bool(np.array_equal(gpu_ids, oids)),
               "gpu_ips_equal_oracle_on_sample": bool(np.array_equal(gpu_ips, oips.astype(np.float32)))}
        log(f"cpu baseline {json.dumps(cpu)}")

    rec_T = curve.get(T_op)
    out = {
        "metric": "queries/sec at recall@10>=0.9 (plain FP32 vs BF16/FP8); scan+rerank HBM GB/s",
        "value": hr["qps"],
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hr["wall_ms"],
        "query_ms_per_step": hr["query_ms"],
        "build_ms_per_step": hr["build_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32+f64",
        "arith": FORMS[head]["arith"],
        "data": "synthetic",
        "config": {**w.describe(), "T": T_op, "form": head, "query_batch": qb,
                   "op_point": ("stated budget; recall@10 >= 0.9 is first reached at T = %s" % T_09)
                   if T_09 is not None else "stated budget (recall@10 >= 0.9 not reached by the sweep)",
                   "rerank": args.rerank, "margin": args.margin, "probe": args.probe,
                   "parallelism": "single GPU"},
        "value_definition": "queries / query-phase time (HIP events on the library stream, inputs "
                            "resident in HBM); the index build of every step is timed apart "
                            "(build_ms_per_step, hashed_items_per_s)",
        "recall_at_T": rec_T,
        "recall10_at_T": curve10.get(T_op),
        "recall_0_9_budget": T_09,
        "recall_curve": {str(k): v for k, v in curve.items()},
        "recall10_curve": {str(k): v for k, v in curve10.items()},
        "forms": {f: {kk: vv for kk, vv in r.items() if kk != "kernels"} for f, r in results.items()},
        "kernels": kern,
        "hashed_items_per_s": hr["hashed_items_per_s"],
        "built_items_per_s": hr["built_items_per_s"],
        "other_batches": batches,
        "exact_mips": exact,
        "norm_stats": norm_stats,
        "roofline": roof,
        "rooflines": roofs,
        "scan": scan,
        "variants": variants,
        "probe_sweep": probe_sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def kernel_roof(nm, kern, w, Tq, qb, qstats):
    """Roofline entry of one query kernel: its algorithmic work per launch
    (or per step) over its HIP-event time, against the peak of the unit that
    bounds it, plus the HBM traffic of a committed counter record when its
    sources are unchanged."""
    per = kern[nm]
    launches = per["launches_per_step"]
    nq_launch = w.nq / launches
    W = (w.L + 31) // 32
    S = next(v for v in (1, 2, 4, 8, 16) if v * 64 >= w.k or v == 16)  # top-k registers per lane
    # the stats are the last query call's: the last batch, of nq - (calls - 1) qb queries
    last_nq = w.nq - (-(-w.nq // qb) - 1) * qb

    def with_traffic(d, kname):
        rec = traffic_record(kname, w.name, Tq, nm)
        # counters were taken on full batches: bytes per query x this run's queries per launch
        d["traffic"] = ((rec["fetch_bytes_per_query"] + rec["write_bytes_per_query"]) * nq_launch) if rec else None
        d["traffic_source"] = rec
        return d

    if nm in ("rerank", "rerank_lp", "rerank_exact"):
        # per re-ranked item: its row (4d FP32 / 2d bf16 bytes) and stored
        # position (4); the FP32 passes also read its original id (4), the
        # bf16 pass the row's error bound (4) instead (its top-k of lower
        # bounds needs no ids).  The FP32 pass reads every probed item, the
        # bf16 pass every gathered one (all probed items less those of a
        # dense head), the exact pass after it the kept ones.
        row = 2 * w.d if nm == "rerank_lp" else 4 * w.d
        if nm == "rerank":
            items = nq_launch * Tq
        elif nm == "rerank_lp":
            items = (qstats.get("lp_gathered_total") or 0) / max(1, last_nq) * nq_launch
        else:
            items = (qstats.get("lp_kept_total") or 0) / max(1, last_nq) * nq_launch
        bytes_launch = items * (row + 8)
        achieved = bytes_launch / (per["avg_ms"] * 1e-3) / 1e9
        kname = ("k_rerank_bf16<%d>" if nm == "rerank_lp" else "k_rerank<%d>") % S
        return with_traffic({"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": bytes_launch,
                             "unit_work": "re-ranked item", "bytes_per_unit": row + 8,
                             "units_per_launch": items}, kname)
    if nm in ("scan_hist", "scan_emit", "scan_collect"):
        # pairs of the step from the last batch's scanned fraction, over the
        # kernel's time per step
        frac = (qstats.get("scan_pairs") or 0) / (last_nq * w.n)
        if nm == "scan_emit" or frac == 0:
            frac = 1.0
        mx = nm == "scan_collect"
        ops_per_pair = 64 * W if mx else 2 * W + 1
        peak = INT8_MFMA_PEAK_TOPS if mx else INT_VALU_PEAK_TOPS
        ops_step = frac * w.nq * w.n * ops_per_pair
        achieved = ops_step / (per["ms_per_step"] * 1e-3) / 1e12
        kname = {"scan_hist": "k_scan_hist_s<%d>", "scan_emit": "k_scan_emit_s<%d>",
                 "scan_collect": "k_scan_collect_mx<%d>"}[nm] % W
        d = with_traffic({"kernel": kname, "bound": "mfma" if mx else "alu", "achieved": achieved,
                          "peak": peak, "unit": "TOP/s", "frac": achieved / peak, "ops_per_step": ops_step,
                          "unit_work": "(query, item) pair", "ops_per_unit": ops_per_pair}, kname)
        # the vector instructions around the products bound it: their issue
        # rate (committed SQ_INSTS_VALU per query x queries per launch over
        # the launch's time) against one wave-wide instruction per 4 cycles
        # per SIMD (256 CUs x 4 SIMDs x 2.4 GHz / 4)
        sq = traffic_record(kname, w.name, Tq, nm, tag="sq_record")
        if sq:
            insts = sq["valu_insts_per_query"] * nq_launch
            rate = insts / (per["avg_ms"] * 1e-3)
            d["valu_issue"] = {"insts_per_launch": insts, "per_s": rate, "peak_per_s": VALU_ISSUE_PEAK,
                               "frac": rate / VALU_ISSUE_PEAK, "source": sq}
        return d
    if nm == "head_screen":
        # the keep pass of the dense head: one bf16 product (2d flops) per
        # (query, item) pair it evaluates (tiles skip the chunks none of their
        # queries probes), per query of the last call x queries per launch
        pairs = (qstats.get("dense_head_pairs") or 0) / max(1, last_nq) * nq_launch
        flops = 2.0 * w.d * pairs
        achieved = flops / (per["avg_ms"] * 1e-3) / 1e12
        kname = "k_screen1<%d>" % W
        d = with_traffic({"kernel": kname, "bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFS,
                          "unit": "TFLOP/s", "frac": achieved / BF16_MFMA_PEAK_TFS, "flops_per_launch": flops,
                          "unit_work": "(query, item) pair of the dense head", "flops_per_unit": 2.0 * w.d,
                          "units_per_launch": pairs}, kname)
        sq = traffic_record(kname, w.name, Tq, nm, tag="sq_record")
        if sq:
            insts = sq["valu_insts_per_query"] * nq_launch
            rate = insts / (per["avg_ms"] * 1e-3)
            d["valu_issue"] = {"insts_per_launch": insts, "per_s": rate, "peak_per_s": VALU_ISSUE_PEAK,
                               "frac": rate / VALU_ISSUE_PEAK, "source": sq}
        return d
    if nm == "screen":
        pairs = (qstats.get("screen_pairs") or 0) / max(1, qstats.get("screen_passes") or 1)
        flops = 2.0 * w.d * pairs
        achieved = flops / (per["avg_ms"] * 1e-3) / 1e12
        return {"kernel": "k_screen1<%d>" % W, "bound": "mfma", "achieved": achieved,
                "peak": BF16_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": achieved / BF16_MFMA_PEAK_TFS,
                "traffic": None, "flops_per_launch": flops, "unit_work": "evaluated pair"}
    return None


def roofline(dom, kern, w, Tq, qb, qstats):
    """Roofline of the dominant query kernel (the largest share of the step),
    and of every query kernel with a work model, largest first."""
    if dom is None:
        return None, []
    qk = sorted((nm for nm in kern if nm not in BUILD_KERNELS), key=lambda nm: -kern[nm]["ms_per_step"])
    rows = []
    for nm in qk:
        r = kernel_roof(nm, kern, w, Tq, qb, qstats)
        if r is not None:
            r["timer"] = nm
            r["ms_per_step"] = kern[nm]["ms_per_step"]
            r["avg_ms"] = kern[nm]["avg_ms"]
            rows.append(r)
    top = kernel_roof(dom, kern, w, Tq, qb, qstats)
    if top is None:
        top = {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
               "traffic": None}
    top["dominant_kernel"] = dom
    return top, rows


def run_variants(args, w, Xd, Qd, gt, nrec, margin, ids_buf, ips_buf):
    """The same step under the paper's other settings, each at its own
    recall-0.9 budget: the adjusted metric (Section 3.3), uniform norm ranges
    (Section 5), the paper's code-bit accounting (Section 4), other sub-dataset
    counts (Figure 3b's sweep) and independent projections per sub-dataset."""
    import torch

    import paper_1809_08782_amd as nr
    out = []
    budgets_sweep = sorted({*(1 << e for e in range(8, 40) if (1 << e) < w.n), w.n, *w.budgets})
    for v in [v.strip() for v in args.variants.split(",") if v.strip()]:
        cfg = {"label": v, "eps": 0.0, "partition": "percentile", "m": w.m, "L": w.L,
               "projections": "shared"}
        for part in v.split("+"):
            if part.startswith("eps:"):
                cfg["eps"] = float(part[4:])
            elif part == "uniform":
                cfg["partition"] = "uniform"
            elif part.startswith("m:"):
                cfg["m"] = int(part[2:])
            elif part == "per_subset":
                cfg["projections"] = "per_subset"
            elif part != "bits":
                raise SystemExit(f"unknown variant {v}")
        if "bits" in v.split("+"):
            cfg["L"] = w.L - (math.ceil(math.log2(cfg["m"])) if cfg["m"] > 1 else 0)
        ex = nr.nrlsh_build(Xd, cfg["m"], cfg["L"], w.index_seed, margin=margin, eps=cfg["eps"],
                            partition=cfg["partition"], projections=cfg["projections"])
        vcurve, vT = {}, None
        for T in budgets_sweep:
            ids, _ = nr.nrlsh_query(ex, Qd[:nrec], w.k, T)
            r = recall(ids.cpu().numpy(), gt)
            vcurve[str(T)] = r
            if vT is None and r >= 0.9:
                vT = T
        vT = vT or w.n
        nr.nrlsh_query(ex, Qd, w.k, vT, out=(ids_buf, ips_buf))
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = max(2, args.steps // 2)
        for _ in range(reps):
            nr.nrlsh_query(ex, Qd, w.k, vT, out=(ids_buf, ips_buf))
        torch.cuda.synchronize()
        est = (time.perf_counter() - t) / reps
        ex.close()
        out.append({**cfg, "T": vT, "frac_of_n": vT / w.n, "recall_at_T": vcurve.get(str(vT)),
                    "qps_query_only": w.nq / est, "query_ms": est * 1e3, "recall_curve": vcurve})
        log(f"variant {v}: m={cfg['m']} L={cfg['L']} T_op={vT} recall {vcurve.get(str(vT))} "
            f"query {est * 1e3:.2f} ms")
    return out


def run_probe_sweep(args, w, Xd, Qd):
    """Query-only latency of the two probes (same probed set, same results):
    small batches and budgets are where the bucket tables can skip the scan."""
    import torch

    import paper_1809_08782_amd as nr
    out = []
    for Ls in [int(v) for v in args.probe_sweep.split(",") if v.strip()]:
        with nr.nrlsh_build(Xd, w.m, Ls, w.index_seed, bucket_tables=True) as tx:
            for nqs in (1, 16, 256):
                for T in (100, 1000, 10000):
                    row = {"L": Ls, "nq": nqs, "T": T}
                    ref = None
                    for probe in ("scan", "table"):
                        qs = Qd[:nqs]
                        ids, _ = nr.nrlsh_query(tx, qs, w.k, T, rerank="gather", probe=probe)
                        st = nr.nrlsh_get_query_stats()
                        torch.cuda.synchronize()
                        reps = 10
                        t = time.perf_counter()
                        for _ in range(reps):
                            nr.nrlsh_query(tx, qs, w.k, T, rerank="gather", probe=probe)
                        torch.cuda.synchronize()
                        row[probe + "_ms"] = (time.perf_counter() - t) / reps * 1e3
                        if probe == "table":
                            row["lookups_per_query"] = st["table_lookups"] / nqs
                            row["walked_per_query"] = st["table_walked"] / nqs
                            row["same_result"] = bool(torch.equal(ids, ref))
                        ref = ids
                    out.append(row)
                    log(f"probe L={Ls} nq={nqs} T={T}: scan {row['scan_ms']:.3f} ms, table "
                        f"{row['table_ms']:.3f} ms")
    return out


if __name__ == "__main__":
    main()
