#!/usr/bin/env python3
"""Throughput of the norm-ranging LSH hot path on one MI355X.

One step = the whole path on one batch of synthetic input already resident in
HBM: index build (norm keys, radix sort, percentile partition, SimpleLSH
transform + SRP hash, rank table) over all n items, then the multi-probe query
(query hash, two-pass popcount scan with threshold, FP64 re-rank, top-k) of
all nq queries at probe budget T.  value = nq / step time.

The operating point T is the smallest power-of-two budget at which recall@k
(measured on the first 1000 queries against exact MIPS) reaches 0.9; the
stated budgets are timed as well and reported under "budgets".

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


def traffic_record(kernel, workload, T):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (profiles/*.md, a line "traffic_record: {json}"), provided the sources it
    names still hash to what they were when the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            lines = [ln for ln in f if ln.startswith("traffic_record: ")]
        for ln in lines:
            rec = json.loads(ln[len("traffic_record: "):])
            if rec.get("kernel") != kernel or rec.get("workload") != workload or rec.get("T") != T:
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mf", choices=["tiny", "mf", "precision", "large", "batching"])
    ap.add_argument("--budget", type=int, default=None, help="time this T instead of the recall-0.9 point")
    ap.add_argument("--recall-queries", type=int, default=1000)
    ap.add_argument("--cpu-sample", type=int, default=256, help="queries the oracle baseline times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rerank", default="auto", choices=["auto", "gather", "screen", "screen_fp32", "screen_bf16x3"],
                    help="re-rank mode (all give identical results)")
    ap.add_argument("--hash-storage", default="fp32", choices=["fp32", "bf16", "fp8"],
                    help="precision form of the hash GEMM")
    ap.add_argument("--margin", default="rigorous",
                    help="'rigorous' or a relative margin for the low-precision hash")
    ap.add_argument("--rerank-storage", default="fp32", choices=["fp32", "bf16"],
                    help="rows the gather re-rank reads first (bf16: bounded, then exact)")
    ap.add_argument("--nq", type=int, default=None, help="override the number of queries")
    ap.add_argument("--query-batch", type=int, default=0,
                    help="queries per nrlsh_query call (0: all in one call)")
    ap.add_argument("--no-budgets", action="store_true", help="skip timing the stated budgets")
    ap.add_argument("--variants",
                    default="eps:0.1,eps:0.2,eps:0.3,uniform,bits,uniform+bits,m:8,m:128,per_subset",
                    help="labelled variants timed after the headline, each at its own recall-0.9 "
                         "budget: eps:E (adjusted metric), uniform (norm ranges), bits (paper's "
                         "code-bit accounting), m:M (sub-datasets), per_subset (independent "
                         "projections per sub-dataset); combine with '+'; '' for none")
    ap.add_argument("--probe", default="scan", choices=["scan", "table"],
                    help="how the timed step finds the probed items: linear scan of the codes, "
                         "or the bucket tables (hash lookup, Section 3.3)")
    ap.add_argument("--probe-sweep", default="", metavar="L,...",
                    help="after the headline, time query batches of 1, 16 and 256 queries at "
                         "budgets 100, 1000, 10000 with both probes, on indexes of these code "
                         "lengths (e.g. '16,32'); '' for none")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a MIB-MiB buffer 3 times before the steps (a kernel of known "
                         "traffic that scales hardware byte counters)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the untimed recall sweep (needs --budget); used under a profiler so "
                         "that only timed-step kernels are launched")
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
    margin = args.margin if args.margin == "rigorous" else float(args.margin)
    torch.cuda.set_device(0)
    log(f"workload {w.name}: n={w.n} d={w.d} m={w.m} L={w.L} nq={w.nq} k={w.k}")
    t0 = time.perf_counter()
    X = w.items()
    Q = w.queries()
    log(f"generated inputs in {time.perf_counter() - t0:.1f}s")
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    ids_buf = torch.empty((w.nq, w.k), dtype=torch.int64, device="cuda")
    ips_buf = torch.empty((w.nq, w.k), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- recall sweep
    if args.no_sweep and args.budget is None:
        ap.error("--no-sweep needs --budget")
    nrec = min(args.recall_queries, w.nq)
    gt = ground_truth(Xd, Qd[:nrec], w.k) if not args.no_sweep else None
    curve = {}
    ix = nr.nrlsh_build(Xd, w.m, w.L, w.index_seed, hash_storage=args.hash_storage, margin=margin)
    norms = torch.linalg.vector_norm(Xd, dim=1).double()
    med = float(norms.median())
    norm_stats = {"max_over_median": float(norms.max()) / med,
                  "p999_over_median": float(torch.quantile(norms[:1_000_000].float(), 0.999)) / med}
    del norms
    budgets_sweep = sorted({*(1 << e for e in range(8, 40) if (1 << e) < w.n), w.n, *w.budgets})
    if args.no_sweep:
        budgets_sweep = []
    T_op = None
    for T in budgets_sweep:
        ids, _ = nr.nrlsh_query(ix, Qd[:nrec], w.k, T, rerank_storage=args.rerank_storage)
        r = recall(ids.cpu().numpy(), gt)
        curve[T] = r
        log(f"recall@{w.k} T={T}: {r:.4f}")
        if T_op is None and r >= 0.9 and (T & (T - 1) == 0 or T == w.n):
            T_op = T
    build_stats = ix.build_stats()
    ix.close()
    if args.budget is not None:
        T_op = args.budget
    if T_op is None:
        T_op = w.n

    if args.copy_calibration > 0:
        # a fill (writes B bytes) and an elementwise copy (reads B, writes B)
        # of B = MIB MiB: kernels of known traffic for the byte counters
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: fill + 3 elementwise copies of {args.copy_calibration} MiB")
        del src, dst

    # ---------------------------------------------------------------- timed steps
    qb = args.query_batch if args.query_batch > 0 else w.nq

    def step(T, eps=0.0):
        with nr.nrlsh_build(Xd, w.m, w.L, w.index_seed, hash_storage=args.hash_storage,
                            margin=margin, eps=eps, bucket_tables=args.probe == "table") as sx:
            for b0 in range(0, w.nq, qb):
                b1 = min(w.nq, b0 + qb)
                nr.nrlsh_query(sx, Qd[b0:b1], w.k, T, out=(ids_buf[b0:b1], ips_buf[b0:b1]),
                               rerank=args.rerank, rerank_storage=args.rerank_storage,
                               probe=args.probe)

    def timed(T, steps, warmup, profile, eps=0.0):
        for i in range(warmup):
            step(T, eps)
            log(f"  T={T} warmup {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        nr.nrlsh_profile_reset()
        nr.nrlsh_profile_enable(profile)
        t = time.perf_counter()
        for i in range(steps):
            step(T, eps)
            log(f"  T={T} step {i + 1}/{steps} done ({time.perf_counter() - t:.2f}s)")
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        nr.nrlsh_profile_enable(False)
        return el / steps

    names = ["keys", "sort", "layout", "quant", "hash", "hash_rehash", "hash_fixup", "table", "qhash",
             "scan_hist", "threshold", "tie_locate", "scan_emit", "table_count", "table_emit",
             "rerank", "rerank_lp", "screen_max", "screen", "rerank_exact"]
    # unprofiled timing for the headline, profiled run for the per-kernel split
    s_step = timed(T_op, args.steps, args.warmup, False)
    qstats = nr.nrlsh_get_query_stats()
    ids_op = ids_buf.clone()
    timed(T_op, max(2, args.steps // 2), 0, True)
    kern = {}
    for nm in names:
        ms, cnt = nr.nrlsh_profile_get(nm)
        if cnt:
            kern[nm] = {"avg_ms": ms / cnt, "launches_per_step": cnt / max(2, args.steps // 2)}
    log(f"T={T_op}: {s_step * 1e3:.2f} ms/step; kernels {json.dumps(kern)}")

    # at T >= n every item is probed, so the library runs no query hash, scan
    # or threshold; T = n - 1 probes all but one item and runs every step of
    # the path, which shows what that shortcut saves
    full_path = None
    if T_op >= w.n and w.n > 1 and not args.no_budgets:
        st = timed(w.n - 1, max(2, args.steps // 2), 1, True)
        fk = {}
        for nm in names:
            ms, cnt = nr.nrlsh_profile_get(nm)
            if cnt:
                fk[nm] = round(ms / max(2, args.steps // 2), 3)
        full_path = {"T": w.n - 1, "ms_per_step": st * 1e3, "qps": w.nq / st, "kernel_ms_per_step": fk}
        log(f"full path T={w.n - 1}: {st * 1e3:.2f} ms/step")

    budgets = []
    if not args.no_budgets:
        for T in w.budgets:
            st = timed(T, max(2, args.steps // 2), 1, True)
            bk = {}
            for nm in names:
                ms, cnt = nr.nrlsh_profile_get(nm)
                if cnt:
                    bk[nm] = round(ms / max(2, args.steps // 2), 3)
            budgets.append({"T": T, "frac_of_n": T / w.n, "qps": w.nq / st, "ms_per_step": st * 1e3,
                            "recall": curve.get(T), "query_stats": nr.nrlsh_get_query_stats(),
                            "kernel_ms_per_step": bk})
            log(f"budget T={T}: {st * 1e3:.2f} ms/step recall {curve.get(T)}")

    # ---------------------------------------------------------------- labelled variants
    # the same step under the paper's other settings, each at its own
    # recall-0.9 budget: the adjusted metric s_hat = U_j cos[pi (1 - eps)(1 - l/L)]
    # (Section 3.3), uniform norm ranges (Section 5), the paper's code-bit
    # accounting (ceil(log2 m) of the L bits spent on the sub-dataset id,
    # Section 4), other sub-dataset counts (Figure 3b's sweep) and
    # independent projections per sub-dataset (Algorithm 1 read literally)
    variants = []
    spec = [v.strip() for v in args.variants.split(",") if v.strip()] if not args.no_sweep else []
    for v in spec:
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
                ap.error(f"unknown variant {v}")
        if "bits" in v.split("+"):  # after m is known
            cfg["L"] = w.L - (math.ceil(math.log2(cfg["m"])) if cfg["m"] > 1 else 0)
        if cfg["projections"] != "shared" and args.hash_storage != "fp32":
            log(f"variant {v} skipped: per-subset projections need the FP32 hash")
            continue
        ex = nr.nrlsh_build(Xd, cfg["m"], cfg["L"], w.index_seed, hash_storage=args.hash_storage,
                            margin=margin, eps=cfg["eps"], partition=cfg["partition"],
                            projections=cfg["projections"])
        vcurve, vT = {}, None
        for T in budgets_sweep:
            ids, _ = nr.nrlsh_query(ex, Qd[:nrec], w.k, T)
            r = recall(ids.cpu().numpy(), gt)
            vcurve[str(T)] = r
            if vT is None and r >= 0.9 and (T & (T - 1) == 0 or T == w.n):
                vT = T
        ex.close()
        vT = vT or w.n

        def vstep(T, cfg=cfg):
            with nr.nrlsh_build(Xd, cfg["m"], cfg["L"], w.index_seed, hash_storage=args.hash_storage,
                                margin=margin, eps=cfg["eps"], partition=cfg["partition"],
                                projections=cfg["projections"]) as sx:
                nr.nrlsh_query(sx, Qd, w.k, T, out=(ids_buf, ips_buf), rerank=args.rerank,
                               rerank_storage=args.rerank_storage)
        vstep(vT)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = max(2, args.steps // 2)
        for _ in range(reps):
            vstep(vT)
        torch.cuda.synchronize()
        est = (time.perf_counter() - t) / reps
        variants.append({**cfg, "T": vT, "frac_of_n": vT / w.n, "recall_at_T": vcurve.get(str(vT)),
                         "qps": w.nq / est, "ms_per_step": est * 1e3, "recall_curve": vcurve})
        log(f"variant {v}: m={cfg['m']} L={cfg['L']} T_op={vT} recall {vcurve.get(str(vT))} "
            f"{est * 1e3:.2f} ms/step")

    # ---------------------------------------------------------------- probe sweep
    # query-only latency of the two probes (same probed set, same results):
    # small batches and budgets are where the bucket tables can skip the scan
    probe_sweep = []
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
                    probe_sweep.append(row)
                    log(f"probe L={Ls} nq={nqs} T={T}: scan {row['scan_ms']:.3f} ms, table "
                        f"{row['table_ms']:.3f} ms ({row['lookups_per_query']:.0f} lookups, "
                        f"{row['walked_per_query']:.0f} codes walked per query)")

    # ---------------------------------------------------------------- roofline
    Tq = min(T_op, w.n)
    dom = max(kern, key=lambda nm: kern[nm]["avg_ms"] * kern[nm]["launches_per_step"]) if kern else None
    roof = None
    if dom == "screen":
        # algorithmic work of one screen launch: the inner products of the
        # pairs it evaluates, 2d flop each on the bf16 (or FP32) matrix cores
        # (the bf16x3 screen forms each one from three bfloat16 products,
        # hi*hi + hi*lo + lo*hi, 3 x 2d flop).  The keep pass skips chunks no
        # query of a tile can keep (norm bound), so its pairs are the ones the
        # library reports evaluating, not all (queries x T) probed pairs.
        launches = kern["screen"]["launches_per_step"]
        probed_pairs = (w.nq / launches) * Tq
        passes = max(1, qstats.get("screen_passes") or 1)
        pairs = qstats.get("screen_pairs") / passes if qstats.get("screen_pairs") else probed_pairs
        smode = qstats.get("mode")
        products = {"screen": 1, "screen_bf16x3": 3}.get(smode, 1)
        b16 = smode in ("screen", "screen_bf16x3")
        flops = 2.0 * products * w.d * pairs
        peak = BF16_MFMA_PEAK_TFS if b16 else FP32_MFMA_PEAK_TFS
        achieved = flops / (kern["screen"]["avg_ms"] * 1e-3) / 1e12
        # the kernel the library launches: budgets covering every item take
        # the variants that read no codes (128-query tiles for rows of at
        # least 256 coordinates); otherwise one or two code words per item
        dp = (w.d + 7) // 8 * 8
        if Tq >= w.n and smode in ("screen", "screen_bf16x3"):
            kname = ("k_screen_b128" if dp >= 256 else "k_screen1<0>") if smode == "screen" \
                else "k_screen3<0, false, true>"
        else:
            kname = {"screen": "k_screen1<1>",
                     "screen_bf16x3": "k_screen3<1, false, true>"}.get(smode, "k_screen<1, false>")
            if w.L > 32:
                kname = kname.replace("<1", "<2")
        rec = traffic_record(kname, w.name, Tq)
        roof = {"kernel": kname, "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": (rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]) if rec else None,
                "traffic_source": rec, "mfma_dtype": "bf16" if b16 else "f32",
                "bf16_products_per_pair": products if b16 else None,
                "flops_per_launch": flops, "pairs_per_launch": pairs,
                "probed_pairs_per_launch": probed_pairs,
                "fp32_equivalent_tflops": 2.0 * w.d * pairs / (kern["screen"]["avg_ms"] * 1e-3) / 1e12,
                "dominant_kernel": dom}
    elif dom in ("rerank", "rerank_exact", "rerank_lp"):
        # algorithmic bytes per probed item: its row (4d), stored position and id (8)
        launches = kern[dom]["launches_per_step"]
        row_bytes = (2 if dom == "rerank_lp" else 4) * w.d
        per_launch_bytes = (w.nq / launches) * Tq * (row_bytes + 8)
        achieved = per_launch_bytes / (kern[dom]["avg_ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "bytes_per_launch": per_launch_bytes, "dominant_kernel": dom}

    # scan pass 1: effective code-stream rate (every query reads every code
    # once: nq n 4W bytes) and (query, item) pairs per second
    scan = None
    if "scan_hist" in kern:
        W = (w.L + 31) // 32
        per = kern["scan_hist"]
        qpl = w.nq / per["launches_per_step"]
        scan = {"pairs_per_s": qpl * w.n / (per["avg_ms"] * 1e-3),
                "code_stream_GBps": qpl * w.n * 4 * W / (per["avg_ms"] * 1e-3) / 1e9}

    # ---------------------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu_baseline:
        import oracle.oracle as orc
        threads = max(1, min(16, os.cpu_count() or 1))
        S = min(args.cpu_sample, w.nq)
        t = time.perf_counter()
        oix = orc.OracleIndex(X, w.m, w.L, w.index_seed, threads=threads)
        tb = time.perf_counter() - t
        t = time.perf_counter()
        oids, _ = oix.query(Q[:S], w.k, T_op, threads=threads)
        tq = time.perf_counter() - t
        est = tb + tq / S * w.nq
        gpu_ids = ids_op[:S].cpu().numpy()
        cpu = {"value": w.nq / est, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": f"full oracle build of all {w.n} items ({tb:.1f}s) + {S} of {w.nq} "
                         f"queries at T={T_op} ({tq:.1f}s); step time extrapolated to {w.nq} queries",
               "build_s": tb, "query_s_per_query": tq / S,
               "gpu_topk_equals_oracle_on_sample": bool(np.array_equal(gpu_ids, oids))}
        log(f"cpu baseline {json.dumps(cpu)}")

    out = {
        "metric": "queries/sec at recall@10>=0.9 (plain FP32 vs BF16/FP8); scan+rerank HBM GB/s",
        "value": w.nq / s_step,
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "arith": {"hash": "fp32 mfma + fp64 sign fix-up", "scan": "u32", "rerank": "f64"},
        "data": "synthetic",
        "config": {**w.describe(), "T": T_op, "op_point": "smallest power-of-two T with recall>=0.9"
                   if args.budget is None else "fixed T", "parallelism": "single GPU",
                   "hash_storage": args.hash_storage, "margin": args.margin,
                   "rerank": args.rerank, "rerank_storage": args.rerank_storage,
                   "probe": args.probe, "query_batch": qb},
        "recall_at_T": curve.get(T_op),
        "recall_curve": {str(k): v for k, v in curve.items()},
        "budgets": budgets,
        "full_path_at_n_minus_1": full_path,
        "kernels": kern,
        "hashed_items_per_s": (w.n / (kern["hash"]["avg_ms"] * 1e-3)) if "hash" in kern else None,
        "build_stats": build_stats,
        "query_stats": qstats,
        "norm_stats": norm_stats,
        "roofline": roof,
        "scan": scan,
        "variants": variants,
        "probe_sweep": probe_sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
