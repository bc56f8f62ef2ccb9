"""Benchmark: batch-dynamic subgraph matching on one MI355X.

One step = one update batch through the whole path (canonicalise, merge,
filter refresh, seeds, search, commit, results to the host), on a fresh batch
of the workload's stream each step, with the graph resident on the device.

Prints one JSON line:
  metric    incremental matches/s and updates/s on 1 MI355X; p50/p99 batch latency
  value     incremental matches per second over the timed steps (+ and - results)
  roofline  the search kernel (the dominant kernel): algorithmic bytes per
            launch / its average duration (HIP events on the library stream)
  cpu_baseline  the CPU oracle (O2) on a bounded sample of the same batch

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mid|large|tiny]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def percentile(xs, p):
    import numpy as np
    return float(np.percentile(np.array(xs, dtype=float), p)) if xs else 0.0


def cpu_baseline(w, budget_s: float = 20.0):
    """Time the oracle on a deterministic 1-in-M sample of the first batch's
    seeds (by canonical ord), shrinking M until the run takes a few seconds."""
    from oracle import plain as O2
    threads = min(os.cpu_count() or 1, 16)
    g, b = w.graph, w.batches[0]
    M = 2048
    best = None
    spent = 0.0
    while M >= 1:
        tot_matches, tot_s, n_seeds = 0, 0.0, 0
        for qi, q in enumerate(w.queries):
            r = O2.run(g, q, b, qid=qi, threads=threads, sample_mod=M, sample_rem=0, want_tuples=False)
            tot_matches += r.count[0] + r.count[1]
            tot_s += r.seconds
            n_seeds = len(range(0, r.n_canonical, M))
        spent += tot_s
        best = (tot_matches, tot_s, M, n_seeds)
        if tot_s >= budget_s / 4 or M == 1 or spent + 4 * tot_s > budget_s * 1.5:
            break
        M //= 4
    matches, secs, M, n_seeds = best
    return {
        "value": (matches / secs) if secs > 0 else 0.0,
        "unit": "matches/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "first batch, seeds with canonical ord %% %d == 0 (%d of %d updates), all queries; "
                  "%d matches in %.2f s including the oracle's own graph update" % (
                      M, n_seeds, len(b), matches, secs),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mid", choices=["tiny", "mid", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-steal", action="store_true")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import workloads as W
    from paper_2401_17018_amd import Context

    n_batches = args.warmup + args.steps
    t0 = time.time()
    if args.workload == "mid":
        w = W.mid(n_batches=n_batches)
    elif args.workload == "large":
        w = W.large(n_batches=n_batches)
    else:
        w = W.tiny()
        w.batches = w.batches * n_batches if n_batches > 1 else w.batches
    gen_s = time.time() - t0
    print("[bench] workload %s generated in %.1fs: n=%d m=%d queries=%s batches=%d" % (
        w.name, gen_s, w.graph.n, w.graph.m, [q.k for q in w.queries], len(w.batches)), file=sys.stderr, flush=True)

    ctx = Context(device=0, steal=not args.no_steal, waves_per_cu=args.waves_per_cu)
    t0 = time.time()
    ctx.load_graph(w.graph.row_ptr, w.graph.col, w.graph.labels)
    load_s = time.time() - t0
    for q in w.queries:
        ctx.register_query(q.k, q.labels, q.edges)
    print("[bench] graph loaded in %.2fs" % load_s, file=sys.stderr, flush=True)

    batches = w.batches
    if args.workload == "tiny":
        # the tiny stream repeats one insert-only batch: alternate it with its inverse
        batches = [w.batches[0] if i % 2 == 0 else w.batches[0].inverse() for i in range(n_batches)]
    for i in range(args.warmup):
        b = batches[i]
        r = ctx.apply_batch(b.src, b.dst, b.op, hash=True)
        print("[bench] warmup %d: %.1f ms, matches %d" % (i, r.stats["ms_total"], int(r.counts.sum())),
              file=sys.stderr, flush=True)

    lat, upd, mat, dfs_ms, dfs_bytes, stats = [], 0, 0, [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        b = batches[args.warmup + i]
        t1 = time.perf_counter()
        r = ctx.apply_batch(b.src, b.dst, b.op, hash=True)
        t2 = time.perf_counter()
        lat.append((t2 - t1) * 1e3)
        upd += r.stats["n_canonical"]
        mat += int(r.counts.sum())
        dfs_ms.append(r.stats["ms_dfs"])
        dfs_bytes.append(r.stats["bytes_alg_dfs"])
        stats.append(r.stats)
        print("[bench] step %d: %.1f ms (search %.1f ms), %d updates, %d matches, %d steals" % (
            i, lat[-1], r.stats["ms_dfs"], r.stats["n_canonical"], int(r.counts.sum()), r.stats["steals"]),
            file=sys.stderr, flush=True)
    t_total = time.perf_counter() - t_start
    ctx.close()

    avg_dfs_s = sum(dfs_ms) / len(dfs_ms) / 1e3
    avg_bytes = sum(dfs_bytes) / len(dfs_bytes)
    achieved = avg_bytes / avg_dfs_s / 1e9 if avg_dfs_s > 0 else 0.0
    phases = {k: round(sum(s[k] for s in stats) / len(stats), 3)
              for k in ("ms_canon", "ms_merge", "ms_filter", "ms_seed", "ms_dfs", "ms_commit", "ms_total")}
    out = {
        "metric": "incremental matches/s and updates/s on 1 MI355X; p50/p99 batch latency",
        "value": mat / t_total,
        "unit": "matches/s",
        "updates_per_s": upd / t_total,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded R-MAT / ER graphs, random-walk queries, generated update stream)",
        "config": {
            "workload": w.name,
            "vertices": w.graph.n,
            "edges": w.graph.m,
            "queries": [{"k": q.k, "edges": q.m, "kind": q.kind} for q in w.queries],
            "batch_updates": len(batches[args.warmup]),
            "mode": "counts + hash (every match enumerated)",
        },
        "phases_ms": phases,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_dfs",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_alg_per_launch": avg_bytes,
            "avg_launch_ms": avg_dfs_s * 1e3,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
