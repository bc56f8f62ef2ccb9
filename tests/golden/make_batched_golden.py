"""Write the oracle's per-update results for a sample of the first batch of
the batched-queries workload (the mid R-MAT graph, 2^20 vertices, 64
standing queries of 4..12 vertices, 10^4 updates), for every query:
batched_rmat20_batch0.json.

Only the oracle (O2, oracle/plain.c) and the input generators run here.
Attribution follows the order rule after Algorithm 1 (Sec. IV-C): every
incremental match belongs to its minimum-ord batch edge.  For each query
(registered in order, so its id is its index: the id enters the checksum),
O2 searches the canonical updates with ord % MOD == 0 under two per-seed
caps: a seed with more than `cap` matches is given up (its true count is
only known to exceed `cap`), and so is one whose search examines more than
`scan_cap` neighbour-list entries (its true count is only known to be at least
what it had found); every other sampled seed's figures are exact.
The file records the inputs' SHA-256 (graph, labels, batch, every query),
the canonical batch's SHA-256, and per query:

  nonzero    [ord, count, sum-hash, xor-hash] of every exact sampled seed with matches
  over_cap   sampled ords given up at the match cap (count > cap)
  work_cap   [ord, found] of sampled ords given up at the scan cap (count >= found)
Every other sampled ord has no incremental match of that query.

Usage: python tests/golden/make_batched_golden.py [--cap N] [--scan-cap N] [--mod M] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import plain as O2  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "batched_rmat20_batch0.json")


def input_fingerprints(w, b) -> dict:
    g = w.graph
    ql = np.concatenate([np.asarray(q.labels, np.uint32) for q in w.queries])
    qe = np.concatenate([np.asarray(q.edges, np.uint32).reshape(-1) for q in w.queries])
    qk = np.asarray([q.k for q in w.queries] + [q.m for q in w.queries], np.uint32)
    return {
        "row_ptr": W.fingerprint(g.row_ptr), "col": W.fingerprint(g.col), "labels": W.fingerprint(g.labels),
        "batch_src": W.fingerprint(b.src), "batch_dst": W.fingerprint(b.dst), "batch_op": W.fingerprint(b.op),
        "query_sizes": W.fingerprint(qk), "query_labels": W.fingerprint(ql), "query_edges": W.fingerprint(qe),
    }


def canonical_fingerprint(lo, hi, sign) -> str:
    return W.fingerprint(np.concatenate([np.asarray(lo, np.uint32), np.asarray(hi, np.uint32),
                                         np.asarray(sign, np.uint32)]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cap", type=int, default=20000)
    ap.add_argument("--scan-cap", type=int, default=200000000)
    ap.add_argument("--mod", type=int, default=1)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t0 = time.time()
    w = W.batched_queries()
    b = w.batches[0]
    print("generated in %.1f s" % (time.time() - t0), flush=True)
    recs, canon = [], None
    for qi, q in enumerate(w.queries):
        r = O2.run(w.graph, q, b, qid=qi, threads=args.threads, sample_mod=args.mod, sample_rem=0,
                   want_tuples=False, seed_cap=args.cap, scan_cap=args.scan_cap)
        assert r.status == 0
        c = canonical_fingerprint(r.canon_lo, r.canon_hi, r.canon_sign)
        assert canon is None or c == canon
        canon = c
        idx = np.arange(0, r.n_canonical, args.mod)
        flag = r.seed_incomplete[idx]
        inc = r.seed_incomplete.astype(bool)
        nz = idx[(r.seed_count[idx] > 0) & ~inc[idx]]
        recs.append({
            "qid": qi, "kind": q.kind, "k": q.k,
            "nonzero": [[int(i), int(r.seed_count[i]), str(int(r.seed_hsum[i])), str(int(r.seed_hxor[i]))]
                        for i in nz.tolist()],
            "over_cap": [int(i) for i in idx[flag == 1].tolist()],
            "work_cap": [[int(i), int(r.seed_count[i])] for i in idx[flag == 2].tolist()],
            "oracle_seconds": round(r.seconds, 2),
        })
        print("q%-2d %-6s k=%-2d: %d sampled ords with matches (%d matches), %d over the cap, %d over the scan cap, "
              "%.1f s" % (qi, q.kind, q.k, len(nz), int(r.seed_count[nz].sum()), int((flag == 1).sum()),
                          int((flag == 2).sum()), r.seconds), flush=True)
    rec = {
        "cite": "Sec. II-A (the incremental matches of a batch) and the order rule after Algorithm 1 "
                "(Sec. IV-C): per canonical update, the matches whose minimum-ord batch edge it is",
        "written_by": "tests/golden/make_batched_golden.py (the oracle O2 only)",
        "workload": w.name, "batch": 0, "n_queries": len(w.queries),
        "inputs": input_fingerprints(w, b),
        "n_canonical": int(r.n_canonical),
        "canonical": canon,
        "mod": args.mod, "cap": args.cap, "scan_cap": args.scan_cap,
        "queries": recs,
    }
    with open(PATH, "w") as fh:
        json.dump(rec, fh, indent=0)
        fh.write("\n")
    print("written %s in %.0f s" % (PATH, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
