"""Write the oracle's per-update results for the first batch of the large
workload (R-MAT scale 24, 2^29 CSR entries, 10^5 updates), one file per
query: large_rmat24_<kind>_batch0.json.

Only the oracle (O2, oracle/plain.c) and the input generators run here.
Attribution follows the order rule after Algorithm 1 (Sec. IV-C): every
incremental match belongs to its minimum-ord batch edge.  O2 enumerates the
whole batch with a per-seed cap: a seed with more than `cap` matches is given
up (its true count is only known to exceed `cap`); every other seed's count
and checksums are exact.  The file records:

  inputs     SHA-256 of the generated graph, labels, batch and query, so a
             changed generator is detected instead of compared against
  canonical  SHA-256 of the oracle's canonical batch (lo, hi, sign by ord)
  nonzero    [ord, count, sum-hash, xor-hash] of every exact seed with matches
  over_cap   ords of the seeds given up (count > cap)
Every other ord has no incremental match.

Usage: python tests/golden/make_large_golden.py [--cap N] [--threads T] [--kind sparse|dense]
(about 20 minutes of 8 CPU threads for the dense query at the default cap)
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


def input_fingerprints(w, q, b) -> dict:
    g = w.graph
    return {
        "row_ptr": W.fingerprint(g.row_ptr), "col": W.fingerprint(g.col), "labels": W.fingerprint(g.labels),
        "batch_src": W.fingerprint(b.src), "batch_dst": W.fingerprint(b.dst), "batch_op": W.fingerprint(b.op),
        "query_labels": W.fingerprint(np.ascontiguousarray(q.labels, dtype=np.uint32)),
        "query_edges": W.fingerprint(np.ascontiguousarray(q.edges, dtype=np.uint32)),
    }


def canonical_fingerprint(lo, hi, sign) -> str:
    return W.fingerprint(np.concatenate([np.asarray(lo, np.uint32), np.asarray(hi, np.uint32),
                                         np.asarray(sign, np.uint32)]))


def path_of(kind: str) -> str:
    return os.path.join(HERE, "large_rmat24_%s_batch0.json" % kind)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cap", type=int, default=1000000)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--kind", action="append", choices=["sparse", "dense"])
    args = ap.parse_args()
    kinds = args.kind or ["sparse", "dense"]
    t0 = time.time()
    w = W.large()
    b = w.batches[0]
    print("generated in %.1f s" % (time.time() - t0), flush=True)
    for qi, q in enumerate(w.queries):
        if q.kind not in kinds:
            continue
        r = O2.run(w.graph, q, b, qid=0, threads=args.threads, want_tuples=False, seed_cap=args.cap)
        assert r.status == 0
        inc = r.seed_incomplete.astype(bool)
        nz = np.nonzero((r.seed_count > 0) & ~inc)[0]
        rec = {
            "cite": "Sec. II-A (the incremental matches of a batch) and the order rule after Algorithm 1 "
                    "(Sec. IV-C): per canonical update, the matches whose minimum-ord batch edge it is",
            "written_by": "tests/golden/make_large_golden.py (the oracle O2 only)",
            "workload": w.name, "batch": 0, "query_index": qi, "kind": q.kind, "k": q.k,
            "qlabels": [int(x) for x in q.labels], "qedges": [[int(a), int(c)] for a, c in q.edges.tolist()],
            "inputs": input_fingerprints(w, q, b),
            "n_canonical": int(r.n_canonical),
            "canonical": canonical_fingerprint(r.canon_lo, r.canon_hi, r.canon_sign),
            "cap": args.cap,
            "nonzero": [[int(i), int(r.seed_count[i]), str(int(r.seed_hsum[i])), str(int(r.seed_hxor[i]))]
                        for i in nz.tolist()],
            "over_cap": [int(i) for i in np.nonzero(inc)[0].tolist()],
            "oracle_seconds": round(r.seconds, 1), "oracle_threads": r.threads,
        }
        with open(path_of(q.kind), "w") as fh:
            json.dump(rec, fh, indent=0)
            fh.write("\n")
        print("%s: %d exact seeds with matches (%d matches), %d over the cap, %.0f s" % (
            q.kind, len(nz), int(r.seed_count[nz].sum()), int(inc.sum()), r.seconds), flush=True)


if __name__ == "__main__":
    main()
