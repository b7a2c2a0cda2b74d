"""Measured shape tuning for the fused Sinkhorn kernel.

    python -m paper_2107_06433_amd.tune --workloads single batched serving

For every (padded query width S, document-length bucket) pair that a
workload's queries meet, each candidate shape the library offers is timed
(HIP events around the launches, one launch per bucket) on the workload's own
corpus, and the fastest is kept.  The pins apply to buckets that launch on
their own; buckets that share a query's merged launch keep the merged
kernel's shape.  Entries are keyed by (S, bucket capacity, log2 of the
bucket's document count), because the best shape depends on how many
documents one launch holds.  The table is written to
paper_2107_06433_amd/tuning/gfx950_sink_shapes.json, which Corpus applies
when it is created.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from collections import defaultdict

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(PKG) not in sys.path:
    sys.path.insert(0, os.path.dirname(PKG))

from paper_2107_06433_amd import synth, wmd  # noqa: E402


def ndocs_class(n: int) -> int:
    return int(math.floor(math.log2(max(1, n))))


def representative_queries(Q: synth.Queries, limit: int) -> synth.Queries:
    """One query per distinct padded width (at most `limit`), in width order."""
    lens = np.diff(Q.q_ptr)
    seen = {}
    for b, n in enumerate(lens):
        S = int((n + 3) // 4 * 4)
        seen.setdefault(S, b)
    picks = [seen[S] for S in sorted(seen)][:limit]
    ids = [Q.query(b)[0] for b in picks]
    ws = [Q.query(b)[1] for b in picks]
    ptr = np.concatenate([[0], np.cumsum([len(x) for x in ids])]).astype(np.int64)
    return synth.Queries(q_ptr=ptr, ids=np.concatenate(ids).astype(np.int32),
                         weights=np.concatenate(ws).astype(np.float32))


def tune_workload(name: str, cdist: str = "fp32", reps: int = 2, max_candidates: int = 32,
                  max_queries: int = 128, per_query: bool = False, log=print) -> list[dict]:
    import torch

    w = synth.make_workload(name)
    c = w.corpus
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights, tuning=None)
    corpus.set_merge("none")  # every bucket on its own, so each pinned shape is timed
    info = corpus.info()
    bucket_docs = dict(zip(info["bucket_cap"], info["bucket_docs"]))
    Q = w.queries if w.queries.B <= max_queries else representative_queries(w.queries, max_queries)
    batch = wmd.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights)
    widths = sorted({int((n + 3) // 4 * 4) for n in np.diff(Q.q_ptr)})
    pairs = [(S, cap) for S in widths for cap, nd in bucket_docs.items() if nd > 0]
    cands = {p: corpus.sink_candidates(*p)[:max_candidates] for p in pairs}
    R = max(len(v) for v in cands.values())
    log(f"[tune] {name}: {len(pairs)} (S, cap) pairs, up to {R} candidates each, {Q.B} queries")
    # Shapes are timed in the regime the workload runs in: the whole batch in
    # one call (launch groups overlap on the side streams, so a shape is ranked
    # by its time while sharing the device), or with per_query one query per
    # call (each launch alone on the device, which favours latency).
    if per_query:
        singles = [wmd.QueryBatch.from_arrays([0, len(Q.query(b)[0])], *Q.query(b)) for b in range(Q.B)]
    else:
        singles = [batch]
    out = torch.empty((max(sb.B for sb in singles), c.N), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(corpus.workspace_bytes(sb) for sb in singles), dtype=torch.uint8, device="cuda")
    # every query keeps launches of its own (queries sharing a launch would
    # blur which (S, cap) pair a launch time belongs to)
    for sb in singles:  # warm caches and code
        corpus.query(sb, w.lam, w.max_iter, cdist=cdist, out=out, workspace=ws, per_query_launches=True)
    times = defaultdict(lambda: defaultdict(float))
    t0 = time.time()
    for r in range(R):
        for p, cs in cands.items():
            corpus.set_sink_shape(*p, cs[min(r, len(cs) - 1)])
        for _ in range(reps):
            corpus.set_timing(True)
            for sb in singles:
                corpus.query(sb, w.lam, w.max_iter, cdist=cdist, out=out, workspace=ws, check=False,
                             per_query_launches=True)
            torch.cuda.synchronize()
            recs = corpus.launches()
            corpus.set_timing(False)
            for rec in recs:
                key = (rec["S"], rec["cap"])
                if rec["S"] and key in cands and r < len(cands[key]):
                    times[key][r] += rec["ms"]
        if r % 8 == 7:
            log(f"[tune] {name}: candidate round {r + 1}/{R} ({time.time() - t0:.1f} s)")
    entries = []
    for p, cs in cands.items():
        best = min(range(len(cs)), key=lambda i: times[p][i])
        entries.append({"S": p[0], "cap": p[1], "ndocs_log2": ndocs_class(bucket_docs[p[1]]),
                        "shape": cs[best], "us": 1e3 * times[p][best] / reps,
                        "model_choice_us": 1e3 * times[p][0] / reps, "workload": name, "cdist": cdist,
                        "mode": "per_query" if per_query else "batch"})
    corpus.close()
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["single", "batched"])
    ap.add_argument("--out", default=wmd.TUNING_FILE)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--max-queries", type=int, default=128)
    ap.add_argument("--per-query", action="store_true", help="time one query per call")
    ap.add_argument("--cdist", default="fp32", choices=["fp32", "bf16"])
    args = ap.parse_args()
    table = {"arch": "gfx950", "entries": []}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    for name in args.workloads:
        new = tune_workload(name, cdist=args.cdist, reps=args.reps, max_queries=args.max_queries,
                            per_query=args.per_query)
        keys = {(e["S"], e["cap"], e["ndocs_log2"]) for e in new}
        table["entries"] = [e for e in table["entries"] if (e["S"], e["cap"], e["ndocs_log2"]) not in keys] + new
        gain = sum(e["model_choice_us"] for e in new) / max(1e-9, sum(e["us"] for e in new))
        print(f"[tune] {name}: {len(new)} entries, tuned shapes {gain:.2f}x faster than the model's first choice",
              flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    table["entries"].sort(key=lambda e: (e["S"], e["cap"], e["ndocs_log2"]))
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[tune] wrote {len(table['entries'])} entries to {args.out}")


if __name__ == "__main__":
    main()
