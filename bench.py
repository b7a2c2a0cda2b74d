"""Throughput benchmark of the Sinkhorn WMD hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload single|batched|tiny]
                    [--cdist fp32|bf16] [--schedule auto|resident|per_iteration|unfused]
                    [--plain] [--no-cpu-baseline]

A step is one call of the whole path (query selection, cost matrix + K,
max_iter fused SDDMM-SpMM iterations and the final pass) for the workload's
query batch against its resident corpus; inputs are in device memory before
the timed region starts.  The value is target-docs x iterations per second.
With --plain the batched workload's queries are issued one call each.

The default run (workload single) also reports, under "legs", the metric's
other parts at full size: the batched workload in one call (bf16 and fp32
cost matrix) against the same 64 queries issued one plain fp32 call each, with
their ratio; a short open-loop serving trace (p50/p99 latency at 2,000
queries/s and the highest stable rate tried); and the measured ceilings of
the GPU (HBM stream, K^T row gather, VALU rates) that the roofline fractions
are also given against.  --no-legs skips them.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target-docs·iters/s for Sinkhorn WMD (plain vs batched); p50/p99 query latency"
HBM_PEAK_GBS = 8000.0
# FP32 VALU: every HIP source is built with packed FP32 instructions disabled,
# so an FMA is one wave64 instruction per 4 cycles per SIMD: 256 CU x 4 SIMD x
# 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s (the published 157.3 counts packed
# FP32, reported beside it).  Matrix-core peaks as published.
PEAK_TFLOPS = {"alu": 78.6, "alu_packed_published": 157.3, "mfma_fp32": 157.3, "mfma_bf16": 2500.0}
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="single", choices=["tiny", "single", "batched", "serving"])
    ap.add_argument("--cdist", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "resident", "per_iteration", "unfused"])
    ap.add_argument("--plain", action="store_true", help="batched workload: one call per query")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-compact", action="store_true", help="cost matrix over the full vocabulary")
    ap.add_argument("--untuned", action="store_true", help="ignore the measured shape table")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="stop each document once x changes by at most tol (max_iter is the cap); "
                         "the value then counts the iterations actually run")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrival rate (queries/s)")
    ap.add_argument("--serve-queries", type=int, default=20000, help="serving: measured queries")
    ap.add_argument("--serve-warmup", type=int, default=2000, help="serving: warm-up queries")
    ap.add_argument("--sweep", type=float, nargs="*", default=[], help="serving: extra arrival rates to try")
    ap.add_argument("--mem-budget-gb", type=float, default=24.0, help="serving: device memory for queries")
    ap.add_argument("--max-batch", type=int, default=64)
    ap.add_argument("--per-query-launches", action="store_true",
                    help="every query gets its own Sinkhorn launches (no launches shared between queries)")
    ap.add_argument("--graph", action="store_true",
                    help="capture each call's launches into a HIP graph once and replay it (on a side stream)")
    ap.add_argument("--no-legs", action="store_true",
                    help="single workload: skip the batched, serving and ceiling legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scale for HBM counters)")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2107_06433_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def describe(w, plain: bool) -> str:
    p = w.info
    c = w.corpus
    vr = np.diff(w.queries.q_ptr)
    vr_txt = f"v_r={int(vr[0])}" if len(vr) == 1 else f"B={len(vr)} v_r={int(vr.min())}-{int(vr.max())} (sum {int(vr.sum())})"
    mode = " issued one query per call" if plain else ""
    return (f"{w.name}: V={c.V} d={c.d} N={c.N} docs of {p['n_lo']}-{p['n_hi']} Zipf(1.1) words "
            f"(nnz={c.nnz}), {vr_txt}, lambda={w.lam:g}, {w.max_iter} iterations{mode}")


def cpu_baseline(w, seconds: float):
    """The FP64 oracle as it stands (dense Algorithm 1 over the full vocabulary),
    timed on a bounded seeded sample of the workload's documents."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info() if t.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    c = w.corpus
    rng = np.random.default_rng(7)
    order = rng.permutation(c.N)
    ids, qw = w.queries.query(0)
    block = 64 if c.V >= 50_000 else 256
    done, t_total = 0, 0.0
    while t_total < seconds and done < c.N:
        docs = order[done:done + block]
        t0 = time.perf_counter()
        oracle.wmd_dense_corpus(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter,
                                docs=docs, block=block)
        t_total += time.perf_counter() - t0
        done += len(docs)
    dense_rate = done * w.max_iter / t_total
    # the support-restricted form of the same oracle, same kind of sample
    t0 = time.perf_counter()
    ns = 0
    while time.perf_counter() - t0 < min(5.0, seconds / 3) and ns < c.N:
        chunk = order[ns:ns + 32]
        oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter,
                                    docs=chunk)
        ns += len(chunk)
    sup_rate = ns * w.max_iter / (time.perf_counter() - t0)
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": dense_rate, "unit": "docs*iters/s", "cores": int(threads), "kind": "oracle",
        "sample": f"dense full-vocabulary FP64 Algorithm 1, query 0, {done} seeded random documents "
                  f"of the same corpus, {t_total:.1f} s",
        "support_restricted_value": sup_rate,
        "support_restricted_sample": f"{ns} documents",
        "cpu_model": cpu, "affinity_cores": len(os.sched_getaffinity(0)),
    }


def serving(args):
    """Open-loop serving run: Poisson arrivals, continuous batching, p50/p99."""
    import torch

    from paper_2107_06433_amd import serve, synth, wmd

    nq = args.serve_warmup + args.serve_queries
    w = synth.make_workload("serving", n_queries=nq)
    c = w.corpus
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights, device="cuda:0",
                                   tuning=None if args.untuned else wmd.TUNING_FILE)
    info = corpus.info()
    print(f"[bench] serving corpus ready: U={info['U']}", file=sys.stderr, flush=True)
    Q = w.queries

    def trace(rate, n, warm):
        ex = serve.GpuExecutor(corpus, w.lam, w.max_iter, cdist=args.cdist, streams=3)
        sch = serve.Scheduler(ex, int(args.mem_budget_gb * (1 << 30)), args.max_batch, max_inflight=3)
        reqs = [serve.Request(ids=Q.query(b)[0], weights=Q.query(b)[1], arrival=0.0) for b in range(n)]
        arr = w.arrivals[:n] * (args.rate / rate)
        arr = arr - arr[0]
        st = serve.run_trace(sch, reqs, arr, warmup=warm)
        torch.cuda.synchronize()
        st["rate"] = rate
        st["docs_iters_per_s"] = st["served_qps"] * c.N * w.max_iter
        print(f"[bench] rate {rate:g} q/s: served {st['served_qps']:.0f} q/s, p50 {st['p50_ms']:.1f} ms, "
              f"p99 {st['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        return st

    trace(args.rate, min(nq, 300), 0)  # compile paths, warm the allocator
    main_st = trace(args.rate, nq, args.serve_warmup)
    sweep = [trace(r, min(nq, 4000), 500) for r in args.sweep]
    stable = [s for s in [main_st] + sweep if s["served_qps"] >= 0.97 * s["rate"]]
    # roofline of the dominant kernel over one 64-query batch of the trace's queries
    sub = wmd.QueryBatch.from_arrays(Q.q_ptr[:65], Q.ids[:Q.q_ptr[64]], Q.weights[:Q.q_ptr[64]])
    corpus.set_timing(True)
    corpus.query(sub, w.lam, w.max_iter, cdist=args.cdist, check=False)
    torch.cuda.synchronize()
    stats = corpus.timing()
    corpus.set_timing(False)
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    tfl = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": tfl, "peak": PEAK_TFLOPS["alu"], "unit": "TFLOP/s",
            "frac": tfl / PEAK_TFLOPS["alu"], "kernel": dom["name"], "avg_launch_us": avg_ms * 1e3,
            "peak_basis": "FP32 FMA without packed instructions: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz",
            "frac_of_published_packed_peak": tfl / PEAK_TFLOPS["alu_packed_published"], "traffic": None}
    res = {
        "metric": METRIC, "value": main_st["docs_iters_per_s"], "unit": "docs*iters/s", "n_gpus": 1,
        "steps": main_st["completed"], "warmup": args.serve_warmup,
        "ms_per_step": 1e3 / max(1e-9, main_st["served_qps"]), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16-gemm+f32" if args.cdist == "bf16" else "f32",
        "data": "synthetic (seeded Zipf corpus, lognormal query lengths, Poisson arrivals; no dataset)",
        "config": {"workload": (f"serving: V={c.V} d={c.d} N={c.N} docs of 20-60 Zipf(1.1) words (nnz={c.nnz}), "
                                f"v_r lognormal median 25 sigma 1 cap 500, Poisson {args.rate:g} q/s, "
                                f"lambda={w.lam:g}, {w.max_iter} iterations"),
                   "cdist": args.cdist, "mem_budget_gb": args.mem_budget_gb, "max_batch": args.max_batch,
                   "streams": 3, "vocab_rows_U": info["U"], "tuned_shapes": corpus.pinned,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": main_st["p50_ms"], "p99": main_st["p99_ms"], "mean": main_st["mean_ms"]},
        "offered_qps": main_st["offered_qps"], "served_qps": main_st["served_qps"],
        "batches": main_st["batches"], "peak_mem_bytes": main_st["peak_mem_bytes"],
        "rate_sweep": sweep, "highest_stable_rate": max([s["rate"] for s in stable], default=None),
        "roofline": roof, "source_hash": source_hash(),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res))


def _ms_per_step(fn, warmup: int, steps: int) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def batched_leg() -> dict:
    """The batched workload at full size: one call for all 64 queries (bf16
    and fp32 cost matrix) and the same queries issued one plain fp32 call
    each (also with the paper's one-launch-per-iteration schedule, as
    context); docs*iters/s and the batched/plain ratios."""
    import torch

    from paper_2107_06433_amd import synth, wmd
    w = synth.make_workload("batched")
    c, Q = w.corpus, w.queries
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    dev = corpus.device
    batch = wmd.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights)
    singles = [wmd.QueryBatch.from_arrays([0, len(Q.query(b)[0])], *Q.query(b)) for b in range(Q.B)]
    out = torch.empty((Q.B, c.N), dtype=torch.float32, device=dev)
    ws = torch.empty(corpus.workspace_bytes(batch), dtype=torch.uint8, device=dev)
    sws = {sch: torch.empty(max(corpus.workspace_bytes(b, sch) for b in singles), dtype=torch.uint8, device=dev)
           for sch in ("auto", "per_iteration")}
    docs_iters = Q.B * c.N * w.max_iter

    def one_call(cd):
        return lambda: corpus.query(batch, w.lam, w.max_iter, cdist=cd, out=out, workspace=ws, check=False)

    def per_query(sch):
        def run():
            for b, sb in enumerate(singles):
                corpus.query(sb, w.lam, w.max_iter, cdist="fp32", schedule=sch, out=out[b:b + 1],
                             workspace=sws[sch], check=False)
        return run

    res = {"config": describe(w, False)}
    for key, fn, warm, steps in (("batched_bf16", one_call("bf16"), 1, 4), ("batched_fp32", one_call("fp32"), 1, 4),
                                 ("plain_fp32", per_query("auto"), 1, 3),
                                 ("plain_fp32_per_iteration_schedule", per_query("per_iteration"), 1, 1)):
        ms = _ms_per_step(fn, warm, steps)
        res[key] = {"ms_per_step": ms, "value": docs_iters / (ms * 1e-3), "steps": steps}
        print(f"[bench] batched leg {key}: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    res["ratio_batched_bf16_vs_plain_fp32"] = res["batched_bf16"]["value"] / res["plain_fp32"]["value"]
    res["ratio_batched_bf16_vs_plain_fp32_per_iteration"] = (
        res["batched_bf16"]["value"] / res["plain_fp32_per_iteration_schedule"]["value"])
    res["unit"] = "docs*iters/s"
    res["note"] = ("plain = the same 64 queries, one wmd_query(B=1) each, resident fused kernel (the library's "
                   "own per-query path); plain_fp32_per_iteration_schedule = one fused SDDMM-SpMM launch per "
                   "iteration per query, the paper's loop structure (context only)")
    del corpus
    torch.cuda.empty_cache()
    return res


def serving_leg(rates=(2000.0, 1500.0, 1250.0, 1000.0), measured=4000, warm=500) -> dict:
    """A short open-loop serving trace on the full serving corpus (Poisson
    arrivals, continuous batching on three streams, bf16 cost matrix): p50/p99
    at 2,000 queries/s and at lower rates; the highest rate served within 3%."""
    import torch

    from paper_2107_06433_amd import serve, synth, wmd
    n = warm + measured
    w = synth.make_workload("serving", n_queries=n)
    c, Q = w.corpus, w.queries
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    reqs_of = lambda k: [serve.Request(ids=Q.query(b)[0], weights=Q.query(b)[1], arrival=0.0) for b in range(k)]

    def trace(rate, k, wk):
        ex = serve.GpuExecutor(corpus, w.lam, w.max_iter, cdist="bf16", streams=3)
        sch = serve.Scheduler(ex, 24 << 30, 64, max_inflight=3)
        arr = w.arrivals[:k] * (2000.0 / rate)
        st = serve.run_trace(sch, reqs_of(k), arr - arr[0], warmup=wk)
        torch.cuda.synchronize()
        st["rate"] = rate
        st["docs_iters_per_s"] = st["served_qps"] * c.N * w.max_iter
        print(f"[bench] serving leg {rate:g} q/s: served {st['served_qps']:.0f} q/s, p50 {st['p50_ms']:.1f} ms, "
              f"p99 {st['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        return {k2: st[k2] for k2 in ("rate", "offered_qps", "served_qps", "p50_ms", "p99_ms", "mean_ms",
                                      "completed", "batches", "docs_iters_per_s")}

    trace(rates[0], 300, 0)  # warm the allocator and the launch plans
    runs = [trace(rates[0], n, warm)] + [trace(r, min(n, 2500), 300) for r in rates[1:]]
    stable = [r["rate"] for r in runs if r["served_qps"] >= 0.97 * r["rate"]]
    res = {"config": (f"serving: V={c.V} d={c.d} N={c.N} docs of 20-60 Zipf(1.1) words (nnz={c.nnz}), v_r lognormal "
                      f"median 25 sigma 1 cap 500, Poisson arrivals, bf16 cost matrix, lambda={w.lam:g}, "
                      f"{w.max_iter} iterations, {measured} measured queries after {warm}"),
           "at_2000_qps": runs[0], "sweep": runs[1:], "highest_stable_rate_tried": max(stable, default=None),
           "unit": "docs*iters/s"}
    del corpus
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: no multi-GPU path is implemented (asked for --gpus {args.gpus}). "
              "Documents would shard across GPUs with no per-iteration exchange.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2107_06433_amd import synth, wmd

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return
    if args.workload == "serving":
        serving(args)
        return
    dev = torch.device("cuda:0")
    w = synth.make_workload(args.workload)
    c = w.corpus
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights, device=dev,
                                   compact_vocab=not args.no_compact,
                                   tuning=None if args.untuned else wmd.TUNING_FILE)
    info = corpus.info()
    Q = w.queries
    if args.plain:
        batches = [wmd.QueryBatch.from_arrays([0, len(Q.query(b)[0])], *Q.query(b), device=dev) for b in range(Q.B)]
    else:
        batches = [wmd.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights, device=dev)]
    outs = [torch.empty((bt.B, c.N), dtype=torch.float32, device=dev) for bt in batches]
    itss = [torch.zeros((bt.B, c.N), dtype=torch.int32, device=dev) if args.tol > 0 else None for bt in batches]
    wss = [torch.empty(corpus.workspace_bytes(bt, args.schedule), dtype=torch.uint8, device=dev) for bt in batches]

    # graphs replay on a stream of their own (capture needs one other than the legacy default)
    run_stream = torch.cuda.Stream(device=dev) if args.graph else None

    def step():
        for bt, o, ws, its in zip(batches, outs, wss, itss):
            corpus.query(bt, w.lam, w.max_iter, cdist=args.cdist, schedule=args.schedule, out=o,
                         workspace=ws, check=False, tol=args.tol, iters=its, stream=run_stream,
                         graph=args.graph, per_query_launches=args.per_query_launches)

    # validity check of the configuration before timing
    step()
    torch.cuda.synchronize()
    for bt, ws in zip(batches, wss):
        codes = corpus.query_errors(ws, bt.B, run_stream)
        assert not codes.any(), codes
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # timed region: plain, for the value
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    docs_iters = Q.B * c.N * w.max_iter
    if args.tol > 0:  # the iterations actually executed (every step runs the same ones)
        docs_iters = int(sum(int(its.sum().item()) for its in itss))
    value = docs_iters / (ms / 1e3)
    print(f"[bench] timed {args.steps} steps: {ms:.4f} ms/step", file=sys.stderr, flush=True)

    # the same steps again with HIP events around every kernel launch (eager:
    # per-kernel timing bypasses graph replay)
    corpus.set_timing(True)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stats = corpus.timing()
    corpus.set_timing(False)
    ms_events = (t3 - t2) * 1e3 / args.steps
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    name = dom["name"]
    if name.startswith("cdist"):
        bf16 = ",1," in name
        gbs = dom["bytes"] / dom["launches"] / (avg_ms * 1e-3) / 1e9
        tfl = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
        peak_t = PEAK_TFLOPS["mfma_bf16" if bf16 else "mfma_fp32"]
        if gbs / HBM_PEAK_GBS >= tfl / peak_t:
            roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            roof = {"bound": "mfma", "achieved": tfl, "peak": peak_t, "unit": "TFLOP/s"}
    elif args.schedule in ("auto", "resident"):
        tfl = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": tfl, "peak": PEAK_TFLOPS["alu"], "unit": "TFLOP/s",
                "peak_basis": "FP32 FMA without packed instructions: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz",
                "frac_of_published_packed_peak": tfl / PEAK_TFLOPS["alu_packed_published"]}
    else:
        gbs = dom["bytes"] / dom["launches"] / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = name
    roof["avg_launch_us"] = avg_ms * 1e3
    roof["traffic"] = None
    try:
        with open(PMC_FILE) as f:
            pmc = json.load(f)
        key = f"{args.workload}|{args.cdist}|{args.schedule}|{'plain' if args.plain else 'batch'}"
        ent = pmc.get("entries", {}).get(key)
        if ent and ent.get("kernel") == name and ent.get("source_hash") == source_hash():
            roof["traffic"] = ent["traffic_bytes_per_launch"]
    except (OSError, ValueError):
        pass

    if args.workload == "single" and not args.no_legs:
        from paper_2107_06433_amd import microbench
        ids_c, U_c = microbench.corpus_ids(c.word_ids)
        S_c = int((int(np.diff(Q.q_ptr).max()) + 3) // 4 * 4)
        ceil = microbench.measure(torch.from_numpy(ids_c).to(dev), U_c, S_c)
        print(f"[bench] ceilings: {json.dumps(ceil)}", file=sys.stderr, flush=True)
        if roof["unit"] == "TFLOP/s" and roof["bound"] == "alu":
            roof["measured_peak"] = ceil["valu"]["fma_TFLOPs"]
            roof["measured_peak_source"] = "wmd_bench_valu float32 FMA chains (this run)"
            # the paper's bandwidth model next to the ALU one: the launch's
            # HBM stream (entries, records) and its K^T row gather at the
            # measured ceilings, its flops at the measured FMA rate
            nnz = float(c.nnz)
            vr = float(np.diff(Q.q_ptr).sum())
            t_stream = (8.0 * nnz + 20.0 * c.N) / (ceil["hbm"]["read_GBps"] * 1e9)
            t_gather = 4.0 * vr * nnz / (ceil["gather"]["GBps"] * 1e9)
            t_alu = dom["flops"] / dom["launches"] / (ceil["valu"]["fma_TFLOPs"] * 1e12)
            roof["model_fraction"] = max(t_stream, t_gather, t_alu) / (avg_ms * 1e-3)
            roof["model_terms_us"] = {"hbm_stream": t_stream * 1e6, "row_gather": t_gather * 1e6,
                                      "fma": t_alu * 1e6}
        elif roof["unit"] == "GB/s":
            roof["measured_peak"] = ceil["hbm"]["read_GBps"]
            roof["measured_peak_source"] = "wmd_bench_stream read (this run)"
        if "measured_peak" in roof:
            roof["frac_of_measured"] = roof["achieved"] / roof["measured_peak"]
        legs = {"ceilings": ceil}
        legs["batched"] = batched_leg()
        legs["serving"] = serving_leg()
    else:
        legs = None
    if roof.get("traffic") is not None:
        roof["traffic_source"] = ("profiles/pmc_traffic.json: rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel "
                                  "and source hash, scaled by a plain copy (not measured in this run)")

    res = {
        "metric": METRIC, "value": value, "unit": "docs*iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.cdist == "fp32" else "bf16-gemm+f32",
        "data": "synthetic (seeded Zipf corpus and N(0,1/d) embeddings; no dataset)",
        "config": {"workload": describe(w, args.plain), "queries_per_step": Q.B, "docs": c.N,
                   "max_iter": w.max_iter, "cdist": args.cdist, "schedule": args.schedule, "tol": args.tol, "graph": args.graph,
                   "compact_vocab": not args.no_compact, "vocab_rows_U": info["U"],
                   "tuned_shapes": corpus.pinned,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernels": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in s.items()} for s in stats],
        "ms_per_step_with_events": ms_events,
        "source_hash": source_hash(),
        "device": torch.cuda.get_device_name(0),
    }
    if legs is not None:
        res["legs"] = legs
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
