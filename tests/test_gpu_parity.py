"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: float32 cost matrix and iteration within 1e-4 relative of the
oracle; bf16 cost-matrix GEMM within 1e-3; both as |g - o| <= tol |o| + 1e-7
(the absolute floor only matters for identical documents, whose distance is
near zero).  Integer outputs (error codes) and NaN placement are exact.
"""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

import oracle
from paper_2107_06433_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-4
TOL16 = 1e-3


@pytest.fixture(scope="module")
def W():
    from paper_2107_06433_amd import wmd  # loads libwmd.so; fails loudly if missing
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wmd


def rel_err(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return np.abs(g - o) / (np.abs(o) + 1e-7 / TOL32)


def assert_close(g, o, tol, what=""):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    assert g.shape == o.shape
    nan_g, nan_o = np.isnan(g), np.isnan(o)
    assert np.array_equal(nan_g, nan_o), f"{what}: NaN placement differs"
    ok = ~nan_o
    err = np.abs(g[ok] - o[ok])
    lim = tol * np.abs(o[ok]) + 1e-7
    bad = np.nonzero(err > lim)[0]
    assert bad.size == 0, (f"{what}: {bad.size} of {ok.sum()} outside tol {tol}; worst rel "
                           f"{(err / np.abs(o[ok])).max():.3e}")


def corpus_of(W, c, compact=True):
    return W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights, compact_vocab=compact)


def run(W, corpus, queries, lam, iters, **kw):
    batch = W.QueryBatch.from_arrays(queries.q_ptr, queries.ids, queries.weights)
    out = corpus.query(batch, lam, iters, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_support(c, ids, qw, lam, iters, docs=None):
    return oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, lam, iters, docs=docs)


# ---------------------------------------------------------------- tiny workload

@pytest.fixture(scope="module")
def tiny():
    w = synth.make_workload("tiny")
    ids, qw = w.queries.query(0)
    ref = oracle.wmd_dense_corpus(w.corpus.emb, w.corpus.doc_ptr, w.corpus.word_ids, w.corpus.weights,
                                  ids, qw, w.lam, w.max_iter)
    return w, ref


@pytest.mark.parametrize("schedule", ["resident", "per_iteration", "unfused"])
def test_tiny_fp32_matches_dense_oracle(W, tiny, schedule):
    w, ref = tiny
    got = run(W, corpus_of(W, w.corpus), w.queries, w.lam, w.max_iter, schedule=schedule)[0]
    assert_close(got, ref, TOL32, schedule)


def test_tiny_bf16_matches_dense_oracle(W, tiny):
    w, ref = tiny
    got = run(W, corpus_of(W, w.corpus), w.queries, w.lam, w.max_iter, cdist="bf16")[0]
    assert_close(got, ref, TOL16, "bf16")


def test_vocab_compaction_changes_nothing(W, tiny):
    w, _ = tiny
    a = run(W, corpus_of(W, w.corpus, compact=True), w.queries, w.lam, w.max_iter)
    b = run(W, corpus_of(W, w.corpus, compact=False), w.queries, w.lam, w.max_iter)
    assert np.array_equal(a, b)


def test_deterministic_and_schedules_agree(W, tiny):
    w, _ = tiny
    c = corpus_of(W, w.corpus)
    a = run(W, c, w.queries, w.lam, w.max_iter)
    b = run(W, c, w.queries, w.lam, w.max_iter)
    assert np.array_equal(a, b)
    p = run(W, c, w.queries, w.lam, w.max_iter, schedule="per_iteration")
    assert np.array_equal(a, p), "resident and per-iteration schedules run the same arithmetic"


@pytest.mark.parametrize("iters", [0, 1, 2, 40])
def test_iteration_counts(W, tiny, iters):
    w, _ = tiny
    ids, qw = w.queries.query(0)
    ref = oracle.wmd_dense_corpus(w.corpus.emb, w.corpus.doc_ptr, w.corpus.word_ids, w.corpus.weights,
                                  ids, qw, w.lam, iters)
    got = run(W, corpus_of(W, w.corpus), w.queries, w.lam, iters)[0]
    assert_close(got, ref, TOL32, f"iters={iters}")


# ------------------------------------------------------------ single-query size

@pytest.fixture(scope="module")
def single():
    return synth.make_workload("single")


@pytest.fixture(scope="module")
def single_run(W, single):
    c = corpus_of(W, single.corpus)
    g32 = run(W, c, single.queries, single.lam, single.max_iter)[0]
    g16 = run(W, c, single.queries, single.lam, single.max_iter, cdist="bf16")[0]
    return c, g32, g16


SAMPLE = 240


def sample_docs(N, seed=0):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(SAMPLE, N), replace=False))


def test_single_fp32_sampled(W, single, single_run):
    _, g32, _ = single_run
    docs = sample_docs(single.corpus.N)
    ids, qw = single.queries.query(0)
    ref = oracle_support(single.corpus, ids, qw, single.lam, single.max_iter, docs)
    assert_close(g32[docs], ref, TOL32, "single fp32")


def test_single_bf16_sampled(W, single, single_run):
    _, _, g16 = single_run
    docs = sample_docs(single.corpus.N, seed=1)
    ids, qw = single.queries.query(0)
    ref = oracle_support(single.corpus, ids, qw, single.lam, single.max_iter, docs)
    assert_close(g16[docs], ref, TOL16, "single bf16")


def test_single_error_distribution(W, single, single_run):
    """Relative WMD error of every document of the single-query workload
    against the FP64 oracle, for the f32 and the bf16 cost-matrix inputs
    (max, median and 99th percentile are printed; with WMD_REPORT_DIR set they
    are also written there as JSON)."""
    _, g32, g16 = single_run
    ids, qw = single.queries.query(0)
    ref = oracle_support(single.corpus, ids, qw, single.lam, single.max_iter)
    ok = ~np.isnan(ref)
    report = {"docs": int(ok.sum())}
    for name, g, tol in (("fp32", g32, TOL32), ("bf16", g16, TOL16)):
        e = np.abs(g[ok].astype(np.float64) - ref[ok]) / np.abs(ref[ok])
        report[name] = {"max_rel": float(e.max()), "median_rel": float(np.median(e)),
                        "p99_rel": float(np.quantile(e, 0.99)), "tolerance": tol}
        assert_close(g, ref, tol, f"single {name}, every document")
    print("single-query WMD error vs FP64 oracle:", json.dumps(report))
    out = os.environ.get("WMD_REPORT_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "precision_single.json"), "w") as f:
            json.dump(report, f, indent=1)


def test_single_every_document_within_cost_range(W, single, single_run):
    """At any size: d_k is a convex combination of the costs between the
    query's words and document k's words (the plan has total mass 1)."""
    _, g32, _ = single_run
    c = single.corpus
    ids, qw = single.queries.query(0)
    sel, _ = oracle.select_query(c.V, ids, qw)
    Eq = c.emb[sel].astype(np.float64)
    for k in range(c.N):
        wk = c.word_ids[c.doc_ptr[k]:c.doc_ptr[k + 1]]
        M = cdist(Eq, c.emb[wk].astype(np.float64))
        assert M.min() * (1 - 1e-5) - 1e-6 <= g32[k] <= M.max() * (1 + 1e-5) + 1e-6


# ------------------------------------------------------------------- batched

@pytest.fixture(scope="module")
def batched():
    return synth.make_workload("batched", scale_docs=0.02)  # N = 1,000 documents, 64 queries


def test_batched_fp32_and_bf16(W, batched):
    c = corpus_of(W, batched.corpus)
    g32 = run(W, c, batched.queries, batched.lam, batched.max_iter)
    g16 = run(W, c, batched.queries, batched.lam, batched.max_iter, cdist="bf16")
    rng = np.random.default_rng(3)
    for b in range(batched.queries.B):
        docs = np.sort(rng.choice(batched.corpus.N, size=12, replace=False))
        ids, qw = batched.queries.query(b)
        ref = oracle_support(batched.corpus, ids, qw, batched.lam, batched.max_iter, docs)
        assert_close(g32[b, docs], ref, TOL32, f"batched fp32 q{b} vr={len(ids)}")
        assert_close(g16[b, docs], ref, TOL16, f"batched bf16 q{b} vr={len(ids)}")


def test_batch_invariance(W, batched):
    c = corpus_of(W, batched.corpus)
    full = run(W, c, batched.queries, batched.lam, batched.max_iter)
    for b in (0, 17, 63):
        ids, qw = batched.queries.query(b)
        one = synth.Queries(q_ptr=np.array([0, len(ids)]), ids=ids, weights=qw)
        alone = run(W, c, one, batched.lam, batched.max_iter)[0]
        assert np.array_equal(alone, full[b]), f"query {b} differs alone vs in the batch"


@pytest.mark.parametrize("vr", [3, 8, 12, 16, 20, 24, 28, 32])
def test_narrow_query_alone_and_among_wide_ones(W, vr):
    """A query of at most 32 padded columns alone runs the skinny cost-matrix
    kernel; among wide queries its columns go through the tiled kernel.  Both
    add the k products of a 16-column tile in the same order, so bf16 inputs
    and f32 widths of whole tiles (16, 32) give identical bits.  The f32
    4-column groups (widths 17-28 and at most 12) add k in four interleaved
    partial sums: the same distances to within a few float32 ulp."""
    rng = np.random.default_rng(700 + vr)
    c = handmade_corpus(rng, 3000, 300, rng.integers(5, 60, size=300))
    corpus = corpus_of(W, c)
    wide = [(rng.choice(3000, 60, replace=False), rng.integers(1, 4, 60)) for _ in range(2)]
    q = (rng.choice(3000, vr, replace=False), rng.integers(1, 4, vr))

    def batch(qs):
        return synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(a) for a, _ in qs])]),
                             ids=np.concatenate([a for a, _ in qs]).astype(np.int32),
                             weights=np.concatenate([x for _, x in qs]).astype(np.float32))

    for cd in ("fp32", "bf16"):
        alone = run(W, corpus, batch([q]), 10.0, 15, cdist=cd)[0]
        among = run(W, corpus, batch([wide[0], q, wide[1]]), 10.0, 15, cdist=cd)[1]
        if cd == "bf16" or (vr + 3) // 4 * 4 in (16, 32):
            assert np.array_equal(alone, among), f"{cd} v_r={vr}: alone differs from among wide queries"
        else:
            assert_close(alone, among, 1e-6, f"{cd} v_r={vr}: alone vs among wide queries")


def test_graph_replays_match_eager(W, batched):
    """Captured launches replay bit-identically to eager calls, with eager
    work (a fill of the output, another query on another stream) between the
    replays; new query contents written in place are picked up by a replay."""
    corpus = corpus_of(W, batched.corpus)
    Q, N, lam, it = batched.queries, batched.corpus.N, batched.lam, batched.max_iter
    batch = W.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights)
    other = W.QueryBatch.from_arrays(Q.q_ptr[:6], Q.ids[:Q.q_ptr[5]], Q.weights[:Q.q_ptr[5]])
    s = torch.cuda.Stream()
    for tol in (0.0, 1e-3):
        ref_it = torch.zeros(Q.B * N, dtype=torch.int32, device="cuda")
        ref = corpus.query(batch, lam, it, tol=tol, iters=ref_it, stream=s).cpu().numpy()
        out = torch.empty((Q.B, N), dtype=torch.float32, device="cuda")
        ws = torch.empty(corpus.workspace_bytes(batch), dtype=torch.uint8, device="cuda")
        g_it = torch.zeros(Q.B * N, dtype=torch.int32, device="cuda")
        for rep in range(4):
            with torch.cuda.stream(s):
                out.fill_(float("nan"))
                g_it.fill_(-1)
            corpus.query(batch, lam, it, tol=tol, iters=g_it, out=out, workspace=ws, stream=s, graph=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), ref, err_msg=f"tol={tol} replay {rep}")
            assert torch.equal(g_it, ref_it), f"tol={tol} replay {rep}: iteration counts differ"
            corpus.query(other, lam, it)  # eager work between replays
            torch.cuda.synchronize()
    # same tensors, new contents: the replay reads them at run time
    ids2 = ((Q.ids.astype(np.int64) + 1) % batched.corpus.emb.shape[0]).astype(np.int32)
    ref2_it = torch.zeros_like(g_it)
    ref2 = corpus.query(W.QueryBatch.from_arrays(Q.q_ptr, ids2, Q.weights), lam, it, tol=1e-3,
                        iters=ref2_it).cpu().numpy()
    batch.ids.copy_(torch.from_numpy(ids2))
    torch.cuda.synchronize()
    corpus.query(batch, lam, it, tol=1e-3, iters=g_it, out=out, workspace=ws, stream=s, graph=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref2)
    assert torch.equal(g_it, ref2_it)


# ----------------------------------------------------------------- edge cases

def handmade_corpus(rng, V, d, lengths, dup=False):
    E = (rng.standard_normal((V, d)) / math.sqrt(d)).astype(np.float32)
    ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    ids = np.concatenate([rng.choice(V, size=n, replace=dup) if n else np.zeros(0, int) for n in lengths])
    w = rng.integers(1, 5, size=len(ids)).astype(np.float32)
    return synth.Corpus(V=V, d=d, emb=E, doc_ptr=ptr, word_ids=ids.astype(np.int32), weights=w)


def test_single_query_word_closed_form(W):
    rng = np.random.default_rng(40)
    c = handmade_corpus(rng, 500, 48, rng.integers(1, 70, size=60))
    q = synth.Queries(q_ptr=np.array([0, 2]), ids=np.array([7, 7], np.int32), weights=np.array([1, 2], np.float32))
    got = run(W, corpus_of(W, c), q, 10.0, 15)[0]
    M = cdist(c.emb[[7]].astype(np.float64), c.emb.astype(np.float64))[0]
    want = np.array([(c.weights[s:e] / c.weights[s:e].sum() * M[c.word_ids[s:e]]).sum()
                     for s, e in zip(c.doc_ptr[:-1], c.doc_ptr[1:])])
    assert_close(got, want, 2e-6, "v_r = 1")


def test_empty_zero_weight_and_duplicate_entries(W):
    rng = np.random.default_rng(41)
    V, d = 300, 32
    E = (rng.standard_normal((V, d)) / math.sqrt(d)).astype(np.float32)
    docs = [([], []), ([5, 9, 5], [1, 2, 3]), ([11, 12], [0, 0]), ([3, 4, 8], [1, 0, 2]), ([250], [4])]
    ptr = np.concatenate([[0], np.cumsum([len(a) for a, _ in docs])]).astype(np.int64)
    ids = np.array([i for a, _ in docs for i in a], np.int32)
    w = np.array([x for _, b in docs for x in b], np.float32)
    c = synth.Corpus(V=V, d=d, emb=E, doc_ptr=ptr, word_ids=ids, weights=w)
    q = synth.Queries(q_ptr=np.array([0, 5]), ids=np.array([9, 3, 9, 100, 42], np.int32),
                      weights=np.array([1, 2, 2, 0, 1], np.float32))
    got = run(W, corpus_of(W, c), q, 10.0, 15)[0]
    ref = oracle.wmd_dense_corpus(E, ptr, ids, w, q.ids, q.weights, 10.0, 15)
    assert np.isnan(got[0]) and np.isnan(got[2])
    assert_close(got, ref, TOL32, "edge docs")


def test_short_and_long_query_selection_agree(W):
    """Queries of at most 64 entries are selected by one wave, longer ones by
    the block-wide path.  The same words, with repeats and zero weights, padded
    with more zero weights to 50 and 70 entries, give the same distances (to
    the rounding of a different slot width) and match the oracle, first in
    the call or last."""
    rng = np.random.default_rng(46)
    c = handmade_corpus(rng, 400, 24, rng.integers(1, 40, size=60))
    base_ids = rng.choice(400, size=20, replace=False)
    ids_a = np.concatenate([base_ids, base_ids[:4], rng.choice(400, size=3)]).astype(np.int32)
    w_a = rng.integers(0, 4, size=len(ids_a)).astype(np.float32)
    w_a[:3] = [1, 2, 3]
    qs = [(ids_a, w_a)]
    for total in (50, 70):
        pad = rng.choice(400, size=total - len(ids_a)).astype(np.int32)
        qs.append((np.concatenate([ids_a, pad]), np.concatenate([w_a, np.zeros(len(pad), np.float32)])))
    assert len(qs[0][0]) <= 32 < len(qs[1][0]) <= 64 < len(qs[2][0])
    ref = oracle_support(c, ids_a, w_a, 10.0, 15)
    corpus = corpus_of(W, c)
    for order in ((0, 1, 2), (2, 1, 0)):
        q = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(qs[i][0]) for i in order])]),
                          ids=np.concatenate([qs[i][0] for i in order]),
                          weights=np.concatenate([qs[i][1] for i in order]))
        for cd, tol in (("fp32", TOL32), ("bf16", TOL16)):
            got = run(W, corpus, q, 10.0, 15, cdist=cd)
            for b, i in enumerate(order):
                assert_close(got[b], ref, tol, f"{cd} query of {len(qs[i][0])} entries at position {b}")
                assert_close(got[b], got[order.index(0)], 1e-5 if cd == "fp32" else 1e-4,
                             f"{cd} {len(qs[i][0])} vs {len(qs[0][0])} entries")


def test_all_length_buckets_and_multiwave_items(W):
    rng = np.random.default_rng(42)
    lengths = [1, 2, 15, 16, 17, 33, 64, 65, 127, 128, 200, 256, 257, 511, 700, 1024, 1500, 2048, 3000, 4096]
    c = handmade_corpus(rng, 6000, 40, lengths)
    qs = [rng.choice(6000, size=v, replace=False) for v in (3, 21, 70, 150)]
    q = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(x) for x in qs])]),
                      ids=np.concatenate(qs).astype(np.int32),
                      weights=rng.integers(1, 4, size=sum(len(x) for x in qs)).astype(np.float32))
    got = run(W, corpus_of(W, c), q, 10.0, 15)
    for b in range(q.B):
        ids, qw = q.query(b)
        ref = oracle_support(c, ids, qw, 10.0, 15)
        assert_close(got[b], ref, TOL32, f"query width {len(ids)}")


def test_schedules_agree_on_multiwave_items(W):
    """Long documents and wide queries run as items of several waves (column
    sums exchanged through LDS); the per-iteration and unfused schedules, which
    keep u and w in memory between launches, compute what the resident one
    does, and all match the oracle."""
    rng = np.random.default_rng(47)
    lengths = np.concatenate([rng.integers(150, 700, size=24), rng.integers(700, 1500, size=6)])
    c = handmade_corpus(rng, 5000, 40, lengths)
    qs = [rng.choice(5000, size=v, replace=False) for v in (70, 150)]
    q = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(x) for x in qs])]),
                      ids=np.concatenate(qs).astype(np.int32),
                      weights=rng.integers(1, 4, size=sum(len(x) for x in qs)).astype(np.float32))
    corpus = corpus_of(W, c)
    res = run(W, corpus, q, 10.0, 15)
    per = run(W, corpus, q, 10.0, 15, schedule="per_iteration")
    unf = run(W, corpus, q, 10.0, 15, schedule="unfused")
    for b in range(q.B):
        ids, qw = q.query(b)
        ref = oracle_support(c, ids, qw, 10.0, 15)
        assert_close(res[b], ref, TOL32, f"resident, query width {len(ids)}")
        assert_close(per[b], res[b], 1e-6, f"per-iteration vs resident, width {len(ids)}")
        assert_close(unf[b], res[b], 1e-6, f"unfused vs resident, width {len(ids)}")


def test_merged_launches_match_separate_launches(W):
    """One launch over several length buckets computes what one launch per
    bucket computes.  A short bucket may run with more rows per lane in the
    shared launch (or another column layout), which reorders its float32 sums,
    so the two agree to rounding rather than bit for bit; both match the
    oracle on sampled documents."""
    rng = np.random.default_rng(44)
    lengths = np.concatenate([rng.integers(1, 300, size=700), rng.integers(300, 1100, size=40), [0, 0]])
    rng.shuffle(lengths)
    c = handmade_corpus(rng, 5000, 40, lengths)
    qs = [rng.choice(5000, size=v, replace=False) for v in (1, 7, 20, 33, 64, 130)]
    q = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(x) for x in qs])]),
                      ids=np.concatenate(qs).astype(np.int32),
                      weights=rng.integers(1, 4, size=sum(len(x) for x in qs)).astype(np.float32))
    corpus = corpus_of(W, c)
    merged = run(W, corpus, q, 10.0, 15)
    corpus.set_merge("none")
    separate = run(W, corpus, q, 10.0, 15)
    assert_close(merged, separate, 1e-5, "merged vs separate launches")
    with pytest.raises(W.WMDError):  # an unknown mode is rejected
        W._check(W.lib().wmd_set_merge(corpus._h, 7))
    docs = np.sort(rng.choice(len(lengths), size=40, replace=False))
    for b in range(q.B):
        ids, qw = q.query(b)
        ref = oracle_support(c, ids, qw, 10.0, 15, docs)
        assert_close(merged[b, docs], ref, TOL32, f"merged, query width {len(ids)}")


@pytest.mark.parametrize("d", [37, 130])
def test_embedding_widths_off_the_vector_path(W, d):
    """Widths that are not a multiple of 4 take the scalar row copies in query
    selection; 130 also pads to 192 columns in the cost matrix."""
    rng = np.random.default_rng(45 + d)
    c = handmade_corpus(rng, 3000, d, rng.integers(1, 90, size=120))
    qs = [rng.choice(3000, size=v, replace=False) for v in (6, 25, 40)]
    q = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(x) for x in qs])]),
                      ids=np.concatenate(qs).astype(np.int32),
                      weights=rng.integers(1, 4, size=sum(len(x) for x in qs)).astype(np.float32))
    corpus = corpus_of(W, c)
    got32 = run(W, corpus, q, 10.0, 15)
    got16 = run(W, corpus, q, 10.0, 15, cdist="bf16")
    for b in range(q.B):
        ids, qw = q.query(b)
        ref = oracle_support(c, ids, qw, 10.0, 15)
        assert_close(got32[b], ref, TOL32, f"d={d} fp32 query {b}")
        assert_close(got16[b], ref, TOL16, f"d={d} bf16 query {b}")


@pytest.mark.parametrize("vr", [1, 3, 4, 5, 9, 13, 21, 27, 30, 63, 64, 65, 500, 2048])
def test_query_widths(W, vr):
    """Every skinny cost-matrix column split (4-column groups, 16-column
    tiles and both) up to 32 padded columns, then the tiled kernel."""
    rng = np.random.default_rng(43 + vr)
    c = handmade_corpus(rng, 4000, 24, rng.integers(1, 60, size=50))
    ids = rng.choice(4000, size=vr, replace=False).astype(np.int32)
    q = synth.Queries(q_ptr=np.array([0, vr]), ids=ids, weights=rng.integers(1, 4, size=vr).astype(np.float32))
    got = run(W, corpus_of(W, c), q, 10.0, 15)[0]
    ref = oracle_support(c, ids, q.weights, 10.0, 15)
    assert_close(got, ref, TOL32, f"v_r={vr}")


def test_invalid_queries_are_nan_with_codes(W):
    rng = np.random.default_rng(44)
    c = handmade_corpus(rng, 300, 16, rng.integers(1, 20, size=10))
    corpus = corpus_of(W, c)
    q_ptr = np.array([0, 2, 4, 6, 8])
    ids = np.array([1, 2, 3, 300, 5, 6, 7, 8], np.int32)
    w = np.array([1, 1, 1, 1, 1, -1, 0, 0], np.float32)
    batch = W.QueryBatch.from_arrays(q_ptr, ids, w)
    with pytest.raises(ValueError):
        corpus.query(batch, 10.0, 15)
    out = corpus.query(batch, 10.0, 15, check=False)
    codes = corpus.query_errors(corpus.last_workspace, 4)
    assert list(codes) == [0, 1, 2, 3]
    o = out.cpu().numpy()
    assert np.all(np.isfinite(o[0])) and np.all(np.isnan(o[1:]))
    # each query alone: a short single query is selected inside the cost-matrix kernel
    for b in range(4):
        one = W.QueryBatch.from_arrays(np.array([0, 2]), ids[2 * b:2 * b + 2], w[2 * b:2 * b + 2])
        for cd in ("fp32", "bf16"):
            row = corpus.query(one, 10.0, 15, cdist=cd, check=False).cpu().numpy()[0]
            assert list(corpus.query_errors(corpus.last_workspace, 1)) == [b], f"query {b} alone, {cd}"
            assert np.all(np.isfinite(row)) if b == 0 else np.all(np.isnan(row)), f"query {b} alone, {cd}"
            if b == 0 and cd == "fp32":
                assert_close(row, o[0], 1e-6, "query 0 alone vs in the batch")


def test_corpus_validation_errors(W):
    rng = np.random.default_rng(45)
    c = handmade_corpus(rng, 100, 8, [3, 4])
    bad_ids = c.word_ids.copy()
    bad_ids[2] = 100
    with pytest.raises(W.WMDError):
        W.Corpus.from_numpy(c.emb, c.doc_ptr, bad_ids, c.weights)
    bad_w = c.weights.copy()
    bad_w[0] = -1
    with pytest.raises(W.WMDError):
        W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, bad_w)
    bad_w[0] = np.nan
    with pytest.raises(W.WMDError):
        W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, bad_w)
    with pytest.raises(W.WMDError):
        W.Corpus.from_numpy(c.emb, np.array([0, 4, 3, 7]), c.word_ids, c.weights)
    long = handmade_corpus(rng, 9000, 8, [4097], dup=True)
    with pytest.raises(W.WMDError):
        W.Corpus.from_numpy(long.emb, long.doc_ptr, long.word_ids, long.weights)


# ------------------------------------------------------- stop once x settles

@pytest.mark.parametrize("tol", [1e-2, 1e-4])
def test_tolerance_stop_counts_and_values(W, single, tol):
    """The GPU decides each document's iteration count k in float32.  k must
    lie between the oracle's counts at tol*1.1 and tol*0.9 (the decision may
    flip within rounding of the threshold), and the distance must match the
    oracle run for exactly k iterations."""
    c = single.corpus
    corpus = corpus_of(W, c)
    batch = W.QueryBatch.from_arrays(single.queries.q_ptr, single.queries.ids, single.queries.weights)
    iters = torch.zeros(c.N, dtype=torch.int32, device="cuda")
    got = corpus.query(batch, single.lam, 200, tol=tol, iters=iters)
    torch.cuda.synchronize()
    got, k = got.cpu().numpy()[0], iters.cpu().numpy()
    docs = sample_docs(c.N, seed=4)[:80]
    ids, qw = single.queries.query(0)
    _, k_hi = oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, single.lam, 200,
                                          docs=docs, tol=tol * 0.9)
    _, k_lo = oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, single.lam, 200,
                                          docs=docs, tol=tol * 1.1)
    kd = k[docs]
    assert np.all(kd >= 1) and np.all(kd <= 200)  # documents may run up to the cap
    assert np.all((k_lo <= kd) & (kd <= k_hi)), list(zip(k_lo, kd, k_hi))
    for kk in np.unique(kd):
        sel = docs[kd == kk]
        ref = oracle_support(c, ids, qw, single.lam, int(kk), sel)
        assert_close(got[sel], ref, TOL32, f"tol={tol} k={kk}")


@pytest.mark.parametrize("vr", [7, 12, 20])
def test_permuted_slot_shapes_every_schedule(W, vr):
    """One-wave shapes with 2 or 4 column lanes hold the rows of their small
    bodies (at most 40 cells per lane) in permuted register slots.  Each such
    shape, pinned in turn for documents of 1-16, 17-32 and 33-64 words,
    matches the oracle under the resident schedule, runs the same arithmetic
    under the per-iteration schedule (bitwise: w and u go through memory in the
    permuted order and come back) and agrees under the unfused one."""
    rng = np.random.default_rng(60 + vr)
    lengths = np.concatenate([rng.integers(1, 17, size=24), rng.integers(17, 33, size=24),
                              rng.integers(33, 65, size=24)])
    c = handmade_corpus(rng, 3000, 40, lengths)
    ids = rng.choice(3000, size=vr, replace=False).astype(np.int32)
    q = synth.Queries(q_ptr=np.array([0, vr]), ids=ids, weights=rng.integers(1, 4, size=vr).astype(np.float32))
    ref = oracle_support(c, ids, q.weights, 10.0, 15)
    corpus = corpus_of(W, c)
    S = (vr + 3) // 4 * 4
    tested = 0
    for cap in (16, 32, 64):
        for sh in corpus.sink_candidates(S, cap):
            if sh["maxw"] != 1 or sh["stream"] or sh["lg_cg"] not in (1, 2):
                continue
            try:
                corpus.set_sink_shape(S, cap, sh)
            except W.WMDError:
                continue  # a shape the library cannot run for this bucket
            what = f"S={S} cap={cap} shape={sh}"
            res = run(W, corpus, q, 10.0, 15)[0]
            per = run(W, corpus, q, 10.0, 15, schedule="per_iteration")[0]
            unf = run(W, corpus, q, 10.0, 15, schedule="unfused")[0]
            assert_close(res, ref, TOL32, what)
            assert np.array_equal(per, res), what
            assert_close(unf, res, 1e-6, what)
            tested += 1
        corpus.set_sink_shape(S, cap, None)
    assert tested >= 3, f"only {tested} permuted-slot shapes ran for S={S}"
