"""Parity at the full sizes the benchmark runs: the batched workload (64
queries of 5-200 words against 50,000 documents) and the serving corpus
(200,000 documents over a 300,000-word vocabulary).

The calls are the ones the benchmark makes (same corpus, same query batch,
same options), so the kernel shapes the shape model picks for them -- which
depend on the query widths and on how many documents each length bucket
holds -- are the ones that run here.  The oracle cannot score every document
of every query in seconds, so each query is checked on documents drawn from
every length bucket (its shortest and longest documents among them): every
Sinkhorn launch of the call, and every row body inside it, computes some of
the checked distances.  The timing records of the call name the launches;
the test asserts that each one ran a bucket with checked documents.
"""
import numpy as np
import pytest
import torch

from paper_2107_06433_amd import synth

from test_gpu_parity import TOL16, TOL32, assert_close, oracle_support

pytestmark = pytest.mark.gpu

BUCKET_CAPS = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]


@pytest.fixture(scope="module")
def W():
    from paper_2107_06433_amd import wmd  # loads libwmd.so; fails loudly if missing
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wmd


def bucket_of(lengths):
    return np.searchsorted(np.array(BUCKET_CAPS), lengths, side="left")


def stratified_docs(doc_ptr, per_bucket, total, seed):
    """Documents from every length bucket: its shortest and longest ones and
    random others (per_bucket each), then random documents up to total."""
    lengths = np.diff(doc_ptr)
    bk = bucket_of(lengths)
    rng = np.random.default_rng(seed)
    pick = []
    for b in np.unique(bk[lengths > 0]):
        ids = np.nonzero((bk == b) & (lengths > 0))[0]
        order = ids[np.argsort(lengths[ids], kind="stable")]
        chosen = {int(order[0]), int(order[-1])}
        rest = rng.choice(ids, size=min(len(ids), per_bucket), replace=False)
        for k in rest:
            if len(chosen) >= per_bucket:
                break
            chosen.add(int(k))
        pick.extend(sorted(chosen))
    pick = set(pick)
    while len(pick) < min(total, len(lengths)):
        pick.add(int(rng.integers(len(lengths))))
    return np.array(sorted(pick), dtype=np.int64)


def check_launch_coverage(launches, doc_ptr, checked):
    """Every query has checked documents in every length bucket the corpus
    has, so whatever (query, bucket) pairs a Sinkhorn launch runs -- one
    query's buckets, or the same buckets of several queries that share the
    launch -- some of its distances are checked.  Each launch record names a
    bucket capacity (0 when several buckets share the launch) that must be one
    of those buckets."""
    lengths = np.diff(doc_ptr)
    bk = bucket_of(lengths)
    present = set(bk[lengths > 0].tolist())
    for docs in checked:
        assert set(bk[docs].tolist()) >= present
    names = set()
    for rec in launches:
        if not rec["name"].startswith("sink"):
            continue
        names.add(rec["name"])
        if rec["cap"]:
            assert BUCKET_CAPS.index(rec["cap"]) in present, rec
    return sorted(names)


# ------------------------------------------------------------------ batched

@pytest.fixture(scope="module")
def batched(W):
    w = synth.make_workload("batched")
    c = w.corpus
    corpus = W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    Q = w.queries
    checked, refs = [], []
    for b in range(Q.B):
        docs = stratified_docs(c.doc_ptr, per_bucket=12, total=64, seed=100 + b)
        ids, qw = Q.query(b)
        checked.append(docs)
        refs.append(oracle_support(c, ids, qw, w.lam, w.max_iter, docs))
    return w, corpus, checked, refs


@pytest.mark.parametrize("cd,tol", [("fp32", TOL32), ("bf16", TOL16)])
def test_batched_full_size(W, batched, cd, tol):
    w, corpus, checked, refs = batched
    Q = w.queries
    batch = W.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights)
    corpus.set_timing(True)
    out = corpus.query(batch, w.lam, w.max_iter, cdist=cd)
    torch.cuda.synchronize()
    launches = corpus.launches()
    corpus.set_timing(False)
    g = out.cpu().numpy()
    assert np.isfinite(g).all()
    for b in range(Q.B):
        assert_close(g[b, checked[b]], refs[b], tol, f"batched {cd} query {b} (v_r={Q.q_ptr[b + 1] - Q.q_ptr[b]})")
    names = check_launch_coverage(launches, w.corpus.doc_ptr, checked)
    print(f"batched {cd}: {len(launches)} launches, Sinkhorn shapes {names}")
    assert any(n.startswith("sink_kernel<") for n in names), "the multi-wave shapes were not exercised"


def test_batched_full_size_queries_alone_match_the_batch(W, batched):
    """Four queries of the full batch, each alone (plain per-query calls): the
    same distances as in the batched call (bitwise with bf16 inputs)."""
    w, corpus, checked, refs = batched
    Q = w.queries
    full = corpus.query(W.QueryBatch.from_arrays(Q.q_ptr, Q.ids, Q.weights), w.lam, w.max_iter,
                        cdist="bf16").cpu().numpy()
    for b in (0, 9, 31, int(np.argmax(np.diff(Q.q_ptr)))):
        ids, qw = Q.query(b)
        one = corpus.query(W.QueryBatch.from_arrays([0, len(ids)], ids, qw), w.lam, w.max_iter,
                           cdist="bf16").cpu().numpy()[0]
        assert np.array_equal(one, full[b]), f"query {b} alone differs from the batch"


# ------------------------------------------------------------------ serving

@pytest.fixture(scope="module")
def serving(W):
    w = synth.make_workload("serving", n_queries=4000)
    c = w.corpus
    corpus = W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    Q = w.queries
    vr = np.diff(Q.q_ptr)
    rng = np.random.default_rng(9)
    longest = list(np.argsort(vr, kind="stable")[::-1][:8])
    others = [int(b) for b in rng.choice(Q.B, size=40, replace=False) if b not in longest][:24]
    sel = sorted(int(b) for b in longest + others)
    assert vr[sel].max() >= 256 and len(sel) == 32
    checked, refs = [], []
    for i, b in enumerate(sel):
        docs = stratified_docs(c.doc_ptr, per_bucket=10, total=32, seed=300 + i)
        ids, qw = Q.query(b)
        checked.append(docs)
        refs.append(oracle_support(c, ids, qw, w.lam, w.max_iter, docs))
    return w, corpus, sel, checked, refs


def test_serving_full_size_mix_alone_and_oracle(W, serving):
    """32 queries (the 8 longest of 4,000, up to the 500-word cap, and 24
    others) through the continuous-batching server on the full serving corpus:
    each result equals the same query scored alone (bitwise) and the FP64
    oracle (bf16 cost-matrix tolerance); the same batch as one fp32 call
    matches the oracle at the fp32 tolerance."""
    from paper_2107_06433_amd import serve
    w, corpus, sel, checked, refs = serving
    Q = w.queries
    srv = serve.Server(corpus, w.lam, w.max_iter, cdist="bf16", mem_budget=8 << 30, max_batch=6, max_inflight=3)
    futs = [srv.submit(*Q.query(b)) for b in sel]
    rows = [f.result(timeout=300) for f in futs]
    srv.close()
    assert srv.sched.batches > 1
    for i, b in enumerate(sel):
        ids, qw = Q.query(b)
        alone = corpus.query(W.QueryBatch.from_arrays([0, len(ids)], ids, qw), w.lam, w.max_iter,
                             cdist="bf16").cpu().numpy()[0]
        got = rows[i].numpy()
        assert np.array_equal(got, alone), f"query {b} (v_r={len(ids)}) differs in the mix"
        assert_close(got[checked[i]], refs[i], TOL16, f"serving bf16 query {b} (v_r={len(ids)})")
    sub = synth.Queries(q_ptr=np.concatenate([[0], np.cumsum([len(Q.query(b)[0]) for b in sel])]),
                        ids=np.concatenate([Q.query(b)[0] for b in sel]),
                        weights=np.concatenate([Q.query(b)[1] for b in sel]))
    corpus.set_timing(True)
    g32 = corpus.query(W.QueryBatch.from_arrays(sub.q_ptr, sub.ids, sub.weights), w.lam, w.max_iter).cpu().numpy()
    launches = corpus.launches()
    corpus.set_timing(False)
    for i, b in enumerate(sel):
        assert_close(g32[i, checked[i]], refs[i], TOL32, f"serving fp32 query {b}")
    names = check_launch_coverage(launches, w.corpus.doc_ptr, checked)
    print(f"serving fp32: Sinkhorn shapes {names}")
