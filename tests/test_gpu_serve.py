"""Serving path on the GPU: every result is the same alone and in the mix.

Queries go through the continuous-batching server (batches formed from
whatever has arrived, several batches in flight on different streams) and are
compared with the same query scored alone through the C ABI: the per-query
arithmetic does not depend on its batch-mates, so the rows must be bitwise
equal.  A sample is also checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2107_06433_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2107_06433_amd import wmd
    w = synth.make_workload("serving", scale_docs=0.01, n_queries=48)  # N = 2,000 documents
    c = w.corpus
    corpus = wmd.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    return w, corpus, wmd


def alone(wmd, corpus, w, b, cdist):
    ids, qw = w.queries.query(b)
    batch = wmd.QueryBatch.from_arrays([0, len(ids)], ids, qw)
    out = corpus.query(batch, w.lam, w.max_iter, cdist=cdist)
    torch.cuda.synchronize()
    return out.cpu().numpy()[0]


def test_server_results_equal_alone_and_oracle(setup):
    from paper_2107_06433_amd import serve
    w, corpus, wmd = setup
    srv = serve.Server(corpus, w.lam, w.max_iter, cdist="bf16", mem_budget=2 << 30, max_batch=8, max_inflight=3)
    futs = [srv.submit(*w.queries.query(b)) for b in range(w.queries.B)]
    rows = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.sched.batches > 1
    for b in range(w.queries.B):
        got = rows[b].numpy()
        assert np.array_equal(got, alone(wmd, corpus, w, b, "bf16")), f"query {b} differs in the mix"
    rng = np.random.default_rng(5)
    c = w.corpus
    for b in (0, 7, 31):
        docs = np.sort(rng.choice(c.N, size=25, replace=False))
        ids, qw = w.queries.query(b)
        ref = oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter,
                                          docs=docs)
        g = rows[b].numpy()[docs].astype(np.float64)
        assert np.all(np.abs(g - ref) <= 1e-3 * np.abs(ref) + 1e-7)


def test_open_loop_trace_and_budget_rejection(setup):
    from paper_2107_06433_amd import serve
    w, corpus, wmd = setup
    ex = serve.GpuExecutor(corpus, w.lam, w.max_iter, cdist="bf16", streams=2)
    one = ex.cost([serve.Request(ids=w.queries.query(0)[0], weights=w.queries.query(0)[1], arrival=0.0)])
    widest = int(np.argmax(np.diff(w.queries.q_ptr)))
    big = ex.cost([serve.Request(ids=w.queries.query(widest)[0], weights=w.queries.query(widest)[1], arrival=0.0)])
    budget = max(one * 3, big - 1) if big > one * 3 else one * 3
    sch = serve.Scheduler(ex, budget, max_batch=4, max_inflight=2)
    reqs = [serve.Request(ids=w.queries.query(b)[0], weights=w.queries.query(b)[1], arrival=0.0)
            for b in range(w.queries.B)]
    arr = np.linspace(0.0, 0.05, len(reqs))
    st = serve.run_trace(sch, reqs, arr)
    assert st["completed"] + st["rejected"] == len(reqs)
    assert sch.peak_used <= budget
    for r in reqs:
        if r.future.exception() is None:
            assert np.array_equal(r.future.result().numpy(), alone(wmd, corpus, w, r.rid, "bf16"))
        else:
            assert isinstance(r.future.exception(), serve.RejectedError)
            assert ex.cost([r]) > budget
