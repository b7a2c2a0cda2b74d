"""Calls from several host threads on one corpus, each with its own stream
and workspace, as include/wmd.h allows: two threads capture and replay graphs
while two call eagerly; then all four call with per-kernel timing on (timed
calls are serialised inside the library; graphs are not used while timing).
Every result equals the same call made alone, bit for bit."""
import threading

import numpy as np
import pytest
import torch

from paper_2107_06433_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    from paper_2107_06433_amd import wmd  # loads libwmd.so; fails loudly if missing
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return wmd


@pytest.mark.parametrize("timed", [False, True])
def test_threads_with_own_streams_eager_graph_and_timed(W, timed):
    w = synth.make_workload("batched", scale_docs=0.02)  # N = 1,000 documents, 64 queries
    c = w.corpus
    corpus = W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    Q = w.queries
    parts = [W.QueryBatch.from_arrays(*slice_queries(Q, lo, hi)) for lo, hi in ((0, 16), (16, 40), (40, 64), (5, 6))]
    refs = [corpus.query(b, w.lam, w.max_iter).cpu().numpy() for b in parts]
    errors = []
    results = {}

    def worker(i, graph):
        try:
            s = torch.cuda.Stream()
            b = parts[i]
            out = torch.empty((b.B, c.N), dtype=torch.float32, device="cuda")
            ws = torch.empty(corpus.workspace_bytes(b), dtype=torch.uint8, device="cuda")
            got = []
            for rep in range(6):
                with torch.cuda.stream(s):
                    out.fill_(float("nan"))
                corpus.query(b, w.lam, w.max_iter, out=out, workspace=ws, stream=s, check=False, graph=graph)
                s.synchronize()
                got.append(out.cpu().numpy().copy())
            results[i] = got
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((i, repr(e)))

    corpus.set_timing(timed)
    threads = [threading.Thread(target=worker, args=(i, g)) for i, g in ((0, True), (1, False), (2, False), (3, True))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    if timed:
        recs = corpus.launches()
        assert len(recs) >= 4 * 6 * 2 and all(r["ms"] > 0 for r in recs)
    corpus.set_timing(False)
    assert not errors, errors
    for i, ref in enumerate(refs):
        for rep, g in enumerate(results[i]):
            assert np.array_equal(g, ref), f"thread {i} call {rep} differs from the call alone"


def slice_queries(Q, lo, hi):
    a, b = int(Q.q_ptr[lo]), int(Q.q_ptr[hi])
    return Q.q_ptr[lo:hi + 1] - a, Q.ids[a:b], Q.weights[a:b]
