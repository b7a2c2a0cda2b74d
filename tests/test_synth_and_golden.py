import os

import numpy as np

import oracle
from paper_2107_06433_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_wmd.txt")


def test_generator_is_deterministic_and_well_formed():
    a = synth.make_workload("tiny")
    b = synth.make_workload("tiny")
    for x, y in [(a.corpus.emb, b.corpus.emb), (a.corpus.word_ids, b.corpus.word_ids),
                 (a.corpus.weights, b.corpus.weights), (a.queries.ids, b.queries.ids)]:
        assert np.array_equal(x, y)
    c = a.corpus
    assert c.emb.dtype == np.float32 and c.emb.shape == (2000, 64)
    assert c.doc_ptr[0] == 0 and np.all(np.diff(c.doc_ptr) >= 10) and np.all(np.diff(c.doc_ptr) <= 30)
    assert c.word_ids.min() >= 0 and c.word_ids.max() < c.V
    for k in range(c.N):
        ids = c.word_ids[c.doc_ptr[k]:c.doc_ptr[k + 1]]
        assert np.all(np.diff(ids) > 0)  # unique and ascending
    assert np.all(c.weights >= 1) and np.all(c.weights == np.round(c.weights))
    assert a.queries.B == 1 and len(a.queries.ids) == 8


def test_zipf_ids_favour_low_ranks():
    rng = synth.rng_for(5)
    cdf = synth.zipf_cdf(1000)
    _, ids = synth.unique_bags(rng, cdf, np.full(2000, 5))
    counts = np.bincount(ids, minlength=1000)
    assert counts[0] > counts[10] > counts[500]


def test_batched_query_lengths_in_range():
    w = synth.make_workload("batched", scale_docs=0.002)
    lens = np.diff(w.queries.q_ptr)
    assert w.queries.B == 64 and lens.min() >= 5 and lens.max() <= 200


def test_oracle_reproduces_tiny_golden():
    want = np.loadtxt(GOLDEN)
    w = synth.make_workload("tiny")
    c = w.corpus
    ids, qw = w.queries.query(0)
    got = oracle.wmd_dense_corpus(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    sup = oracle.sinkhorn_wmd_support(c.emb, c.doc_ptr, c.word_ids, c.weights, ids, qw, w.lam, w.max_iter)
    np.testing.assert_allclose(sup, want, rtol=1e-11)
