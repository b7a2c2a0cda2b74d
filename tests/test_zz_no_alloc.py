"""wmd_query_static (the query entry point that allocates nothing: its query
workspace is the library's static device scratch) against wmd_query with a
caller workspace, through the C ABI.

Both run the same kernels on the same inputs, so the distances must be equal
bit for bit.  Two static calls in a row, the second with fewer and narrower
queries, show that what the first left in the shared scratch does not leak
into the second.  A call that needs more workspace than the scratch holds is
refused.
"""
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


def queries_of(parts):
    lens = [len(a) for a, _ in parts]
    return (np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
            np.concatenate([a for a, _ in parts]).astype(np.int32),
            np.concatenate([b for _, b in parts]).astype(np.float32))


def test_static_scratch_matches_workspace_entry_point(W):
    w = synth.make_workload("single")
    c = w.corpus
    corpus = W.Corpus.from_numpy(c.emb, c.doc_ptr, c.word_ids, c.weights)
    rng = np.random.default_rng(21)
    ids0, qw0 = w.queries.query(0)
    wide = (rng.choice(c.V, size=70, replace=False), rng.integers(1, 4, size=70).astype(np.float32))
    mid = (rng.choice(c.V, size=33, replace=False), rng.integers(1, 4, size=33).astype(np.float32))
    first = W.QueryBatch.from_arrays(*queries_of([wide, (ids0, qw0), mid]))
    second = W.QueryBatch.from_arrays(*queries_of([(ids0[:9], qw0[:9])]))
    assert corpus.workspace_bytes(first) <= W.lib().wmd_query_static_capacity()
    for cd in ("fp32", "bf16"):
        refs = [corpus.query(b, w.lam, w.max_iter, cdist=cd).cpu().numpy() for b in (first, second)]
        for rep in range(2):
            outs = [torch.full((b.B, c.N), float("nan"), dtype=torch.float32, device="cuda") for b in (first, second)]
            torch.cuda.synchronize()
            # nothing is allocated meanwhile: torch's peak stays where it is and
            # the device's free memory is unchanged (the library calls no hipMalloc)
            torch.cuda.reset_peak_memory_stats()
            peak = torch.cuda.max_memory_allocated()
            free = torch.cuda.mem_get_info()[0]
            for b, o in zip((first, second), outs):
                corpus.query_static(b, w.lam, w.max_iter, o, cdist=cd)
            torch.cuda.synchronize()
            assert torch.cuda.max_memory_allocated() <= peak
            assert torch.cuda.mem_get_info()[0] == free
            for o, r in zip(outs, refs):
                got = o.cpu().numpy()
                assert np.isfinite(got).all()
                assert np.array_equal(got, r), f"{cd} repetition {rep}: static scratch differs from a workspace"


def test_static_scratch_refuses_what_does_not_fit(W):
    rng = np.random.default_rng(22)
    V, d = 20_000, 32
    E = (rng.standard_normal((V, d)) / np.sqrt(d)).astype(np.float32)
    lengths = rng.integers(5, 40, size=200)
    ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    ids = np.concatenate([rng.choice(V, size=n, replace=False) for n in lengths]).astype(np.int32)
    corpus = W.Corpus.from_numpy(E, ptr, ids, rng.integers(1, 4, size=len(ids)).astype(np.float32))
    cap = W.lib().wmd_query_static_capacity()
    U = corpus.info()["U"]
    width = 2048
    nq = cap // (4 * U * width) + 1  # enough full-width queries to overflow the scratch
    parts = [(rng.choice(V, size=width, replace=False), np.ones(width, np.float32)) for _ in range(nq)]
    big = W.QueryBatch.from_arrays(*queries_of(parts))
    assert corpus.workspace_bytes(big) > cap
    out = torch.empty((big.B, corpus.N), dtype=torch.float32, device="cuda")
    with pytest.raises(W.WMDError) as e:
        corpus.query_static(big, 10.0, 15, out)
    assert e.value.status == 4 and "static scratch" in str(e.value)
    # and it still works afterwards for a call that fits
    one = W.QueryBatch.from_arrays(*queries_of(parts[:1]))
    o = torch.empty((1, corpus.N), dtype=torch.float32, device="cuda")
    corpus.query_static(one, 10.0, 15, o)
    ref = corpus.query(one, 10.0, 15).cpu().numpy()
    assert np.array_equal(o.cpu().numpy(), ref)
