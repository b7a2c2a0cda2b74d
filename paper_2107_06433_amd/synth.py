"""Seeded synthetic inputs for Sinkhorn WMD workloads.

This module only draws numbers: embeddings, Zipf-distributed word ids, word
counts, query lengths and arrival times.  It holds none of the method's
arithmetic (no normalisation, no distances, no Sinkhorn step): both the GPU path
and the FP64 oracle take its raw output and do their own work on it.

Stand-ins for the paper's data (Section III-B-2: 100,000 x 300 fastText vectors,
dbpedia documents), which are not available here:

* embeddings ``E = standard_normal((V, d)) / sqrt(d)`` cast to float32; the
  float32 values are canonical and the oracle up-casts them exactly;
* word ids Zipf(s=1.1) over a finite vocabulary by inverse CDF, rank k -> id
  k-1 (frequent words have low ids, as in a frequency-sorted vocabulary);
* every document (and query) has ``n`` *unique* ids (duplicates redrawn), with
  counts ``Poisson(2) + 1`` as float32 integers (raw counts, not normalised);
* documents are stored doc-major: ``doc_ptr[N+1]`` (int64), ``word_ids[nnz]``
  (int32, ascending inside a document), ``counts[nnz]`` (float32).  This is the
  CSC form of the paper's V x N histogram matrix ``c``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ZIPF_S = 1.1


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def embeddings(rng: np.random.Generator, V: int, d: int) -> np.ndarray:
    """V x d float32 embedding table, entries ~ N(0, 1/d)."""
    return (rng.standard_normal((V, d)) / math.sqrt(d)).astype(np.float32)


def zipf_cdf(V: int, s: float = ZIPF_S) -> np.ndarray:
    w = np.arange(1, V + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def _draw_ids(rng: np.random.Generator, cdf: np.ndarray, n: int) -> np.ndarray:
    u = rng.random(n)
    ids = np.searchsorted(cdf, u, side="right")
    return np.minimum(ids, len(cdf) - 1).astype(np.int64)


def unique_bags(rng: np.random.Generator, cdf: np.ndarray, lengths: np.ndarray):
    """Draw len(lengths) bags of unique Zipf ids; bag i has lengths[i] ids.

    Returns (ptr int64[n_bags+1], ids int32[total]) with ids ascending in each bag.
    Duplicates inside a bag are redrawn until none remain: each round finds,
    in (bag, id, position) order, every entry that repeats an earlier one of
    its bag and draws new ids for them in that order.  Only the bags that had
    a repeat can have one in the next round, so later rounds look at those
    bags alone (the draws are the same as re-examining every bag).
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    ptr = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=ptr[1:])
    total = int(ptr[-1])
    bag = np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)
    ids = _draw_ids(rng, cdf, total)
    live = np.arange(total, dtype=np.int64)  # positions examined this round, ascending
    while live.size:
        lb, li = bag[live], ids[live]
        order = np.lexsort((li, lb))
        sb, si = lb[order], li[order]
        dup = (sb[1:] == sb[:-1]) & (si[1:] == si[:-1])
        if not dup.any():
            break
        pos = live[order[1:][dup]]
        ids[pos] = _draw_ids(rng, cdf, len(pos))
        hit = np.zeros(len(lengths), dtype=bool)
        hit[bag[pos]] = True
        live = np.nonzero(hit[bag])[0]
    order = np.lexsort((ids, bag))
    return ptr, ids[order].astype(np.int32)


def counts(rng: np.random.Generator, n: int) -> np.ndarray:
    return (rng.poisson(2.0, size=n) + 1).astype(np.float32)


@dataclass
class Corpus:
    V: int
    d: int
    emb: np.ndarray          # float32 [V, d]
    doc_ptr: np.ndarray      # int64 [N+1]
    word_ids: np.ndarray     # int32 [nnz]
    weights: np.ndarray      # float32 [nnz] raw counts

    @property
    def N(self) -> int:
        return len(self.doc_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.doc_ptr[-1])


@dataclass
class Queries:
    q_ptr: np.ndarray        # int64 [B+1]
    ids: np.ndarray          # int32 [T]
    weights: np.ndarray      # float32 [T] raw counts

    @property
    def B(self) -> int:
        return len(self.q_ptr) - 1

    def query(self, b: int):
        s, e = int(self.q_ptr[b]), int(self.q_ptr[b + 1])
        return self.ids[s:e], self.weights[s:e]


@dataclass
class Workload:
    name: str
    corpus: Corpus
    queries: Queries
    lam: float
    max_iter: int
    arrivals: np.ndarray | None = None   # seconds, serving workloads only
    info: dict = field(default_factory=dict)


def make_corpus(rng, V, d, N, n_lo, n_hi, cdf=None) -> Corpus:
    E = embeddings(rng, V, d)
    cdf = zipf_cdf(V) if cdf is None else cdf
    lengths = rng.integers(n_lo, n_hi + 1, size=N)
    ptr, ids = unique_bags(rng, cdf, lengths)
    w = counts(rng, len(ids))
    return Corpus(V=V, d=d, emb=E, doc_ptr=ptr, word_ids=ids, weights=w)


def make_queries(rng, cdf, lengths) -> Queries:
    ptr, ids = unique_bags(rng, cdf, np.asarray(lengths, dtype=np.int64))
    w = counts(rng, len(ids))
    return Queries(q_ptr=ptr, ids=ids, weights=w)


# The five workloads.  Seeds are 1000 + workload number; the BF16 precision
# variant reuses the plain single-query inputs so that its error is measured on
# exactly the same problem.
WORKLOADS = {
    "tiny": dict(V=2_000, d=64, N=100, n_lo=10, n_hi=30, vr=8, lam=10.0, iters=15, seed=1001),
    "single": dict(V=100_000, d=300, N=5_000, n_lo=20, n_hi=100, vr=20, lam=10.0, iters=15, seed=1002),
    "batched": dict(V=100_000, d=300, N=50_000, n_lo=20, n_hi=100, B=64, vr_lo=5, vr_hi=200,
                    lam=10.0, iters=15, seed=1004),
    "serving": dict(V=300_000, d=300, N=200_000, n_lo=20, n_hi=60, vr_median=25.0, vr_sigma=1.0,
                    vr_cap=500, rate=2000.0, n_queries=22_000, lam=10.0, iters=15, seed=1005),
}


def make_workload(name: str, scale_docs: float = 1.0, n_queries: int | None = None) -> Workload:
    """Build a named workload.  ``scale_docs`` < 1 shrinks N (tests only)."""
    p = dict(WORKLOADS[name])
    rng = rng_for(p["seed"])
    N = max(1, int(round(p["N"] * scale_docs)))
    cdf = zipf_cdf(p["V"])
    corpus = make_corpus(rng, p["V"], p["d"], N, p["n_lo"], p["n_hi"], cdf)
    arrivals = None
    if name in ("tiny", "single"):
        queries = make_queries(rng, cdf, [p["vr"]])
    elif name == "batched":
        B = p["B"] if n_queries is None else n_queries
        lengths = rng.integers(p["vr_lo"], p["vr_hi"] + 1, size=B)
        queries = make_queries(rng, cdf, lengths)
    elif name == "serving":
        B = p["n_queries"] if n_queries is None else n_queries
        raw = rng.lognormal(mean=math.log(p["vr_median"]), sigma=p["vr_sigma"], size=B)
        lengths = np.clip(np.rint(raw), 1, p["vr_cap"]).astype(np.int64)
        queries = make_queries(rng, cdf, lengths)
        arr_rng = rng_for(p["seed"] + 1)
        arrivals = np.cumsum(arr_rng.exponential(1.0 / p["rate"], size=B))
    else:
        raise KeyError(name)
    return Workload(name=name, corpus=corpus, queries=queries, lam=float(p["lam"]),
                    max_iter=int(p["iters"]), arrivals=arrivals, info=p)
