"""Plain float64 Sinkhorn WMD, written from Algorithm 1 and Table I of the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation follows Section III-A: ``r`` is the query histogram restricted to its
nonzero words (length ``v_r``), ``c`` the V x N matrix of target-document
histograms (columns sum to one), ``M`` the v_r x V Euclidean cost matrix,
``K = exp(-lambda M)``, ``x`` / ``u = 1/x`` the v_r x N row scalings and ``v``
the sparse V x N column scalings.

Readings of points the paper leaves open (each is listed in the design doc):

* the cost is the plain Euclidean distance (Section II-A gives the square-root
  form; Table I calls ``cdist`` with its default metric);
* ``K = exp(-lambda M)`` with ``lambda > 0`` (Algorithm 1; the prose of
  Section III-B-1 passes a negated lambda, which is the same thing);
* the loop that repeats until x stops changing runs exactly ``max_iter`` times (the cut-off of
  Section III-B-1); the final u, v update follows it;
* ``k^T`` in the update of Algorithm 1 is ``K^T``;
* duplicate query words are summed (``r`` is a histogram over the vocabulary),
  zero weights are dropped, ``r`` and every column of ``c`` are normalised to
  sum to one;
* a document whose weights sum to zero (or that has no words) gives NaN.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def select_query(V: int, ids, weights):
    """Algorithm 1, first step (``I = (r > 0); r = r(I)``).

    Builds the query histogram over the vocabulary (duplicates summed),
    normalises it to sum 1 (Section III-B-1) and keeps the words with r > 0,
    in ascending vocabulary order.  Returns ``(sel, r)``.
    """
    ids = np.asarray(ids, dtype=np.int64)
    w = np.asarray(weights, dtype=np.float64)
    if ids.size == 0:
        raise ValueError("empty query")
    if ids.min() < 0 or ids.max() >= V:
        raise ValueError("query word id out of range")
    if not np.all(np.isfinite(w)) or np.any(w < 0):
        raise ValueError("query weights must be finite and >= 0")
    r_full = np.zeros(V, dtype=np.float64)
    np.add.at(r_full, ids, w)
    total = r_full.sum()
    if not total > 0:
        raise ValueError("query has no positive weight")
    r_full /= total
    sel = np.nonzero(r_full > 0)[0]
    return sel, r_full[sel]


def normalized_columns(V: int, doc_ptr, word_ids, weights) -> sp.csc_matrix:
    """The paper's ``c``: V x N sparse, each column divided by its sum.

    Duplicate word ids inside a document are summed (histogram semantics).
    A column whose sum is zero becomes all-NaN in its stored entries, which
    makes that document's distance NaN.
    """
    # private copies: scipy sorts the index arrays it is given in place
    doc_ptr = np.array(doc_ptr, dtype=np.int64, copy=True)
    N = len(doc_ptr) - 1
    data = np.array(weights, dtype=np.float64, copy=True)
    rows = np.array(word_ids, dtype=np.int64, copy=True)
    c = sp.csc_matrix((data, rows, doc_ptr), shape=(V, N))
    c.sum_duplicates()
    col_sum = np.asarray(c.sum(axis=0)).ravel()
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = 1.0 / col_sum
    c = c @ sp.diags(scale)
    return sp.csc_matrix(c)


def cost_rows(E, sel) -> np.ndarray:
    """``M[i, j] = sqrt(sum_t (E[sel_i, t] - E[j, t])^2)`` for every vocabulary word j.

    The lazily computed v_r x V cost matrix of Table I (``cdist(vecs[sel],
    vecs)``), evaluated as the difference form in float64, so the distance of
    a word to itself is exactly zero.
    """
    E = np.asarray(E, dtype=np.float64)
    sel = np.asarray(sel, dtype=np.int64)
    M = np.empty((len(sel), E.shape[0]), dtype=np.float64)
    for i, q in enumerate(sel):
        diff = E - E[q]
        M[i] = np.sqrt(np.einsum("ij,ij->i", diff, diff))
    return M


def sinkhorn_scalings(r, M, c, lam: float, max_iter: int):
    """Algorithm 1 on dense arrays; returns the final ``(u, v, K)``.

    ``r``: (v_r,) ; ``M``: (v_r, V) ; ``c``: dense (V, n) histogram columns.
    ``x`` starts at ``1/v_r``; each of the ``max_iter`` iterations sets
    ``u = 1/x``, ``v = c .* 1/(K^T u)`` (only where c > 0, as the sparse
    ``c.multiply`` of Table I) and ``x = diag(1/r) K v``; afterwards one more
    ``u``, ``v`` update gives the returned scalings.
    """
    r = np.asarray(r, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    K = np.exp(-lam * M)
    v_r = r.shape[0]
    x = np.ones((v_r, c.shape[1]), dtype=np.float64) / v_r
    mask = c > 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for _ in range(max_iter):
            u = 1.0 / x
            v = np.where(mask, c / (K.T @ u), 0.0)
            x = (1.0 / r)[:, None] * (K @ v)
        u = 1.0 / x
        v = np.where(mask, c / (K.T @ u), 0.0)
    return u, v, K


def sinkhorn_scalings_until(r, M, c, lam: float, max_iter: int, tol: float):
    """Algorithm 1 with its loop until x stops changing, for one document column.

    Iterates as ``sinkhorn_scalings`` but stops after the first iteration whose
    relative change of x, max_i |x_new_i - x_i| / x_new_i, is at most ``tol``
    (at ``max_iter`` iterations at the latest).  Returns ``(u, v, K, iters)``.
    """
    r = np.asarray(r, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64).reshape(-1, 1)
    K = np.exp(-lam * M)
    x = np.ones((r.shape[0], 1), dtype=np.float64) / r.shape[0]
    mask = c > 0
    done = 0
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        for it in range(max_iter):
            u = 1.0 / x
            v = np.where(mask, c / (K.T @ u), 0.0)
            x_new = (1.0 / r)[:, None] * (K @ v)
            change = np.max(np.abs(x_new - x) / x_new)
            x = x_new
            done = it + 1
            if change <= tol:
                break
        u = 1.0 / x
        v = np.where(mask, c / (K.T @ u), 0.0)
    return u, v, K, done


def sinkhorn_wmd_dense(r, M, c, lam: float, max_iter: int) -> np.ndarray:
    """``d_M^lambda(r, c) = sum(u .* ((K .* M) v))`` per column (Algorithm 1, last line)."""
    u, v, K = sinkhorn_scalings(r, M, c, lam, max_iter)
    with np.errstate(invalid="ignore", over="ignore"):
        return np.sum(u * ((K * M) @ v), axis=0)


def transport_plan(u_col, v_col, K) -> np.ndarray:
    """``P = diag(u) K diag(v)`` for one document (Cuturi's form of the solution)."""
    return u_col[:, None] * K * v_col[None, :]


def wmd_dense_corpus(E, doc_ptr, word_ids, weights, q_ids, q_weights, lam: float,
                     max_iter: int, docs=None, block: int = 256) -> np.ndarray:
    """Dense full-vocabulary Algorithm 1 for one query against a corpus.

    Every operation of Algorithm 1 acts on each column of ``c`` on its own, so
    the documents are fed in column blocks of ``block`` to bound memory; the
    numbers produced for a column do not depend on which other columns share
    its block.  ``docs`` optionally selects a subset of documents.
    """
    E = np.asarray(E)
    V = E.shape[0]
    sel, r = select_query(V, q_ids, q_weights)
    M = cost_rows(E, sel)
    c = normalized_columns(V, doc_ptr, word_ids, weights)
    if docs is not None:
        c = c[:, np.asarray(docs, dtype=np.int64)]
    out = np.empty(c.shape[1], dtype=np.float64)
    for s in range(0, c.shape[1], block):
        cb = c[:, s:s + block].toarray()
        out[s:s + block] = sinkhorn_wmd_dense(r, M, cb, lam, max_iter)
    return out


def sinkhorn_wmd_support(E, doc_ptr, word_ids, weights, q_ids, q_weights, lam: float,
                         max_iter: int, docs=None, tol: float | None = None):
    """The same iteration restricted to each document's own words.

    For document k only the rows of ``c`` with ``c_jk > 0`` take part (every
    other entry of v is zero), so Algorithm 1 reduces to Cuturi's Sinkhorn on
    the v_r x n_k cost matrix ``M[:, words of k]``.  Documents are processed
    one at a time with the dense routine above on that small problem.  With
    ``tol`` each document stops as ``sinkhorn_scalings_until`` does, and the
    iteration counts are returned as a second array.
    """
    E = np.asarray(E)
    V = E.shape[0]
    sel, r = select_query(V, q_ids, q_weights)
    Eq = np.asarray(E[sel], dtype=np.float64)
    doc_ptr = np.asarray(doc_ptr, dtype=np.int64)
    N = len(doc_ptr) - 1
    docs = np.arange(N) if docs is None else np.asarray(docs, dtype=np.int64)
    out = np.empty(len(docs), dtype=np.float64)
    its = np.zeros(len(docs), dtype=np.int64)
    for n, k in enumerate(docs):
        s, e = doc_ptr[k], doc_ptr[k + 1]
        ids = np.asarray(word_ids[s:e], dtype=np.int64)
        w = np.asarray(weights[s:e], dtype=np.float64)
        tot = w.sum()
        if not tot > 0:
            out[n] = np.nan
            continue
        # merge duplicate words of the document (histogram semantics)
        uid, inv = np.unique(ids, return_inverse=True)
        cw = np.zeros(len(uid))
        np.add.at(cw, inv, w)
        cw /= tot
        keep = cw > 0
        uid, cw = uid[keep], cw[keep]
        Ed = np.asarray(E[uid], dtype=np.float64)
        diff = Eq[:, None, :] - Ed[None, :, :]
        Md = np.sqrt(np.einsum("ijt,ijt->ij", diff, diff))
        if tol is None:
            out[n] = sinkhorn_wmd_dense(r, Md, cw[:, None], lam, max_iter)[0]
        else:
            u, v, K, its[n] = sinkhorn_scalings_until(r, Md, cw, lam, max_iter, tol)
            with np.errstate(invalid="ignore", over="ignore"):
                out[n] = np.sum(u * ((K * Md) @ v), axis=0)[0]
    return out if tol is None else (out, its)
