"""Exact earth mover's distance for tiny problems.

TEST INFRASTRUCTURE ONLY.  Used to pin the Sinkhorn oracle: the Sinkhorn
distance is bounded below by the exact transport cost and tends to it as the
entropic weight lambda grows (Section II-A, after Cuturi).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog


def emd_linprog(r, c, M) -> float:
    """min <P, M> s.t. P 1 = r, P^T 1 = c, P >= 0, solved by HiGHS."""
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    n, m = M.shape
    A = []
    for i in range(n):
        row = np.zeros((n, m))
        row[i, :] = 1
        A.append(row.ravel())
    for j in range(m):
        col = np.zeros((n, m))
        col[:, j] = 1
        A.append(col.ravel())
    b = np.concatenate([r, c])
    res = linprog(M.ravel(), A_eq=np.array(A), b_eq=b, bounds=(0, None), method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return float(res.fun)


def emd_vertices(r, c, M) -> float:
    """Brute force: the optimum of a linear program sits on a vertex of the
    transport polytope; a vertex is a feasible basic solution supported on
    n + m - 1 cells.  Enumerate every such support, solve the square system and
    keep the feasible minimum.  Only for n * m <= 16.
    """
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    n, m = M.shape
    if n * m > 16:
        raise ValueError("too large for enumeration")
    cells = [(i, j) for i in range(n) for j in range(m)]
    rhs = np.concatenate([r, c])
    best = np.inf
    for support in itertools.combinations(range(n * m), n + m - 1):
        A = np.zeros((n + m, n + m - 1))
        for col, idx in enumerate(support):
            i, j = cells[idx]
            A[i, col] = 1
            A[n + j, col] = 1
        sol, res, rank, _ = np.linalg.lstsq(A, rhs, rcond=None)
        if rank < n + m - 1:
            continue
        if np.abs(A @ sol - rhs).max() > 1e-12 or sol.min() < -1e-12:
            continue
        cost = sum(sol[col] * M[cells[idx]] for col, idx in enumerate(support))
        best = min(best, cost)
    return float(best)
