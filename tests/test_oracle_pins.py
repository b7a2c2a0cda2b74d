"""Pins for the FP64 oracle: closed forms, invariants, exact transport bounds.

None of these compare the oracle with a retyped copy of itself.  Each checks a
fact that the mathematics of Sinkhorn / optimal transport fixes independently
of how Algorithm 1 is coded: closed forms for degenerate shapes, the exact
column marginal after the final v update, the EMD lower / entropic upper
bound (Section II-A, after Cuturi), the cross-ratio characterisation of the
2 x 2 entropic optimum, the 1-D Wasserstein closed form, scale and permutation
invariance, symmetry at convergence, and agreement of the full-vocabulary and
support-restricted forms.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle import emd

RNG = np.random.default_rng(12345)


def rand_problem(rng, V=40, d=6, vr=3, nk=4):
    E = rng.standard_normal((V, d)) / math.sqrt(d)
    q = rng.choice(V, size=vr, replace=False)
    qw = rng.integers(1, 4, size=vr).astype(float)
    dw_ids = rng.choice(V, size=nk, replace=False)
    dw = rng.integers(1, 4, size=nk).astype(float)
    return E, q, qw, dw_ids, dw


def one_doc(E, q, qw, ids, w, lam, iters):
    ptr = np.array([0, len(ids)])
    return oracle.wmd_dense_corpus(E, ptr, ids, w, q, qw, lam, iters)[0]


def entropy(p):
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())


# --- cost matrix -----------------------------------------------------------------

def test_cost_matches_scipy_cdist_and_zero_self_distance():
    E = RNG.standard_normal((300, 17))
    sel = np.array([3, 99, 250])
    M = oracle.cost_rows(E, sel)
    np.testing.assert_allclose(M, cdist(E[sel], E), rtol=1e-13, atol=1e-14)
    assert all(M[i, s] == 0.0 for i, s in enumerate(sel))


def test_select_query_merges_duplicates_and_drops_zeros():
    sel, r = oracle.select_query(10, [7, 2, 7, 5], [1.0, 2.0, 3.0, 0.0])
    assert list(sel) == [2, 7]
    np.testing.assert_allclose(r, [2 / 6, 4 / 6], rtol=0, atol=1e-16)
    with pytest.raises(ValueError):
        oracle.select_query(10, [3], [0.0])
    with pytest.raises(ValueError):
        oracle.select_query(10, [10], [1.0])


# --- closed forms ----------------------------------------------------------------

@pytest.mark.parametrize("lam", [0.5, 10.0, 60.0])
@pytest.mark.parametrize("iters", [0, 1, 15])
def test_single_query_word_closed_form(lam, iters):
    """v_r = 1: every plan must send all mass from the one query word, so the
    distance is sum_j c_j M(q, j) for any lambda and any iteration count."""
    E, q, qw, ids, w = rand_problem(RNG, vr=1, nk=6)
    # the query word repeated with two weights must merge into one word
    got = one_doc(E, [q[0], q[0]], [1.0, 2.0], ids, w, lam, iters)
    c = w / w.sum()
    want = float((c * cdist(E[q[:1]], E[ids])[0]).sum())
    assert abs(got - want) <= 1e-13 * want


@pytest.mark.parametrize("lam", [1.0, 10.0, 80.0])
def test_single_word_document_closed_form(lam):
    """A one-word document receives everything: d = sum_i r_i M(i, j) once at
    least one iteration has set u (with zero iterations it does not hold)."""
    E, q, qw, ids, _ = rand_problem(RNG, vr=5, nk=1)
    r = qw / qw.sum()
    want = float((r * cdist(E[q], E[ids])[:, 0]).sum())
    for iters in (1, 2, 15):
        got = one_doc(E, q, qw, ids, [3.0], lam, iters)
        assert abs(got - want) <= 1e-12 * want
    got0 = one_doc(E, q, qw, ids, [3.0], lam, 0)
    assert abs(got0 - want) > 1e-6 * want


@pytest.mark.parametrize("s", [0.5, 2.0])
def test_equidistant_embeddings(s):
    """E = s I: distinct words are s*sqrt(2) apart, so a query and a document
    with no common word are s*sqrt(2) apart for any plan of total mass 1."""
    V = 12
    E = s * np.eye(V)
    got = one_doc(E, [0, 1, 2], [1, 2, 3], [5, 6, 7, 8], [4, 1, 1, 2], 3.0, 7)
    assert abs(got - s * math.sqrt(2)) <= 1e-14


def test_two_by_two_entropic_closed_form():
    """For a 2 x 2 problem the entropic optimum P = diag(u) K diag(v) is fixed
    by the marginals and the cross ratio P11 P22 / (P12 P21) = K11 K22 / (K12 K21);
    with P11 = a this is a quadratic in a.  The converged oracle must match it."""
    E, q, qw, ids, w = rand_problem(RNG, vr=2, nk=2)
    qw = np.array([1.0, 3.0])
    w = np.array([2.0, 1.0])
    r, c = qw / qw.sum(), w / w.sum()
    lam = 4.0
    order = np.argsort(q)  # the oracle keeps query words in vocabulary order
    q, r = q[order], r[order]
    M = cdist(E[q], E[ids])
    K = np.exp(-lam * M)
    kappa = K[0, 0] * K[1, 1] / (K[0, 1] * K[1, 0])
    r1, r2, c1 = r[0], r[1], c[0]
    A = 1 - kappa
    Bq = r2 - c1 + kappa * (r1 + c1)
    C = -kappa * r1 * c1
    lo, hi = max(0.0, c1 - r2), min(r1, c1)
    roots = [(-Bq + sgn * math.sqrt(Bq * Bq - 4 * A * C)) / (2 * A) for sgn in (1, -1)]
    a = [x for x in roots if lo - 1e-15 <= x <= hi + 1e-15][0]
    P = np.array([[a, r1 - a], [c1 - a, r2 - c1 + a]])
    want = float((P * M).sum())
    got = one_doc(E, q, r, ids, c, lam, 3000)
    assert abs(got - want) <= 1e-11 * want


def test_one_dimensional_wasserstein():
    """d = 1: the exact transport cost is the integral of |F_r - F_c|.  At large
    lambda and convergence the Sinkhorn value lies in [W1, W1 + min(H)/lambda]."""
    rng = np.random.default_rng(7)
    V = 30
    E = rng.uniform(0, 1, size=(V, 1))
    q = np.array([2, 9, 17, 25])
    qw = np.array([1.0, 2.0, 1.0, 3.0])
    ids = np.array([1, 4, 12, 20, 28])
    w = np.array([2.0, 1.0, 1.0, 1.0, 2.0])
    r, c = qw / qw.sum(), w / w.sum()
    pts = np.concatenate([E[q, 0], E[ids, 0]])
    mass = np.concatenate([r, -c])
    order = np.argsort(pts)
    F = np.cumsum(mass[order])[:-1]
    W1 = float(np.sum(np.abs(F) * np.diff(pts[order])))
    lam = 150.0
    got = one_doc(E, q, qw, ids, w, lam, 20000)
    assert W1 - 1e-9 <= got <= W1 + min(entropy(r), entropy(c)) / lam


# --- marginals ---------------------------------------------------------------------

def test_column_marginal_exact_and_row_marginal_converges():
    E, q, qw, ids, w = rand_problem(RNG, V=60, d=5, vr=4, nk=6)
    sel, r = oracle.select_query(E.shape[0], q, qw)
    M = cdist(E[sel], E[ids])
    c = (w / w.sum())[:, None]
    errs = []
    for iters in (1, 5, 15, 60, 400):
        u, v, K = oracle.sinkhorn_scalings(r, M, c, 6.0, iters)
        P = oracle.transport_plan(u[:, 0], v[:, 0], K)
        np.testing.assert_allclose(P.sum(axis=0), c[:, 0], rtol=1e-13, atol=0)
        errs.append(np.abs(P.sum(axis=1) - r).sum())
    assert all(b <= a * 1.0000001 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10 and errs[0] > 1e-4


# --- exact transport bounds -----------------------------------------------------------

def test_lp_solver_matches_vertex_enumeration():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n, m = 3, 4
        r = rng.uniform(0.1, 1, n)
        r /= r.sum()
        c = rng.uniform(0.1, 1, m)
        c /= c.sum()
        M = rng.uniform(0, 2, (n, m))
        assert abs(emd.emd_linprog(r, c, M) - emd.emd_vertices(r, c, M)) < 1e-9


@pytest.mark.parametrize("lam", [5.0, 20.0, 80.0])
def test_emd_bracket(lam):
    """EMD <= d_lambda <= EMD + min(H(r), H(c)) / lambda at convergence, and the
    gap shrinks as lambda grows (Sinkhorn distance -> EMD)."""
    rng = np.random.default_rng(11)
    E, q, qw, ids, w = rand_problem(rng, V=50, d=4, vr=3, nk=4)
    sel, r = oracle.select_query(E.shape[0], q, qw)
    c = w / w.sum()
    M = cdist(E[sel], E[ids])
    exact = emd.emd_vertices(r, c, M)
    got = one_doc(E, q, qw, ids, w, lam, 30000)
    assert exact - 1e-10 <= got <= exact + min(entropy(r), entropy(c)) / lam + 1e-10


def test_gap_to_emd_decreases_with_lambda():
    rng = np.random.default_rng(5)
    E, q, qw, ids, w = rand_problem(rng, V=50, d=4, vr=3, nk=3)
    sel, r = oracle.select_query(E.shape[0], q, qw)
    exact = emd.emd_linprog(r, w / w.sum(), cdist(E[sel], E[ids]))
    gaps = [one_doc(E, q, qw, ids, w, lam, 20000) - exact for lam in (2.0, 8.0, 32.0)]
    assert gaps[0] > gaps[1] > gaps[2] >= -1e-10


def test_identical_documents_near_zero():
    rng = np.random.default_rng(9)
    E = rng.standard_normal((100, 16)) / 4.0
    ids = np.array([4, 8, 15, 16, 23, 42])
    w = np.array([1.0, 2.0, 1.0, 3.0, 1.0, 1.0])
    r = w / w.sum()
    vals = [one_doc(E, ids, w, ids, w, lam, 5000) for lam in (5.0, 20.0, 80.0)]
    assert vals[0] > vals[1] > vals[2] > 0
    for lam, val in zip((5.0, 20.0, 80.0), vals):
        assert val <= entropy(r) / lam


def test_symmetry_at_convergence():
    E, q, qw, ids, w = rand_problem(RNG, V=40, d=5, vr=4, nk=5)
    a = one_doc(E, q, qw, ids, w, 5.0, 20000)
    b = one_doc(E, ids, w, q, qw, 5.0, 20000)
    assert abs(a - b) <= 1e-10 * a


def test_plan_cost_is_convex_combination_of_costs():
    E, q, qw, ids, w = rand_problem(RNG, V=40, d=5, vr=4, nk=5)
    M = cdist(E[np.unique(q)], E[ids])
    for iters in (0, 1, 3, 15):
        got = one_doc(E, q, qw, ids, w, 10.0, iters)
        assert M.min() <= got <= M.max()


# --- invariances and the two formulations -----------------------------------------

def small_corpus(rng, V=300, d=12, N=40, lo=3, hi=15):
    E = rng.standard_normal((V, d)) / math.sqrt(d)
    lens = rng.integers(lo, hi + 1, size=N)
    ptr = np.concatenate([[0], np.cumsum(lens)])
    ids = np.concatenate([rng.choice(V, size=n, replace=False) for n in lens])
    w = rng.integers(1, 5, size=len(ids)).astype(float)
    q = rng.choice(V, size=7, replace=False)
    qw = rng.integers(1, 5, size=7).astype(float)
    return E, ptr, ids, w, q, qw


def test_dense_equals_support_restricted():
    rng = np.random.default_rng(21)
    E, ptr, ids, w, q, qw = small_corpus(rng)
    a = oracle.wmd_dense_corpus(E, ptr, ids, w, q, qw, 10.0, 15, block=16)
    b = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 15)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_scale_invariance():
    rng = np.random.default_rng(22)
    E, ptr, ids, w, q, qw = small_corpus(rng, N=10)
    s = 3.0
    a = oracle.wmd_dense_corpus(E, ptr, ids, w, q, qw, 10.0, 15)
    b = oracle.wmd_dense_corpus(s * E, ptr, ids, w, q, qw, 10.0 / s, 15)
    np.testing.assert_allclose(b, s * a, rtol=1e-13)


def test_permutation_invariance():
    rng = np.random.default_rng(23)
    E, ptr, ids, w, q, qw = small_corpus(rng, N=12)
    base = oracle.wmd_dense_corpus(E, ptr, ids, w, q, qw, 10.0, 15)
    # relabel the vocabulary
    perm = rng.permutation(E.shape[0])
    inv = np.argsort(perm)
    E2 = E[perm]
    a = oracle.wmd_dense_corpus(E2, ptr, inv[ids], w, inv[q], qw, 10.0, 15)
    np.testing.assert_allclose(a, base, rtol=1e-12)
    # reverse the query word order and the documents
    N = len(ptr) - 1
    order = np.arange(N)[::-1]
    lens = np.diff(ptr)[order]
    ptr2 = np.concatenate([[0], np.cumsum(lens)])
    ids2 = np.concatenate([ids[ptr[k]:ptr[k + 1]] for k in order])
    w2 = np.concatenate([w[ptr[k]:ptr[k + 1]] for k in order])
    b = oracle.wmd_dense_corpus(E, ptr2, ids2, w2, q[::-1], qw[::-1], 10.0, 15)
    np.testing.assert_allclose(b, base[order], rtol=1e-12)


def test_duplicate_document_words_merge():
    rng = np.random.default_rng(24)
    E, ptr, ids, w, q, qw = small_corpus(rng, N=2)
    a = oracle.wmd_dense_corpus(E, [0, 3], [5, 9, 5], [1.0, 2.0, 3.0], q, qw, 10.0, 15)
    b = oracle.wmd_dense_corpus(E, [0, 2], [5, 9], [4.0, 2.0], q, qw, 10.0, 15)
    np.testing.assert_allclose(a, b, rtol=1e-13)


def test_empty_and_zero_weight_documents_are_nan():
    rng = np.random.default_rng(25)
    E, ptr, ids, w, q, qw = small_corpus(rng, N=2)
    ptr3 = [0, 2, 2, 4]
    ids3 = [1, 2, 3, 4]
    w3 = [1.0, 1.0, 0.0, 0.0]
    a = oracle.wmd_dense_corpus(E, ptr3, ids3, w3, q, qw, 10.0, 15)
    b = oracle.sinkhorn_wmd_support(E, ptr3, ids3, w3, q, qw, 10.0, 15)
    assert np.isfinite(a[0]) and np.isnan(a[1]) and np.isnan(a[2])
    assert np.isfinite(b[0]) and np.isnan(b[1]) and np.isnan(b[2])


# --- finite iteration counts ----------------------------------------------------------

def _finite_iter_case(seed):
    rng = np.random.default_rng(seed)
    E, q, qw, ids, w = rand_problem(rng, V=60, d=5, vr=4, nk=5)
    sel, r = oracle.select_query(E.shape[0], q, qw)
    c = w / w.sum()
    M = cdist(E[sel], E[ids])
    return E, q, qw, ids, w, r, c, M


@pytest.mark.parametrize("seed", [31, 32])
def test_zero_iterations_closed_form(seed):
    """With no iteration u is constant, so v_j = c_j / sum_i K_ij and the
    distance is the K-weighted mean cost of each document word:
    d = sum_j c_j (sum_i K_ij M_ij) / (sum_i K_ij)."""
    E, q, qw, ids, w, r, c, M = _finite_iter_case(seed)
    lam = 7.0
    K = np.exp(-lam * M)
    want = float((c * (K * M).sum(axis=0) / K.sum(axis=0)).sum())
    assert abs(one_doc(E, q, qw, ids, w, lam, 0) - want) <= 1e-13 * want


@pytest.mark.parametrize("seed", [33, 34])
def test_one_iteration_closed_form(seed):
    """From the uniform start the first v is proportional to c_j / sum_i K_ij,
    so one iteration gives u proportional to r / (K (c / colsum(K))); the final
    update then gives v_j = c_j / (K^T u)_j and the distance is
    sum_ij u_i K_ij M_ij v_j (the scale of u cancels)."""
    E, q, qw, ids, w, r, c, M = _finite_iter_case(seed)
    lam = 7.0
    K = np.exp(-lam * M)
    u = r / (K @ (c / K.sum(axis=0)))
    v = c / (K.T @ u)
    want = float((u[:, None] * K * M * v[None, :]).sum())
    assert abs(one_doc(E, q, qw, ids, w, lam, 1) - want) <= 1e-13 * want


# --- the stop once x settles ---------------------------------------------------------------

def test_tolerance_stop_consistency():
    """tol = 0 runs every iteration; a huge tol stops after one; the count
    grows as tol shrinks, the stopping iteration is the first whose change of
    x is within tol, and the distance approaches the long-run value."""
    rng = np.random.default_rng(51)
    E, ptr, ids, w, q, qw = small_corpus(rng, N=6)
    fixed15 = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 15)
    a, it_a = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 15, tol=0.0)
    np.testing.assert_allclose(a, fixed15, rtol=1e-14)
    assert np.all(it_a == 15)
    one = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 1)
    b, it_b = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 15, tol=1e30)
    np.testing.assert_allclose(b, one, rtol=1e-14)
    assert np.all(it_b == 1)
    long_run = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 4000)
    prev = np.zeros(len(ptr) - 1)
    for tol in (1e-2, 1e-4, 1e-6, 1e-9):
        d, its = oracle.sinkhorn_wmd_support(E, ptr, ids, w, q, qw, 10.0, 4000, tol=tol)
        assert np.all(its >= prev)
        prev = its
        # the count is the first iteration whose relative change of x is within tol
        sel, r = oracle.select_query(E.shape[0], q, qw)
        for k in range(len(ptr) - 1):
            cw = w[ptr[k]:ptr[k + 1]] / w[ptr[k]:ptr[k + 1]].sum()
            Md = cdist(E[sel], E[ids[ptr[k]:ptr[k + 1]]])
            K = np.exp(-10.0 * Md)
            x = np.ones(len(r)) / len(r)
            first = None
            for it in range(1, 4001):
                xn = (K @ (cw / (K.T @ (1.0 / x)))) / r
                if np.max(np.abs(xn - x) / xn) <= tol:
                    first = it
                    break
                x = xn
            assert first == its[k]
    np.testing.assert_allclose(d, long_run, rtol=1e-7)
