"""Planted mistakes in the oracle must trip at least one pin.

Each mutant below is a plausible slip in coding Algorithm 1 (a dropped 1/r, a
missing reciprocal, a flipped exponent, a skipped final update, a squared
cost, a non-uniform start).  The mutant replaces the oracle's function for the
duration of the test, on the CPU; the pins of ``test_oracle_pins`` are then run
against it and at least one must fail.
"""
import numpy as np
import pytest

import oracle
import oracle.wmd as ow
import test_oracle_pins as pins

PIN_CASES = [
    (pins.test_single_query_word_closed_form, dict(lam=10.0, iters=15)),
    (pins.test_single_word_document_closed_form, dict(lam=10.0)),
    (pins.test_two_by_two_entropic_closed_form, {}),
    (pins.test_column_marginal_exact_and_row_marginal_converges, {}),
    (pins.test_emd_bracket, dict(lam=20.0)),
    (pins.test_one_dimensional_wasserstein, {}),
    (pins.test_zero_iterations_closed_form, dict(seed=31)),
    (pins.test_one_iteration_closed_form, dict(seed=33)),
    (pins.test_plan_cost_is_convex_combination_of_costs, {}),
]


def make_scalings(drop_inv_r=False, no_recip=False, flip_sign=False, skip_final=False,
                  start_r=False):
    def scalings(r, M, c, lam, max_iter):
        r = np.asarray(r, float)
        M = np.asarray(M, float)
        c = np.asarray(c, float)
        K = np.exp((lam if flip_sign else -lam) * M)
        v_r = r.shape[0]
        if start_r:
            x = np.repeat(r[:, None], c.shape[1], axis=1)
        else:
            x = np.ones((v_r, c.shape[1])) / v_r
        mask = c > 0
        with np.errstate(all="ignore"):
            u = 1.0 / x
            for _ in range(max_iter):
                u = x if no_recip else 1.0 / x
                v = np.where(mask, c / (K.T @ u), 0.0)
                x = (K @ v) if drop_inv_r else (1.0 / r)[:, None] * (K @ v)
            if not skip_final:
                u = x if no_recip else 1.0 / x
                v = np.where(mask, c / (K.T @ u), 0.0)
        return u, v, K
    return scalings


def squared_cost(E, sel):
    E = np.asarray(E, float)
    return np.stack([((E - E[q]) ** 2).sum(axis=1) for q in np.asarray(sel)])


MUTANTS = {
    "dropped_inverse_r": dict(scalings=make_scalings(drop_inv_r=True)),
    "missing_reciprocal": dict(scalings=make_scalings(no_recip=True)),
    "flipped_exponent": dict(scalings=make_scalings(flip_sign=True)),
    "skipped_final_update": dict(scalings=make_scalings(skip_final=True)),
    "non_uniform_start": dict(scalings=make_scalings(start_r=True)),
    "squared_cost": dict(cost=squared_cost),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    m = MUTANTS[name]
    if "scalings" in m:
        monkeypatch.setattr(ow, "sinkhorn_scalings", m["scalings"])
        monkeypatch.setattr(oracle, "sinkhorn_scalings", m["scalings"])
    if "cost" in m:
        monkeypatch.setattr(ow, "cost_rows", m["cost"])
    failed = []
    for fn, kw in PIN_CASES:
        try:
            fn(**kw)
        except Exception:  # an assertion or a crash both expose the mutant
            failed.append(fn.__name__)
    assert failed, f"mutant {name} passed every pin"


def test_unmutated_oracle_passes_the_same_pins():
    for fn, kw in PIN_CASES:
        fn(**kw)
