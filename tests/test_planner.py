"""Step 1 (Theorem 3 and Lemma 1): the bound functions against exact binomial sums, the
visiting probability the bound promises against a direct computation and a simulation of
the oracle's own sampling."""
import math

import numpy as np
import pytest
from scipy.stats import binom

import synth
from oracle import rng, rsm
from paper_1411_0814_amd import planner


@pytest.mark.parametrize("n", [1, 5, 12, 40, 300, 2000])
@pytest.mark.parametrize("rho", [0.002, 0.05, 0.3, 0.5, 0.9])
def test_lemma1_brackets_the_binomial_distribution_function(n, rho):
    # C(k) <= P(X <= k) <= C(k + 1) for X ~ B(n, rho), equality only at the ends
    for k in range(0, n):
        cdf = binom.cdf(k, n, rho)
        assert planner.lemma1_C(n, rho, k) <= cdf * (1 + 1e-12) + 1e-300
        assert cdf <= planner.lemma1_C(n, rho, k + 1) * (1 + 1e-12) + 1e-300
    assert planner.lemma1_C(n, rho, 0) == pytest.approx(binom.pmf(0, n, rho), rel=1e-12)
    assert planner.lemma1_C(n, rho, n) == pytest.approx(1 - rho ** n, rel=1e-12)


def test_lemma1_increasing_in_k():
    for n, rho in [(50, 0.1), (1000, 0.01), (200, 0.7)]:
        c = [planner.lemma1_C(n, rho, k) for k in range(n + 1)]
        assert all(a <= b for a, b in zip(c, c[1:]))


def _visit_probability_exact(m, n, rho, r, k):
    """P(a known entry is visited in one row-first trial) from the sum in the proof of
    Theorem 3, evaluated exactly: sum_{i > r} B(i; n, rho^k) k i / (m n rho)."""
    p = rho ** k
    i = np.arange(r + 1, n + 1)
    return float(np.sum(binom.pmf(i, n, p) * k * i / (m * n * rho)))


@pytest.mark.parametrize("m,n,rho,r,k", [(1000, 200, 0.5, 3, 4), (65536, 1024, 0.2, 3, 4),
                                         (4000, 64, 0.9, 8, 9), (500, 900, 0.35, 2, 3)])
def test_bound_dominates_the_exact_requirement(m, n, rho, r, k):
    eps = 0.95
    exact = math.log(1 / (1 - eps)) / _visit_probability_exact(m, n, rho, r, k)
    bound = planner.trials_bound_rows_first(m, n, rho, r, k, eps)
    assert bound >= exact * (1 - 1e-12)
    # the bound is ln(1/(1-eps)) times a constant, and proportional to m
    b999 = planner.trials_bound_rows_first(m, n, rho, r, k, 0.999)
    assert b999 / bound == pytest.approx(math.log(1000) / math.log(20), rel=1e-12)
    assert planner.trials_bound_rows_first(2 * m, n, rho, r, k, eps) == \
        pytest.approx(2 * bound, rel=1e-12)


def test_column_first_is_row_first_of_the_transpose():
    assert planner.trials_bound(5000, 300, 0.6, 4, 5, 0.9) == \
        planner.trials_bound_rows_first(300, 5000, 0.6, 4, 5, 0.9)
    assert planner.plan_trials(5000, 300, 0.6, 4) == \
        math.ceil(planner.trials_bound(5000, 300, 0.6, 4, 5, 0.99))


def test_planned_trials_visit_every_known_entry_with_the_promised_probability():
    # a tiny column-first problem: after plan_trials(eps) trials drawn by the oracle's own
    # generator, the fraction of known entries visited is at least eps (up to sampling)
    m, n, r, rho, eps = 60, 12, 2, 0.7, 0.9
    p = synth.paper_synthetic(m, n, r, rho, 0.0, 3)
    W = np.asarray(p.W, dtype=bool)
    I = planner.plan_trials(m, n, rho, r, eps=eps)
    visited_fraction = []
    for seed in range(12):
        subsets = rng.draw_subsets(seed, n, r + 1, I)
        seen = np.zeros_like(W)
        for cols in subsets:
            R = rsm.qualifying_rows(W, cols)
            if R.size > r:   # the proof of Theorem 3 counts sub-matrices of > r rows
                seen[np.ix_(R, cols)] = True
        visited_fraction.append(seen[W].mean())
    assert np.mean(visited_fraction) >= eps


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        planner.trials_bound_rows_first(100, 50, 0.5, 3, 3, 0.9)   # k must exceed r
    with pytest.raises(ValueError):
        planner.trials_bound(100, 50, 0.5, 3, 4, 1.0)
    with pytest.raises(ValueError):
        planner.lemma1_C(10, 0.0, 3)


def test_planner_is_the_library_entry_point():
    # the Python names are thin calls of the C ABI: the same numbers come back from ctypes
    import ctypes as C
    from paper_1411_0814_amd import _lib
    out = C.c_double()
    assert _lib.lib().rsm_trials_bound(5000, 300, 0.6, 4, 0, 0.9, 0, C.byref(out)) == _lib.OK
    assert out.value == planner.trials_bound(5000, 300, 0.6, 4, None, 0.9)
    cnt = C.c_int64()
    assert _lib.lib().rsm_plan_trials(5000, 300, 0.6, 4, 5, 0.9, 1, C.byref(cnt)) == _lib.OK
    assert cnt.value == math.ceil(planner.trials_bound_rows_first(5000, 300, 0.6, 4, 5, 0.9))
    assert planner.plan_trials(5000, 300, 0.6, 4, 5, 0.9, rows_first=True) == cnt.value
    # NULL output pointers are rejected
    assert _lib.lib().rsm_lemma1_c(10, 0.5, 3, None) == _lib.E_ARG


def test_hopeless_density_has_no_plan():
    # rho^l so small that no trial keeps more than r rows: the bound is infinite and no
    # trial count is planned
    assert planner.trials_bound(100, 50, 0.01, 3, 4, 0.9) == math.inf
    with pytest.raises(ValueError):
        planner.plan_trials(100, 50, 0.01, 3, 4, 0.9)
