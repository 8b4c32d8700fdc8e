"""Pins of the oracle's rows-first sampling (method M2, Section III) against what the paper
and the mathematics fix: the qualifying columns by brute force, the trace of N, exact
recovery on noise-free data, the full-mask case that reduces to the truncated SVD, and a
brute-force sum over every row subset of a tiny matrix computed with a different routine.
Planted mistakes (on the CPU) show that each pin catches something."""
import itertools

import numpy as np
import pytest

import synth
from oracle import metrics, rsm


def test_qualifying_cols_brute_force():
    g = np.random.default_rng(21)
    W = g.random((12, 70)) < 0.6
    rows = np.array([0, 5, 9])
    brute = [j for j in range(70) if all(W[i, j] for i in rows)]
    assert list(rsm.qualifying_cols(W, rows)) == brute


def test_trace_counts_the_vectors_of_every_trial():
    # each accepted trial adds |C_t| - r orthonormal vectors: trace(N) = sum (|C_t| - r)
    p = synth.paper_synthetic(300, 60, 3, 0.75, 0.05, 22)
    res = rsm.rsm(p.Y, p.W, 3, 400, seed=4, rows_first=True, with_U=False)
    acc = res.rows >= 4
    assert res.accepted == int(acc.sum()) > 0
    assert abs(np.trace(res.N) - float(np.sum(res.rows[acc] - 3))) < 1e-9
    assert np.linalg.eigvalsh(res.N).min() > -1e-11
    # |C_t| by brute force, on the oracle's own subsets (row subsets of [0, m))
    assert res.subsets.shape == (400, 4) and res.subsets.max() < 300
    for t in range(0, 400, 41):
        assert res.rows[t] == p.W[res.subsets[t], :].all(axis=0).sum()


@pytest.mark.parametrize("m,n,r,rho,trials", [(400, 80, 3, 0.8, 600), (200, 150, 5, 0.85, 500)])
def test_exact_recovery_noise_free(m, n, r, rho, trials):
    # Z = U_S V_C^T has rank r, so its right singular vectors past the r largest span the
    # null space of V_C^T: every constraint is exact and V-hat spans the true V.
    p = synth.paper_synthetic(m, n, r, rho, 0.0, 23)
    res = rsm.rsm(p.Y, p.W, r, trials, seed=6, rows_first=True)
    assert res.uncovered == 0
    assert metrics.principal_angle_max(res.V, p.Vbar) < 1e-10
    Vb, _ = np.linalg.qr(p.Vbar)
    assert np.linalg.norm(res.N @ Vb) <= 1e-12 * np.linalg.norm(res.N)
    assert res.eigvals[r - 1] < 1e-12 * res.eigvals[r]


def test_full_mask_all_rows_is_truncated_svd():
    # rho = 1 and k = m: every trial is the whole matrix and contributes I - V_r V_r^T, so
    # N = I (I - V_r V_r^T) and V-hat is the top-r right singular space of Y whatever the
    # noise (Eckart-Young); U-hat V-hat^T is the rank-r truncated SVD.
    g = np.random.default_rng(24)
    m, n, r = 9, 20, 3
    Y = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 0.3 * g.standard_normal((m, n))
    W = np.ones((m, n), dtype=bool)
    res = rsm.rsm(Y, W, r, 4, seed=1, l=m, rows_first=True)
    u, s, vt = np.linalg.svd(Y)
    assert np.abs(res.N - 4 * (np.eye(n) - vt[:r].T @ vt[:r])).max() < 1e-11
    assert metrics.principal_angle_max(res.V, vt[:r].T) < 1e-12
    trunc = (u[:, :r] * s[:r]) @ vt[:r]
    assert np.abs(res.U @ res.V.T - trunc).max() < 1e-10


def test_N_brute_force_all_row_subsets_tiny():
    # m = 7, k = 3: every C(7,3) row subset; N is the sum over subsets with more than r
    # qualifying columns of the projector on the |C| - r smallest eigenvectors of Z^T Z
    # (eigh instead of the SVD), in any order.
    p = synth.paper_synthetic(7, 40, 2, 0.8, 0.05, 25)
    subsets = np.array(list(itertools.combinations(range(7), 3)))
    res = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=subsets, rows_first=True,
                  with_U=False)
    N_ref = np.zeros((40, 40))
    for rows in subsets[::-1]:
        C = [j for j in range(40) if p.W[rows, j].all()]
        if len(C) <= 2:
            continue
        Z = p.Y[np.ix_(rows, C)]
        lam, E = np.linalg.eigh(Z.T @ Z)
        Xi = np.zeros((40, len(C) - 2))
        Xi[C] = E[:, :len(C) - 2]
        N_ref += Xi @ Xi.T
    assert np.abs(res.N - N_ref).max() < 1e-10
    shuffled = subsets[np.random.default_rng(1).permutation(len(subsets))]
    res2 = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=shuffled, rows_first=True,
                   with_U=False)
    assert np.abs(res2.N - res.N).max() < 1e-12


def test_rejects_invalid_arguments():
    p = synth.paper_synthetic(50, 30, 3, 0.8, 0.0, 26)
    with pytest.raises(ValueError):
        rsm.rsm(p.Y, p.W, 3, 10, seed=0, rows_first=True, nvec=1)
    with pytest.raises(ValueError):
        rsm.rsm(p.Y, p.W, 3, 10, seed=0, rows_first=True, min_rows=3)
    with pytest.raises(ValueError):
        rsm.rsm(p.Y, p.W, 3, 10, seed=0, rows_first=True, l=3)


# ------------------------------------------------------------------ planted mistakes

_orig_cols = rsm.qualifying_cols
_orig_constraints = rsm.trial_constraints_rows_first


def _cols_any_known(W, rows):
    # mistake: columns with ANY chosen entry known
    return np.flatnonzero(np.asarray(W[rows, :], dtype=bool).any(axis=0))


def _null_vectors_only(Y, W, rows, r, min_cols):
    # mistake: only the |C| - k null vectors (drops the k - r smallest nonzero ones)
    C = _orig_cols(W, rows)
    if C.size < min_cols:
        return C, None
    Z = np.asarray(Y[np.ix_(rows, C)], dtype=np.float64)
    nv = C.size - len(rows)
    if nv < 1:
        return C, None
    return C, rsm.minor_right_singular_vectors(Z, nv)


def _largest_vectors(Y, W, rows, r, min_cols):
    # mistake: the |C| - r LARGEST right singular vectors
    C = _orig_cols(W, rows)
    if C.size < min_cols:
        return C, None
    Z = np.asarray(Y[np.ix_(rows, C)], dtype=np.float64)
    _, _, vt = np.linalg.svd(Z, full_matrices=True)
    return C, vt[:C.size - r].T.copy()


def _fails(fn) -> bool:
    try:
        fn()
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("attr,bad,pins", [
    ("qualifying_cols", _cols_any_known, [test_qualifying_cols_brute_force]),
    ("trial_constraints_rows_first", _null_vectors_only,
     [test_trace_counts_the_vectors_of_every_trial, test_N_brute_force_all_row_subsets_tiny]),
    ("trial_constraints_rows_first", _largest_vectors,
     [lambda: test_exact_recovery_noise_free(400, 80, 3, 0.8, 600),
      test_full_mask_all_rows_is_truncated_svd]),
])
def test_planted_mistake_is_caught(monkeypatch, attr, bad, pins):
    monkeypatch.setattr(rsm, attr, bad)
    assert all(_fails(pin) for pin in pins), attr
