"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (largest instead of smallest
singular vector, a wrong embedding index, eigenvectors of the largest eigenvalues, a
transposed operand in the U solve, a dropped mask) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import metrics, rsm


def _noise_free(m, n, r, rho, seed):
    return synth.paper_synthetic(m, n, r, rho, 0.0, seed)


# ------------------------------------------------------------------ step 2 pieces

def test_qualifying_rows_brute_force():
    g = np.random.default_rng(1)
    W = g.random((60, 9)) < 0.6
    cols = np.array([1, 4, 7])
    brute = [i for i in range(60) if all(W[i, c] for c in cols)]
    assert list(rsm.qualifying_rows(W, cols)) == brute


def test_minor_vector_is_null_on_true_rows_noise_free():
    # eq.(constrain.barV): the minor right singular vector of a sub-matrix of the noise-free
    # rank-r matrix is orthogonal to the rows of V-bar at the chosen columns.
    p = _noise_free(300, 40, 4, 0.7, 2)
    cols = np.array([0, 3, 9, 21, 33])
    R = rsm.qualifying_rows(p.W, cols)
    z = rsm.minor_right_singular_vectors(p.Y[np.ix_(R, cols)], 1)
    assert z.shape == (5, 1)
    assert abs(np.linalg.norm(z) - 1.0) < 1e-14
    Vb = p.Vbar / np.linalg.norm(p.Vbar, axis=0)
    assert np.linalg.norm(Vb[cols].T @ z) < 1e-12
    # the largest singular vector is certainly not null there
    _, _, vt = np.linalg.svd(p.Y[np.ix_(R, cols)])
    assert np.linalg.norm(Vb[cols].T @ vt[0]) > 1e-3


def test_minor_vector_projector_matches_gram_eigh_noisy():
    g = np.random.default_rng(3)
    Z = g.standard_normal((50, 6)) @ np.diag([5, 4, 3, 2, 1, 0.1])
    z = rsm.minor_right_singular_vectors(Z, 2)
    lam, E = np.linalg.eigh(Z.T @ Z)
    P1 = z @ z.T
    P2 = E[:, :2] @ E[:, :2].T
    assert np.abs(P1 - P2).max() < 1e-12


def test_minor_vector_rows_fewer_than_columns():
    # r rows, r+1 columns: the one-dimensional null space is the minor vector.
    g = np.random.default_rng(4)
    Z = g.standard_normal((3, 4))
    z = rsm.minor_right_singular_vectors(Z, 1)
    assert np.linalg.norm(Z @ z) < 1e-14


def test_embedding():
    xi = rsm.embed(np.array([[1.0], [2.0], [3.0]]), np.array([0, 5, 7]), 9)
    assert xi.shape == (9, 1)
    assert list(xi[:, 0]) == [1, 0, 0, 0, 0, 2, 0, 3, 0]


# ------------------------------------------------------------------ accumulator N

def test_N_invariants_noisy():
    p = synth.paper_synthetic(400, 30, 3, 0.8, 0.05, 5, num_submatrices=300)
    res = rsm.rsm(p.Y, p.W, 3, 300, seed=9, with_U=False)
    N = res.N
    assert np.array_equal(N, N.T) or np.abs(N - N.T).max() < 1e-13
    assert np.linalg.eigvalsh(N).min() > -1e-12
    # each accepted trial adds nvec orthonormal unit vectors: trace(N) = nvec * accepted
    assert abs(np.trace(N) - 1 * res.accepted) < 1e-10
    # N_jj <= number of accepted trials that contain column j
    hits = np.zeros(30)
    for t, cols in enumerate(res.subsets):
        if res.rows[t] >= 3:
            hits[cols] += 1
    assert np.all(np.diag(N) <= hits + 1e-12)
    # rows per trial: brute force
    for t in range(0, 300, 37):
        assert res.rows[t] == p.W[:, res.subsets[t]].all(axis=1).sum()


def test_N_annihilates_true_V_noise_free():
    p = _noise_free(500, 40, 3, 0.8, 6)
    res = rsm.rsm(p.Y, p.W, 3, 800, seed=2, with_U=False)
    Vb, _ = np.linalg.qr(p.Vbar)
    assert np.linalg.norm(res.N @ Vb) <= 1e-12 * np.linalg.norm(res.N)


def test_N_brute_force_all_subsets_tiny():
    # n = 7, l = 3: enumerate every C(7,3) subset; N must be the sum of each sub-matrix's
    # minor projector computed independently (eigh of Z^T Z), in any order.
    p = synth.paper_synthetic(120, 7, 2, 0.85, 0.01, 7)
    subsets = np.array(list(itertools.combinations(range(7), 3)))
    res = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=subsets, with_U=False)
    N_ref = np.zeros((7, 7))
    for cols in subsets[::-1]:
        R = [i for i in range(120) if p.W[i, cols].all()]
        if len(R) < 2:
            continue
        Z = p.Y[np.ix_(R, cols)]
        lam, E = np.linalg.eigh(Z.T @ Z)
        xi = np.zeros(7)
        xi[cols] = E[:, 0]
        N_ref += np.outer(xi, xi)
    assert np.abs(res.N - N_ref).max() < 1e-10
    shuffled = subsets[np.random.default_rng(0).permutation(len(subsets))]
    res2 = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=shuffled, with_U=False)
    assert np.abs(res2.N - res.N).max() < 1e-12


# ------------------------------------------------------------------ V-hat and U-hat

@pytest.mark.parametrize("m,n,r,rho,trials", [(2000, 200, 5, 0.7, 800), (600, 50, 2, 0.6, 600),
                                               (3000, 64, 8, 0.9, 1500)])
def test_exact_recovery_noise_free(m, n, r, rho, trials):
    # Theorem 1 with Psi = 0: the minor subspace of every sub-matrix is exact, so V-hat spans
    # the true row space to rounding (largest principal angle < 1e-10).
    p = _noise_free(m, n, r, rho, 11)
    res = rsm.rsm(p.Y, p.W, r, trials, seed=5, with_e=True)
    assert res.uncovered == 0
    theta = metrics.principal_angle_max(res.V, p.Vbar)
    assert theta < 1e-10, theta
    # and the fit on known entries is exact to rounding
    assert res.e < 1e-10 * np.sqrt(np.mean(p.Y ** 2))
    # eigen-gap: r zero eigenvalues then a clearly positive one
    assert res.eigvals[r - 1] < 1e-12 * res.eigvals[r]


def test_full_mask_l_equals_n_is_truncated_svd():
    # rho = 1 and l = n: every trial is the whole matrix, its l - r minor vectors span the
    # complement of the top-r right singular space, so N = I * (I - V_r V_r^T) and V-hat is
    # the top-r right singular space of Y for any noise (Eckart-Young); U-hat V-hat^T is the
    # rank-r truncated SVD.
    g = np.random.default_rng(12)
    m, n, r = 40, 8, 3
    Y = g.standard_normal((m, r)) @ g.standard_normal((r, n)) + 0.3 * g.standard_normal((m, n))
    W = np.ones((m, n), dtype=bool)
    res = rsm.rsm(Y, W, r, 5, seed=1, l=n)
    u, s, vt = np.linalg.svd(Y)
    assert metrics.principal_angle_max(res.V, vt[:r].T) < 1e-12
    trunc = (u[:, :r] * s[:r]) @ vt[:r]
    assert np.abs(res.U @ res.V.T - trunc).max() < 1e-10
    assert np.abs(res.N - 5 * (np.eye(n) - vt[:r].T @ vt[:r])).max() < 1e-11


def test_U_is_masked_least_squares():
    g = np.random.default_rng(13)
    m, n, r = 200, 30, 4
    Y = g.standard_normal((m, n))
    W = g.random((m, n)) < 0.5
    W[7, :] = False
    W[7, :3] = True              # 3 < r known entries: underdetermined row
    V, _ = np.linalg.qr(g.standard_normal((n, r)))
    U, under = rsm.solve_U(Y, W, V)
    assert under == 1 and np.all(U[7] == 0)
    for i in [0, 1, 50, 199]:
        J = W[i]
        # normal equations solved independently
        A = V[J].T @ V[J]
        b = V[J].T @ Y[i, J]
        assert np.abs(U[i] - np.linalg.solve(A, b)).max() < 1e-10
        # residual orthogonal to the columns of V restricted to the known entries
        res = Y[i, J] - V[J] @ U[i]
        assert np.abs(V[J].T @ res).max() < 1e-10


def test_U_full_mask_closed_form():
    g = np.random.default_rng(14)
    Y = g.standard_normal((50, 12))
    V, _ = np.linalg.qr(g.standard_normal((12, 3)))
    U, under = rsm.solve_U(Y, np.ones((50, 12), bool), V)
    assert under == 0
    assert np.abs(U - Y @ V).max() < 1e-12


def test_error_e_definition():
    g = np.random.default_rng(15)
    Y = g.standard_normal((30, 10))
    W = g.random((30, 10)) < 0.5
    U = g.standard_normal((30, 2))
    V = g.standard_normal((10, 2))
    brute = 0.0
    for i in range(30):
        for j in range(10):
            if W[i, j]:
                brute += (Y[i, j] - U[i] @ V[j]) ** 2
    assert abs(rsm.error_e(Y, W, U, V) - np.sqrt(brute / W.sum())) < 1e-14


def test_principal_angle_forms_agree():
    g = np.random.default_rng(16)
    A = np.linalg.qr(g.standard_normal((50, 4)))[0]
    for eps in [1e-5, 1e-3, 0.1]:
        B = np.linalg.qr(A + eps * g.standard_normal((50, 4)))[0]
        s = metrics.principal_angle_max(A, B)
        c = metrics.principal_angle_max_cos(A, B)
        assert abs(s - c) < 1e-8 + 1e-6 * s
    # and the sine form resolves tiny angles the cosine form cannot
    B = np.linalg.qr(A + 1e-12 * g.standard_normal((50, 4)))[0]
    assert 1e-14 < metrics.principal_angle_max(A, B) < 1e-10


def test_rel_rms_known_brute_force():
    # the parity metric written out entry by entry: only the known entries (w_ij = 1, the
    # W o of eq.(problem)) enter either sum, and the normaliser is the second (reference)
    # product.  The two products differ in scale, so the other normaliser gives another
    # number; half the entries are unknown and carry large differences, so dropping the
    # mask does too.
    g = np.random.default_rng(18)
    m, n, r = 23, 11, 3
    U1, V1 = g.standard_normal((m, r)), g.standard_normal((n, r))
    U2, V2 = 2.5 * g.standard_normal((m, r)), g.standard_normal((n, r))
    W = g.random((m, n)) < 0.5
    num = den = 0.0
    for i in range(m):
        for j in range(n):
            if W[i, j]:
                a = sum(U1[i, k] * V1[j, k] for k in range(r))
                b = sum(U2[i, k] * V2[j, k] for k in range(r))
                num += (a - b) ** 2
                den += b ** 2
    expect = (num / den) ** 0.5
    for block in (5, 8192):  # one row block and several (a ragged last one)
        assert abs(metrics.rel_rms_known(W, U1, V1, U2, V2, block=block) - expect) <= 1e-13 * expect
    # no known entry differs: zero, whatever the unknown entries hold
    U3 = U2.copy()
    U3[~W.any(axis=1)] += 1.0
    Wr = np.zeros_like(W)
    Wr[:, 0] = True
    V3 = V2.copy()
    V3[1:] += 7.0
    assert metrics.rel_rms_known(Wr, U2, V3, U2, V2) == 0.0


def test_rel_rms_basis_invariant():
    g = np.random.default_rng(17)
    U = g.standard_normal((40, 3))
    V = np.linalg.qr(g.standard_normal((9, 3)))[0]
    Q = np.linalg.qr(g.standard_normal((3, 3)))[0]
    W = g.random((40, 9)) < 0.7
    assert metrics.rel_rms_known(W, U @ Q, V @ Q, U, V) < 1e-14


# ------------------------------------------------------------------ the paper's printed numbers

def _table1_rows():
    import csv
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_rsm.csv")
    with open(path) as f:
        return [row for row in csv.DictReader(filter(lambda s: not s.startswith("#"), f))]


def test_golden_table_matches_generator_shapes():
    rows = _table1_rows()
    assert len(rows) == len(synth.TABLE1_ROWS)
    for row, (m, n, rho, sigma) in zip(rows, synth.TABLE1_ROWS):
        assert (int(row["m"]), int(row["n"]), float(row["rho"]), float(row["sigma"])) == (m, n, rho, sigma)


@pytest.mark.slow
def test_table1_error_at_paper_shape():
    # Table I, first row: 65536 x 1024, rho = 0.2, sigma = 0.2, r = 3, l = 4, M1, I in
    # [15n, 35n] (25n here).  The paper prints e = 0.1987 for RSM.  e is an average over
    # ~1.3e7 known entries, so its sampling spread is ~1e-4; allow 1e-3.
    row = _table1_rows()[0]
    p = synth.table1(0)
    res = rsm.rsm(p.Y, p.W, 3, p.num_submatrices, seed=p.seed_rsm, l=4)
    assert abs(res.e - float(row["e_rsm"])) < 1e-3, res.e
    # sanity: RSM's error sits just above the best rank-3 fit's noise floor
    assert res.e < float(row["sigma"])
