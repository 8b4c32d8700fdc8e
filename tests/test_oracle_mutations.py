"""The oracle's pins catch plausible mistakes: each test plants one slip in the oracle (on
the CPU, through monkeypatch) and checks that at least one pin then fails.

A pin that stayed green under a planted mistake would not be pinning anything.
"""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import metrics, rsm

_orig_qualifying_rows = rsm.qualifying_rows
_orig_minor = rsm.minor_right_singular_vectors
_orig_embed = rsm.embed
_orig_solve_V = rsm.solve_V
_orig_solve_U = rsm.solve_U


def _largest_singular_vectors(Z, nvec):
    # mistake: the nvec LARGEST right singular vectors
    _, _, vt = np.linalg.svd(np.asarray(Z, dtype=np.float64), full_matrices=True)
    return vt[:nvec].T.copy()


def _rows_any_known(W, cols):
    # mistake: rows with ANY chosen entry known (OR instead of AND)
    return np.flatnonzero(np.asarray(W[:, cols], dtype=bool).any(axis=1))


def _embed_shifted(zeta, cols, n):
    # mistake: off-by-one embedding index
    xi = np.zeros((n,) + zeta.shape[1:])
    xi[(np.asarray(cols) + 1) % n] = zeta
    return xi


def _largest_eigvecs(N, r):
    # mistake: eigenvectors of the LARGEST eigenvalues
    lam, E = np.linalg.eigh(0.5 * (N + N.T))
    return E[:, -r:].copy(), lam[:r + 1].copy()


def _solve_U_no_mask(Y, W, V, rows=None):
    # mistake: the mask is dropped (every entry treated as known)
    return _orig_solve_U(Y, np.ones_like(np.asarray(W, dtype=bool)), V, rows)


def _solve_U_sign(Y, W, V, rows=None):
    # mistake: a sign error in the right-hand side
    U, under = _orig_solve_U(Y, W, V, rows)
    return -U, under


def _accumulate_drop_last(Y, W, subsets, r, nvec, min_rows, N=None):
    # mistake: the last trial's constraint is dropped but still counted as accepted
    N2, rows, acc = _orig_accumulate(Y, W, subsets[:-1], r, nvec, min_rows, N)
    return N2, np.concatenate([rows, [rows[-1] if len(rows) else 0]]), acc + 1


_orig_accumulate = rsm.accumulate_N


def _rel_rms_no_mask(W, U1, V1, U2, V2, block=8192):
    # mistake: every entry counted, known or not
    P1, P2 = U1 @ V1.T, U2 @ V2.T
    return float(np.sqrt(np.sum((P1 - P2) ** 2) / np.sum(P2 ** 2)))


def _rel_rms_other_normaliser(W, U1, V1, U2, V2, block=8192):
    # mistake: normalised by the first product instead of the reference one
    W = np.asarray(W, dtype=bool)
    P1, P2 = U1 @ V1.T, U2 @ V2.T
    return float(np.sqrt(np.sum(np.where(W, P1 - P2, 0.0) ** 2) / np.sum(np.where(W, P1, 0.0) ** 2)))


def _fails(fn) -> bool:
    try:
        fn()
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("attr,bad,tests", [
    ("qualifying_rows", _rows_any_known,
     ["test_qualifying_rows_brute_force", "test_N_invariants_noisy"]),
    ("minor_right_singular_vectors", _largest_singular_vectors,
     ["test_minor_vector_is_null_on_true_rows_noise_free",
      "test_minor_vector_projector_matches_gram_eigh_noisy", "test_N_brute_force_all_subsets_tiny"]),
    ("embed", _embed_shifted, ["test_embedding"]),
    # the accumulator builds every xi through embed, so the same slip is caught there too
    ("embed", _embed_shifted, ["test_N_brute_force_all_subsets_tiny"]),
    ("solve_V", _largest_eigvecs, ["test_full_mask_l_equals_n_is_truncated_svd"]),
    ("solve_U", _solve_U_no_mask, ["test_U_is_masked_least_squares"]),
    ("solve_U", _solve_U_sign, ["test_U_full_mask_closed_form"]),
    ("accumulate_N", _accumulate_drop_last, ["test_N_invariants_noisy"]),
])
def test_planted_mistake_is_caught(monkeypatch, attr, bad, tests):
    monkeypatch.setattr(rsm, attr, bad)
    caught = [name for name in tests if _fails(getattr(pins, name))]
    assert caught, f"no pin caught the planted mistake in {attr}"


@pytest.mark.parametrize("bad", [_rel_rms_no_mask, _rel_rms_other_normaliser])
def test_planted_mistake_in_the_parity_metric_is_caught(monkeypatch, bad):
    monkeypatch.setattr(metrics, "rel_rms_known", bad)
    assert _fails(pins.test_rel_rms_known_brute_force)


def test_pins_pass_without_mistakes():
    # the same pins, unpatched, are green (guards against a pin that always fails)
    for name in ["test_qualifying_rows_brute_force", "test_embedding",
                 "test_rel_rms_known_brute_force", "test_N_invariants_noisy",
                 "test_U_full_mask_closed_form", "test_minor_vector_projector_matches_gram_eigh_noisy"]:
        getattr(pins, name)()
