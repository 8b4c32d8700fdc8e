"""Plain FP64 CPU oracle of the RSM hot path (M1 and M2 sampling, L2 norm).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

Paper: Y. Liu, "A random algorithm for low-rank decomposition of large-scale matrices
with missing entries" (arXiv 1411.0814).  Every function follows the paper's own
steps, in its order and notation, with numpy/LAPACK routines as the only building
blocks; nothing is blocked, fused or reordered:

  problem  eq.(problem), eq.(def.rho)  min over U,V of ||W o (Y - U V^T)||, rho = sum(w)/(mn)
  step 1   Section IV-A, step 1        l = r + 1 columns per trial, I trials (an input here)
  step 2   Section III, method M1      pick l columns; keep the rows fully known on them
           Section III, method M2      pick k rows; keep the columns fully known on them
           Section III, text before eq.(get_xi): the l - r right singular vectors of the
           smallest singular values of each sub-matrix (zeta_j)
           eq.(get_xi)                 xi = e(zeta): zeta's entries at the chosen columns of a zero n-vector
  step 3   eq.(solve.barV_L2_norm)     V-hat = the r eigenvectors of Xi Xi^T with the smallest eigenvalues
           eq.(solve.barU)             U-hat row by row: masked least squares against V-hat
  metric   eq.(ep)                     e = (sum w)^-1/2 ||W o (Y - U-hat V-hat^T)||_F

Readings of points the paper leaves open (each is also listed with the design notes):
  * subsets: uniform l-subsets from a counter-based generator (oracle.rng);
  * I counts every draw, accepted or not; a rejected trial contributes nothing;
  * a trial is accepted when it has at least `min_rows` (default r) qualifying rows
    (step 2: "not less than r");
  * nvec = l - r minor vectors per accepted trial, each with unit weight in Xi;
  * singular values beyond the number of rows count as zero (full right basis);
  * "||V|| = 1" is read as V^T V = I_r; "min_U" in eq.(solve.barU) as argmin;
  * a row with fewer than r known entries gets u_i = 0 and is counted as underdetermined;
  * M2 (rows first): a trial is accepted when more than r columns qualify (the text of
    Section IV-A on M2), and it contributes all |C_t| - r right singular vectors past the r
    largest (Section III: "use all zeta_j"), null vectors included.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rng import draw_subsets


@dataclass
class OracleResult:
    V: np.ndarray                 # n x r, orthonormal columns (eigenvectors of N, ascending eigenvalues)
    U: np.ndarray                 # m x r
    N: np.ndarray                 # n x n accumulator Xi Xi^T
    eigvals: np.ndarray           # lambda_1 .. lambda_{r+1} of N, ascending
    subsets: np.ndarray           # I x l
    rows: np.ndarray              # |R_t| per trial
    accepted: int
    uncovered: int                # columns j with N_jj == 0
    rows_underdetermined: int
    e: float                      # eq.(ep)
    extra: dict = field(default_factory=dict)


def qualifying_rows(W: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """M1: the rows whose entries at every chosen column are known, ascending."""
    return np.flatnonzero(np.asarray(W[:, cols], dtype=bool).all(axis=1))


def qualifying_cols(W: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """M2: the columns whose entries at every chosen row are known, ascending."""
    return np.flatnonzero(np.asarray(W[rows, :], dtype=bool).all(axis=0))


def minor_right_singular_vectors(Z: np.ndarray, nvec: int) -> np.ndarray:
    """The nvec right singular vectors of Z for its nvec smallest singular values (l x nvec).

    The full right basis is used, so when Z has fewer rows than columns the null space
    (singular values that count as zero) is part of it, ordered last.
    """
    Z = np.asarray(Z, dtype=np.float64)
    # the right basis is complete (l x l) either way; the full left basis is only needed
    # (and cheap) when there are fewer rows than columns
    _, _, vt = np.linalg.svd(Z, full_matrices=Z.shape[0] < Z.shape[1])
    return vt[vt.shape[0] - nvec:, :].T.copy()


def embed(zeta: np.ndarray, cols: np.ndarray, n: int) -> np.ndarray:
    """eq.(get_xi): place zeta's entries at the chosen column indices of a zero n-vector."""
    xi = np.zeros((n,) + zeta.shape[1:], dtype=np.float64)
    xi[cols] = zeta
    return xi


def trial_constraints(Y, W, cols, r, nvec, min_rows):
    """Step 2 for one trial: (qualifying rows, Xi columns of this trial or None if rejected)."""
    R = qualifying_rows(W, cols)
    if R.size < min_rows:
        return R, None
    Z = np.asarray(Y[np.ix_(R, cols)], dtype=np.float64)
    return R, minor_right_singular_vectors(Z, nvec)


def accumulate_N(Y, W, subsets, r, nvec, min_rows, N=None):
    """Steps 2 and the L2 form of step 3's accumulator: N = Xi Xi^T = sum_j xi_j xi_j^T.

    Xi itself is never stored (Section IV-A, text after eq.(solve.barV_L2_norm)).
    Trials are taken in ascending order.  Returns (N, rows per trial, accepted count).
    """
    n = W.shape[1]
    if N is None:
        N = np.zeros((n, n), dtype=np.float64)
    rows = np.zeros(len(subsets), dtype=np.int64)
    accepted = 0
    for t, cols in enumerate(subsets):
        R, zeta = trial_constraints(Y, W, cols, r, nvec, min_rows)
        rows[t] = R.size
        if zeta is None:
            continue
        accepted += 1
        xi = embed(zeta, cols, n)                    # eq.(get_xi): the columns of Xi
        # eq.(XI): N = Xi Xi^T = sum xi xi^T.  xi xi^T vanishes outside the rows (and
        # columns) where xi is nonzero, so only that block of N is added to.
        S = np.flatnonzero(np.any(xi != 0.0, axis=1))
        N[np.ix_(S, S)] += xi[S] @ xi[S].T
    return N, rows, accepted


def trial_constraints_rows_first(Y, W, rows, r, min_cols):
    """Step 2 with M2 for one trial: (qualifying columns, zeta of this trial or None).

    Z = Y[rows, C] is k x |C|; its right singular vectors past the r largest singular
    values (|C| - r of them, the null space of Z included) are the zeta_j."""
    C = qualifying_cols(W, rows)
    if C.size < min_cols:
        return C, None
    Z = np.asarray(Y[np.ix_(rows, C)], dtype=np.float64)
    return C, minor_right_singular_vectors(Z, C.size - r)


def accumulate_N_rows_first(Y, W, subsets, r, min_cols, N=None):
    """Step 2 with M2 and step 3's accumulator: N = sum over trials of sum_j xi_j xi_j^T,
    xi_j = e(zeta_j) placed at the trial's qualifying columns.  Trials in ascending order.
    Returns (N, |C_t| per trial, accepted count)."""
    n = W.shape[1]
    if N is None:
        N = np.zeros((n, n), dtype=np.float64)
    sizes = np.zeros(len(subsets), dtype=np.int64)
    accepted = 0
    for t, rows in enumerate(subsets):
        C, zeta = trial_constraints_rows_first(Y, W, rows, r, min_cols)
        sizes[t] = C.size
        if zeta is None:
            continue
        accepted += 1
        xi = embed(zeta, C, n)                       # eq.(get_xi) at the trial's columns
        S = np.flatnonzero(np.any(xi != 0.0, axis=1))
        N[np.ix_(S, S)] += xi[S] @ xi[S].T           # eq.(XI)
    return N, sizes, accepted


def solve_V(N: np.ndarray, r: int):
    """eq.(solve.barV_L2_norm): V-hat = eigenvectors of N for the r smallest eigenvalues.

    Returns (V-hat, eigenvalues lambda_1..lambda_{r+1} ascending)."""
    Ns = 0.5 * (N + N.T)
    lam, E = np.linalg.eigh(Ns)
    return E[:, :r].copy(), lam[:r + 1].copy()


def solve_U(Y, W, V, rows=None):
    """eq.(solve.barU), row by row: u_i = argmin_u sum_j w_ij (y_ij - u^T v_j)^2.

    Rows with fewer than r known entries get u_i = 0 and are reported.
    `rows` restricts the solve to a subset of row indices (others stay 0).
    Returns (U, number of underdetermined rows among those solved)."""
    m = W.shape[0]
    r = V.shape[1]
    U = np.zeros((m, r), dtype=np.float64)
    under = 0
    idx = range(m) if rows is None else rows
    for i in idx:
        J = np.flatnonzero(W[i])
        if J.size < r:
            under += 1
            continue
        U[i] = np.linalg.lstsq(V[J], np.asarray(Y[i, J], dtype=np.float64), rcond=None)[0]
    return U, under


def error_e(Y, W, U, V) -> float:
    """eq.(ep): e = (sum_ij w_ij)^(-1/2) * ||W o (Y - U V^T)||_F, formed one row block at a time."""
    m = W.shape[0]
    total = 0.0
    for i0 in range(0, m, 4096):
        i1 = min(m, i0 + 4096)
        Wb = np.asarray(W[i0:i1], dtype=bool)
        Rb = np.asarray(Y[i0:i1], dtype=np.float64) - U[i0:i1] @ V.T
        total += float(np.sum(np.where(Wb, Rb, 0.0) ** 2))
    return float(np.sqrt(total / max(1, int(np.asarray(W, dtype=bool).sum()))))


def rsm(Y, W, r, num_submatrices, seed, l=None, nvec=None, min_rows=None,
        trial_begin=0, subsets=None, with_U=True, with_e=True,
        rows_first=False) -> OracleResult:
    """The whole path: subsets -> N -> V-hat -> U-hat (and e).

    Y: m x n (any float dtype; consumed as FP64), W: m x n bool (True = known).
    `subsets` overrides the random column subsets (I x l); otherwise they are drawn
    from (seed, trial_begin .. trial_begin + num_submatrices - 1).

    rows_first: sampling M2 instead of M1.  Then l is the number k of rows per trial
    (default r + 1), the subsets are row subsets drawn from [0, m), min_rows is the least
    number of qualifying columns for a trial to count (default r + 1, at least r + 1),
    nvec must be left unset, and `rows` of the result holds |C_t| per trial."""
    W = np.asarray(W, dtype=bool)
    m, n = W.shape
    l = r + 1 if not l else int(l)
    if rows_first:
        min_cols = r + 1 if not min_rows else int(min_rows)
        if not (1 <= r < min(m, n)) or not (r < l <= m) or nvec or min_cols <= r:
            raise ValueError("invalid r / k / min_cols for rows-first sampling")
        if subsets is None:
            subsets = draw_subsets(seed, m, l, int(num_submatrices), int(trial_begin))
        subsets = np.asarray(subsets, dtype=np.int64)
        N, rows, accepted = accumulate_N_rows_first(Y, W, subsets, r, min_cols)
        return _finish(Y, W, r, N, subsets, rows, accepted, with_U, with_e)
    nvec = l - r if not nvec else int(nvec)
    min_rows = r if not min_rows else int(min_rows)
    if not (1 <= r < min(m, n)) or not (r < l <= n) or not (1 <= nvec <= l - r):
        raise ValueError("invalid r / l / nvec")
    if subsets is None:
        subsets = draw_subsets(seed, n, l, int(num_submatrices), int(trial_begin))
    subsets = np.asarray(subsets, dtype=np.int64)
    N, rows, accepted = accumulate_N(Y, W, subsets, r, nvec, min_rows)
    return _finish(Y, W, r, N, subsets, rows, accepted, with_U, with_e)


def _finish(Y, W, r, N, subsets, rows, accepted, with_U, with_e) -> OracleResult:
    """Step 3 from the accumulated N: V-hat, U-hat and e."""
    m = W.shape[0]
    V, lam = solve_V(N, r)
    if with_U:
        U, under = solve_U(Y, W, V)
    else:
        U, under = np.zeros((m, r)), 0
    e = error_e(Y, W, U, V) if (with_U and with_e) else float("nan")
    uncovered = int(np.sum(np.diag(N) == 0.0))
    return OracleResult(V=V, U=U, N=N, eigvals=lam, subsets=subsets, rows=rows,
                        accepted=accepted, uncovered=uncovered,
                        rows_underdetermined=under, e=e)
