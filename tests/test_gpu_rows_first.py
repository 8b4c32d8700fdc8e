"""Parity of rows-first sampling (method M2, Section III) on the GPU with the FP64 oracle:
subsets and qualifying-column counts bit-exact, the k x k Grams within the dot-product bound,
N, V-hat and U-hat V-hat^T against the oracle; noise-free exact recovery; every row subset
of a tiny matrix; deterministic results alone and in a batch; the paper-scale shape."""
import itertools

import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import gram_bound_ok, lower_N, to_device

pytestmark = pytest.mark.gpu


def _run(p, row_major=False, **kw):
    import torch
    from paper_1411_0814_amd import _lib, decompose
    flags = _lib.ROWS_FIRST | kw.pop("flags", 0)
    Y, W = to_device(p, row_major=row_major)
    res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram="f64", flags=flags,
                    **kw)
    info = res.info()
    torch.cuda.synchronize()
    return res, info


def _compare(p, res, info, ora, theta_tol, rms_tol, n_gram=100):
    # a1: row subsets, a2: qualifying-column counts, bit-exact
    S = res.taps["cols"].cpu().numpy()
    assert np.array_equal(S, ora.subsets)
    cnt = res.taps["rows"].cpu().numpy()
    assert np.array_equal(cnt, ora.rows)
    assert info["accepted"] == ora.accepted > 0
    assert info["rows_total"] == int(ora.rows.sum())
    # a3: H_t = Z_t Z_t^T in FP64, within the dot-product bound; a4: its eigenvalues
    H = res.taps["gram"].cpu().numpy()
    eigs = res.taps["eigs"].cpu().numpy()
    Y64 = np.asarray(p.Y, dtype=np.float64)
    for t in np.linspace(0, len(S) - 1, min(n_gram, len(S))).astype(int):
        C = rsm.qualifying_cols(p.W, S[t])
        Zt = Y64[np.ix_(S[t], C)].T                    # |C| x k: H = Zt^T Zt
        ok, ratio = gram_bound_ok(H[t], Zt, 2.0**-53)
        assert ok, (t, ratio)
        if cnt[t] > p.r:
            lam = np.linalg.eigvalsh(Zt.T @ Zt)
            assert np.allclose(eigs[t], lam, rtol=1e-9, atol=1e-12 * lam[-1]), t
    # a5: N
    N = lower_N(res.N)
    assert np.abs(N - ora.N).max() <= 1e-9 * max(1.0, np.abs(ora.N).max())
    # a6, a7
    V = res.V.cpu().numpy()
    assert np.abs(V.T @ V - np.eye(p.r)).max() < 1e-12
    theta = metrics.principal_angle_max(V, ora.V)
    assert theta <= theta_tol, theta
    rms = metrics.rel_rms_known(p.W, res.U.cpu().numpy(), V, ora.U, ora.V)
    assert rms <= rms_tol, rms
    return theta, rms


# (m, n, r, k, rho, noise, dtype, row_major, trials): ragged m and n, both storage orders,
# FP32 and FP64 Y, k from r + 1 to the wavefront sizes of the k x k eigen-solve
CASES = [(1000, 150, 3, 4, 0.8, 0.01, np.float64, False, 600),
         (3001, 203, 5, 6, 0.85, 0.01, np.float32, True, 900),
         (2000, 300, 10, 13, 0.96, 0.01, np.float64, False, 400),
         (4097, 97, 8, 9, 0.9, 0.05, np.float32, False, 700)]


@pytest.mark.parametrize("m,n,r,k,rho,noise,dt,rm,trials", CASES)
def test_rows_first_parity(m, n, r, k, rho, noise, dt, rm, trials):
    import torch
    p = synth.paper_synthetic(m, n, r, rho, noise, 40 + k, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=trials, l=k, seed_rsm=k)
    N = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    res, info = _run(p, row_major=rm, taps=True, N=N)
    ora = rsm.rsm(p.Y, p.W, r, trials, seed=p.seed_rsm, l=k, rows_first=True)
    theta, rms = _compare(p, res, info, ora, theta_tol=1e-4, rms_tol=1e-5)
    print(f"rows first m={m} n={n} r={r} k={k}: theta={theta:.3e} rms={rms:.3e}")


def test_rows_first_maximum_sizes():
    """n = 2048, r = 16, k = 17 rows per trial (the LDS-resident k x k eigen-solve)."""
    import torch
    p = synth.paper_synthetic(3000, 2048, 16, 0.8, 0.01, 62, num_submatrices=2000, l=17,
                              seed_rsm=5)
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    res, info = _run(p, taps=True, N=N)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=17, rows_first=True,
                  with_e=False)
    theta, rms = _compare(p, res, info, ora, theta_tol=1e-4, rms_tol=1e-5, n_gram=40)
    print(f"rows first maximum sizes: theta={theta:.3e} rms={rms:.3e}")


def test_rows_first_noise_free_exact_recovery():
    p = synth.paper_synthetic(1500, 120, 4, 0.85, 0.0, 51, num_submatrices=800, l=5)
    res, info = _run(p)
    theta = metrics.principal_angle_max(res.V.cpu().numpy(), p.Vbar)
    assert theta < 1e-10, theta
    assert info["lambda"][p.r - 1] < 1e-10 * info["lambda"][p.r]


def test_rows_first_every_row_subset_tiny():
    """m = 7, k = 3: every C(7,3) row subset passed in; N equals the oracle's."""
    import torch
    from paper_1411_0814_amd import _lib, decompose
    p = synth.paper_synthetic(7, 40, 2, 0.8, 0.05, 25)
    subsets = np.array(list(itertools.combinations(range(7), 3)), dtype=np.int32)
    Y, W = to_device(p)
    N = torch.zeros((40, 40), dtype=torch.float64, device="cuda")
    res = decompose(Y, W, 2, len(subsets), 0, l=3, gram="f64", N=N, flags=_lib.ROWS_FIRST,
                    subsets=torch.from_numpy(subsets).cuda())
    info = res.info()
    ora = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=subsets, l=3, rows_first=True)
    assert info["accepted"] == ora.accepted
    assert np.abs(lower_N(res.N) - ora.N).max() < 1e-11


def test_rows_first_no_accepted_trial_is_flagged():
    from paper_1411_0814_amd import _lib
    p = synth.paper_synthetic(500, 60, 3, 0.3, 0.01, 52, num_submatrices=200, l=4)
    # no trial can have 61 of the 60 columns
    res, info = _run(p, min_rows=61)
    assert info["accepted"] == 0
    assert info["warn"] & _lib.W_NO_CONSTRAINTS


def test_rows_first_deterministic_alone_and_in_a_batch():
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose_batched
    a = synth.paper_synthetic(3000, 200, 4, 0.85, 0.01, 53, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=700, l=5)
    b = synth.paper_synthetic(2000, 150, 3, 0.8, 0.01, 54, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=500, l=4)
    flags = _lib.ROWS_FIRST | _lib.DETERMINISTIC

    def req(p, fl):
        Y, W = to_device(p)
        return Request(Y=Y, W=W, r=p.r, num_submatrices=p.num_submatrices, seed=p.seed_rsm,
                       l=p.l, gram="f32", flags=fl,
                       N=torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda"))

    alone = decompose_batched([req(a, flags)])[0]
    mix = decompose_batched([req(b, flags), req(a, 0), req(a, flags), req(b, 0)])[2]
    torch.cuda.synchronize()
    assert torch.equal(alone.N, mix.N)
    assert torch.equal(alone.V, mix.V)
    assert torch.equal(alone.U, mix.U)


def test_rows_first_paper_scale_shape():
    """131072 x 1024, r = 8, k = 9 rows per trial, rho = 0.8, 8192 trials, FP32 Y."""
    import torch
    p = synth.paper_synthetic(131072, 1024, 8, 0.8, 1e-2, 55, factor_dtype=np.float32,
                              y_dtype=np.float32, relative_sigma=True, num_submatrices=8192,
                              l=9, seed_rsm=3)
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    res, info = _run(p, N=N)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=9, rows_first=True,
                  with_U=False)
    assert info["accepted"] == ora.accepted
    assert info["rows_total"] == int(ora.rows.sum())
    assert np.abs(lower_N(res.N) - ora.N).max() <= 1e-9 * np.abs(ora.N).max()
    V = res.V.cpu().numpy()
    theta = metrics.principal_angle_max(V, ora.V)
    # U-hat on a seeded sample of rows, solved by the oracle with its own V-hat
    rows = np.sort(np.random.default_rng(0).choice(p.m, 2000, replace=False))
    Uo, _ = rsm.solve_U(p.Y, p.W, ora.V, rows=rows)
    Ug = res.U.cpu().numpy()
    rms = metrics.rel_rms_known(p.W[rows], Ug[rows], V, Uo[rows], ora.V)
    assert theta <= 1e-4 and rms <= 1e-5, (theta, rms)
    print(f"rows first paper-scale shape: theta={theta:.3e} rms={rms:.3e}")


def test_rows_first_split_run_equals_whole_bitwise():
    """Trials [0, I/3) then [I/3, I) onto one N (deterministic mode: bitwise), then
    finalised: the per-GPU share of a sharded run."""
    import torch
    from paper_1411_0814_amd import _lib, decompose
    p = synth.paper_synthetic(2500, 180, 4, 0.85, 0.01, 56, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=600, l=5)
    Y, W = to_device(p)
    I, cut = p.num_submatrices, p.num_submatrices // 3
    base = _lib.ROWS_FIRST | _lib.DETERMINISTIC
    whole = decompose(Y, W, p.r, I, p.seed_rsm, l=p.l, flags=base,
                      N=torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda"))
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    decompose(Y, W, p.r, cut, p.seed_rsm, l=p.l, N=N, flags=base | _lib.ACCUMULATE_ONLY)
    decompose(Y, W, p.r, I - cut, p.seed_rsm, l=p.l, N=N, trial_begin=cut,
              flags=base | _lib.ACCUMULATE_ONLY | _lib.N_ACCUMULATE)
    fin = decompose(Y, W, p.r, 0, p.seed_rsm, l=p.l, N=N, flags=base | _lib.FINALIZE_ONLY)
    fin.info()
    whole.info()
    torch.cuda.synchronize()
    assert torch.equal(torch.tril(N.T), torch.tril(whole.N.T))
    assert torch.equal(fin.V, whole.V)
    assert torch.equal(fin.U, whole.U)


def test_rows_first_error_e_matches_oracle():
    """eq.(ep) on the rows-first result (the optional error pass shared with M1)."""
    from paper_1411_0814_amd import _lib
    p = synth.paper_synthetic(2000, 120, 4, 0.85, 0.02, 57, num_submatrices=500, l=5)
    res, info = _run(p, flags=_lib.COMPUTE_ERROR)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=5, rows_first=True)
    # the GPU's V-hat differs from the oracle's by ~1e-7 rad here (H_t route, FP64), which
    # moves e by ~1e-8 relative
    assert abs(info["e"] - ora.e) <= 1e-6 * ora.e
    # and close to the noise level of the data
    assert 0.5 * p.sigma < info["e"] < 2.0 * p.sigma
