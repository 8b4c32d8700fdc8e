"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on small and medium
problems that span several tiles and a ragged tail, plus the method's edge cases."""
import itertools

import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import gram_bound_ok, lower_N, to_device

pytestmark = pytest.mark.gpu

THETA_TOL = 1e-4      # largest principal angle vs the oracle (radians)
RMS_TOL = 1e-5        # relative RMS of U V^T on known entries vs the oracle


def _run(p, gram, row_major=False, **kw):
    import torch
    from paper_1411_0814_amd import decompose
    Y, W = to_device(p, row_major=row_major)
    res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram, **kw)
    info = res.info()
    torch.cuda.synchronize()
    return res, info


def _compare_full(p, res, info, ora, u, theta_tol=THETA_TOL, rms_tol=RMS_TOL, n_gram=200,
                  n_tol=None):
    # a1: subsets bit-exact
    cols = res.taps["cols"].cpu().numpy()
    assert np.array_equal(cols, ora.subsets)
    # a2: qualifying row counts bit-exact
    rows = res.taps["rows"].cpu().numpy()
    assert np.array_equal(rows, ora.rows)
    assert info["accepted"] == ora.accepted
    assert info["rows_total"] == int(ora.rows.sum())
    # a3: Grams within the dot-product error bound, on a sample of trials
    G = res.taps["gram"].cpu().numpy()
    Y64 = np.asarray(p.Y, dtype=np.float64)
    for t in np.linspace(0, len(cols) - 1, min(n_gram, len(cols))).astype(int):
        R = rsm.qualifying_rows(p.W, cols[t])
        ok, ratio = gram_bound_ok(G[t], Y64[np.ix_(R, cols[t])], u)
        assert ok, (t, ratio)
    # a4: minor-vector projectors vs the oracle's SVD (trials with a clear eigen-gap)
    vecs = res.taps["vecs"].cpu().numpy()
    eigs = res.taps["eigs"].cpu().numpy()
    nv = vecs.shape[1]
    checked = 0
    for t in range(0, len(cols), max(1, len(cols) // 100)):
        if rows[t] < p.r:
            continue
        lam = eigs[t]
        if lam[nv] - lam[nv - 1] < 1e-6 * max(lam[-1], 1e-300):
            continue
        R = rsm.qualifying_rows(p.W, cols[t])
        z = rsm.minor_right_singular_vectors(Y64[np.ix_(R, cols[t])], nv)
        P_ref = z @ z.T
        P_gpu = vecs[t].T @ vecs[t]
        gap = (lam[nv] - lam[nv - 1]) / lam[-1]
        assert np.abs(P_gpu - P_ref).max() <= max(1e-9, 50 * u / gap), t
        checked += 1
    assert checked > 0
    # a5: N
    N = lower_N(res.N) if res.N is not None else None
    if N is not None:
        tol = 1e3 * u if n_tol is None else n_tol
        assert np.abs(N - ora.N).max() <= tol * max(1.0, np.abs(ora.N).max())
    # a6: V-hat subspace
    V = res.V.cpu().numpy()
    assert np.abs(V.T @ V - np.eye(p.r)).max() < 1e-12
    theta = metrics.principal_angle_max(V, ora.V)
    assert theta <= theta_tol, theta
    # a7: U-hat V-hat^T on known entries
    U = res.U.cpu().numpy()
    rms = metrics.rel_rms_known(p.W, U, V, ora.U, ora.V)
    assert rms <= rms_tol, rms
    return theta, rms


def test_plain_fp64_parity():
    """2000 x 200, r=5, l=6, rho=0.7, noise 1e-3, 800 trials, FP64 end to end."""
    import torch
    from paper_1411_0814_amd import _lib
    p = synth.plain_fp64()
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    res, info = _run(p, "f64", taps=True, N=N, flags=_lib.COMPUTE_ERROR)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l)
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-53)
    assert theta < 1e-9
    assert info["uncovered"] == ora.uncovered == 0
    assert abs(info["e"] - ora.e) <= 1e-8 * ora.e
    assert info["known"] == int(p.W.sum())
    lam = np.array(info["lambda"][:p.r + 1])
    # lambda_1..lambda_r converge with V-hat; lambda_{r+1} is a Ritz value (upper bound)
    assert np.allclose(lam[:p.r], ora.eigvals[:p.r], rtol=1e-6, atol=1e-12 * ora.eigvals[-1])
    assert ora.eigvals[p.r] * (1 - 1e-9) <= lam[p.r] <= 1.5 * ora.eigvals[p.r]
    assert info["warnings"] == []
    print(f"plain_fp64: theta={theta:.3e} rms={rms:.3e} e={info['e']:.6g} (oracle {ora.e:.6g})")


def test_noise_free_exact_recovery_fp64():
    """Theorem 1 with no noise: V-hat spans the true row space to < 1e-10 rad."""
    p = synth.paper_synthetic(3000, 96, 6, 0.75, 0.0, 21, num_submatrices=1500, l=7)
    res, info = _run(p, "f64")
    theta = metrics.principal_angle_max(res.V.cpu().numpy(), p.Vbar)
    assert theta < 1e-10, theta
    assert info["lambda"][p.r - 1] < 1e-10 * info["lambda"][p.r]


def test_fp32_gram_parity_medium():
    """16384 x 256, r=8, l=9, rho=0.8, FP32 data and Gram, 2048 trials."""
    p = synth.paper_synthetic(16384, 256, 8, 0.8, 1e-2, 5, factor_dtype=np.float32,
                              y_dtype=np.float32, relative_sigma=True, num_submatrices=2048,
                              l=9, gram="f32")
    res, info = _run(p, "f32", taps=True)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l)
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-24)
    print(f"fp32 medium: theta={theta:.3e} rms={rms:.3e}")


@pytest.mark.parametrize("gram", ["f64", "f32"])
def test_low_row_regime_of_table1(gram):
    """The regime of the paper's own workloads (Table I): rho = 0.2, l = 4, r = 3, noise 0.2,
    25 n trials, so a trial keeps about m rho^4 = 52 of m = 32768 rows (a reduced 32768 x
    256 shape of its first row)."""
    dt = np.float32 if gram == "f32" else np.float64
    p = synth.paper_synthetic(32768, 256, 3, 0.2, 0.2, 71, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=25 * 256, l=4, seed_rsm=72, gram=gram)
    res, info = _run(p, gram, taps=True)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
    mean_rows = info["rows_total"] / p.num_submatrices
    assert 30 < mean_rows < 80, mean_rows
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-24 if gram == "f32" else 2.0**-53)
    print(f"low-row regime {gram}: mean rows {mean_rows:.1f} theta={theta:.3e} rms={rms:.3e}",
          flush=True)


@pytest.mark.parametrize("gram", ["f32", "f64"])
def test_few_qualifying_rows_gathered(gram):
    """FP32 data whose trials keep about 22 of 30011 rows (rho = 0.3, l = 6): the built-in
    kernel choice gathers the qualifying values from Y instead of staging every column; FP32
    and FP64 sums."""
    p = synth.paper_synthetic(30011, 301, 5, 0.3, 1e-2, 73, factor_dtype=np.float32,
                              y_dtype=np.float32, relative_sigma=True, num_submatrices=2000,
                              l=6, seed_rsm=74, gram=gram)
    res, info = _run(p, gram, taps=True)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-24 if gram == "f32" else 2.0**-53)
    print(f"gathered {gram}: mean rows {info['rows_total'] / p.num_submatrices:.1f} "
          f"theta={theta:.3e} rms={rms:.3e}", flush=True)


def test_ragged_row_major_fp64():
    """m, n not multiples of 64; row-major Y and W (repacked by the library)."""
    import torch
    p = synth.paper_synthetic(1000, 70, 3, 0.8, 0.01, 8, num_submatrices=700, l=4)
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    res, info = _run(p, "f64", row_major=True, taps=True, N=N)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l)
    _compare_full(p, res, info, ora, u=2.0**-53)


def test_nvec_two_l_plus_two():
    """l = r + 2 with both minor vectors per trial (nvec = 2)."""
    p = synth.paper_synthetic(1500, 60, 3, 0.85, 0.01, 9, num_submatrices=500, l=5)
    res, info = _run(p, "f64", taps=True, nvec=2)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=5, nvec=2)
    _compare_full(p, res, info, ora, u=2.0**-53)


# l > r + 1 with fewer minor vectors than l - r (the choice of ell the paper allows),
# through both register Jacobi (l <= 11) and the wavefront Jacobi (l >= 12).  The ell
# vectors are picked among l - r noise directions, so the noise must separate their
# eigenvalues: at l >= 12 and noise 0.01 every trial's gap between the ell-th and the next
# eigenvalue is below 1e-6 of the largest (the chosen subspace is not defined to the
# precision compared); at noise 1 the smallest gap is above 5e-5.
@pytest.mark.parametrize("r,l,nvec,gram,noise", [(3, 6, 1, "f64", 0.01), (3, 6, 2, "f64", 0.01),
                                                 (2, 7, 3, "f32", 0.01), (4, 13, 3, "f64", 1.0),
                                                 (5, 14, 1, "f32", 1.0)])
def test_l_above_r_plus_one_with_fewer_vectors(r, l, nvec, gram, noise):
    dt = np.float32 if gram == "f32" else np.float64
    p = synth.paper_synthetic(2500, 90, r, 0.9, noise, 20 + l, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=900, l=l, gram=gram)
    res, info = _run(p, gram, taps=True, nvec=nvec)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=l, nvec=nvec)
    _compare_full(p, res, info, ora, u=2.0**-24 if gram == "f32" else 2.0**-53)


def test_maximum_sizes_fp64():
    """n = RSM_MAX_N = 2048, r = RSM_MAX_R = 16, l = RSM_MAX_L = 17 (the per-trial streaming
    Gram: the n-column tile does not fit LDS), FP64 end to end."""
    import torch
    p = synth.paper_synthetic(6000, 2048, 16, 0.96, 0.01, 61, num_submatrices=3000, l=17)
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    res, info = _run(p, "f64", taps=True, N=N)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
    # the Gram of ~3000 rows squares the sub-matrix's condition: each minor vector differs
    # from the oracle's SVD by up to |R| u lambda_max / gap (checked per trial above), so N
    # is compared at 1e-10 of its largest entry instead of 1e3 u
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-53, n_gram=40, n_tol=1e-10)
    print(f"maximum sizes: theta={theta:.3e} rms={rms:.3e}")


def test_user_subsets_brute_force_tiny():
    """n = 7, l = 3: every C(7,3) subset passed in; N equals the oracle's brute force."""
    import torch
    from paper_1411_0814_amd import decompose
    p = synth.paper_synthetic(120, 7, 2, 0.85, 0.01, 7)
    subsets = np.array(list(itertools.combinations(range(7), 3)), dtype=np.int32)
    Y, W = to_device(p)
    N = torch.zeros((7, 7), dtype=torch.float64, device="cuda")
    res = decompose(Y, W, 2, len(subsets), 0, l=3, gram="f64", N=N,
                    subsets=torch.from_numpy(subsets).cuda())
    info = res.info()
    ora = rsm.rsm(p.Y, p.W, 2, len(subsets), seed=0, subsets=subsets)
    assert np.abs(lower_N(res.N) - ora.N).max() < 1e-12
    assert info["accepted"] == ora.accepted
    theta = metrics.principal_angle_max(res.V.cpu().numpy(), ora.V)
    assert theta < 1e-8


def test_bad_user_subset_rejected():
    import torch
    from paper_1411_0814_amd import decompose
    p = synth.paper_synthetic(200, 10, 2, 0.9, 0.01, 3)
    subsets = np.array([[0, 1, 2], [3, 3, 4], [5, 6, 11], [7, 8, 9]], dtype=np.int32)
    Y, W = to_device(p)
    res = decompose(Y, W, 2, 4, 0, l=3, gram="f64", subsets=torch.from_numpy(subsets).cuda(),
                    taps=True)
    info = res.info()
    assert "bad_subset" in info["warnings"]
    assert info["accepted"] <= 2


def test_split_run_resume_equals_whole():
    """Trials [0, I/2) then [I/2, I) accumulated onto the same N, then finalised."""
    import torch
    from paper_1411_0814_amd import _lib, decompose
    p = synth.plain_fp64()
    Y, W = to_device(p)
    I = p.num_submatrices
    whole = decompose(Y, W, p.r, I, p.seed_rsm, l=p.l, gram="f64",
                      N=torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda"))
    N = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    decompose(Y, W, p.r, I // 2, p.seed_rsm, l=p.l, gram="f64", N=N,
              flags=_lib.ACCUMULATE_ONLY)
    decompose(Y, W, p.r, I - I // 2, p.seed_rsm, l=p.l, gram="f64", N=N, trial_begin=I // 2,
              flags=_lib.ACCUMULATE_ONLY | _lib.N_ACCUMULATE)
    fin = decompose(Y, W, p.r, 0, p.seed_rsm, l=p.l, gram="f64", N=N, flags=_lib.FINALIZE_ONLY)
    fin.info()
    whole.info()
    assert np.abs(lower_N(N) - lower_N(whole.N)).max() < 1e-12
    theta = metrics.principal_angle_max(fin.V.cpu().numpy(), whole.V.cpu().numpy())
    assert theta < 1e-10
    assert np.abs(fin.U.cpu().numpy() @ fin.V.cpu().numpy().T
                  - whole.U.cpu().numpy() @ whole.V.cpu().numpy().T).max() < 1e-9


def test_no_trials_warns():
    from paper_1411_0814_amd import decompose
    p = synth.paper_synthetic(300, 20, 2, 0.8, 0.01, 4)
    Y, W = to_device(p)
    res = decompose(Y, W, 2, 0, 1, gram="f64")
    info = res.info()
    assert "no_constraints" in info["warnings"]
    assert info["accepted"] == 0
    V = res.V.cpu().numpy()
    assert np.all(np.isfinite(V)) and np.abs(V.T @ V - np.eye(2)).max() < 1e-12


def test_uncovered_column_and_underdetermined_rows():
    p = synth.paper_synthetic(400, 30, 3, 0.8, 0.01, 6, num_submatrices=600)
    p.Wt[5, :] = 0          # column 5 never known -> never in an accepted trial
    p.Wt[:, 17] = 0
    p.Wt[:2, 17] = 1        # row 17 has 2 < r known entries
    res, info = _run(p, "f64")
    assert info["uncovered"] >= 1
    assert "rank_deficient" in info["warnings"]
    assert "rows_underdetermined" in info["warnings"]
    assert info["rows_underdetermined"] == 1
    U = res.U.cpu().numpy()
    assert np.all(U[17] == 0.0)
    ora = rsm.rsm(p.Y, p.W, 3, p.num_submatrices, seed=p.seed_rsm, with_U=False)
    assert ora.uncovered == info["uncovered"]


def test_trial_begin_shifts_the_stream():
    from paper_1411_0814_amd import decompose
    p = synth.paper_synthetic(500, 40, 3, 0.8, 0.01, 2, num_submatrices=100)
    Y, W = to_device(p)
    a = decompose(Y, W, 3, 100, 9, gram="f64", taps=True)
    b = decompose(Y, W, 3, 60, 9, gram="f64", taps=True, trial_begin=40)
    a.info(), b.info()
    assert np.array_equal(a.taps["cols"].cpu().numpy()[40:], b.taps["cols"].cpu().numpy())
    assert np.array_equal(a.taps["rows"].cpu().numpy()[40:], b.taps["rows"].cpu().numpy())


def test_large_l_fp32_parity():
    """r = 12, l = 13 (the LDS Jacobi path and 256-thread Gram tiles), FP32 data and Gram."""
    p = synth.paper_synthetic(8000, 150, 12, 0.95, 1e-3, 12, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=700, l=13, gram="f32")
    res, info = _run(p, "f32", taps=True)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l)
    theta, rms = _compare_full(p, res, info, ora, u=2.0**-24)
    print(f"large l fp32: theta={theta:.3e} rms={rms:.3e}")


def test_small_l_fp64_tiled():
    """r = 1, l = 2: the smallest template instances."""
    p = synth.paper_synthetic(700, 40, 1, 0.8, 1e-2, 13, num_submatrices=300, l=2)
    res, info = _run(p, "f64", taps=True)
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l)
    _compare_full(p, res, info, ora, u=2.0**-53)
