"""Step a6 alone (RSM_FINALIZE_ONLY with a given N): the V-hat solver iterates until its
residual test passes, also when the r-th and (r+1)-th eigenvalues of N are close, and
reports the number of steps it took.  Reference: the r eigenvectors of N with the smallest
eigenvalues (eq.(solve.barV_L2_norm)) from LAPACK's eigh."""
import numpy as np
import pytest

from oracle import metrics

pytestmark = pytest.mark.gpu


def _spd(n, lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    N = (Q * lam) @ Q.T
    return 0.5 * (N + N.T)


def _finalize(N, r, seed=3):
    import torch
    from paper_1411_0814_amd import _lib, decompose
    n = N.shape[0]
    m = 600
    rng = np.random.default_rng(seed)
    Y = torch.from_numpy(rng.standard_normal((n, m))).cuda().T   # column-major m x n
    W = torch.from_numpy(rng.random((n, m)) < 0.8).cuda().T
    Nt = torch.from_numpy(np.ascontiguousarray(N.T)).cuda()      # column-major n x n
    res = decompose(Y, W, r, 0, 1, gram="f64", N=Nt, flags=_lib.FINALIZE_ONLY)
    info = res.info()
    return res.V.cpu().numpy(), info


CASES = {
    # lambda_r / lambda_{r+1} = 0.99, the rest spread above
    "gap_0.99": (300, 6, lambda n, r: np.concatenate(
        [np.linspace(1.0, 5.0, r), [5.0 / 0.99], np.linspace(5.2, 40.0, n - r - 1)])),
    # the wanted directions at the edge of a dense bulk (the shape of the precision-stress
    # workload's N: lambda_8 = 4.51, lambda_9 = 4.80, about 1% apart further up)
    "bulk_edge": (512, 8, lambda n, r: np.concatenate(
        [[9.86e-06, 7.25e-05, 6.21e-04, 9.85e-03, 2.71e-01, 3.83, 3.92, 4.51, 4.80, 4.99,
          5.09, 5.14, 5.16, 5.22, 5.25, 5.32, 5.40, 5.43, 5.49, 5.50],
         np.linspace(5.6, 45.0, n - 20)])),
    # wanted eigenvalues near zero and well separated (the paper-scale workload's N)
    "near_zero": (400, 8, lambda n, r: np.concatenate(
        [np.geomspace(1e-9, 3e-7, r), np.linspace(2.5, 30.0, n - r)])),
}


@pytest.mark.parametrize("name", list(CASES))
def test_solver_converges_by_residual(name):
    n, r, lam_fn = CASES[name]
    lam = lam_fn(n, r)
    N = _spd(n, lam, seed=len(name))
    V, info = _finalize(N, r)
    w, E = np.linalg.eigh(N)
    theta = metrics.principal_angle_max(V, E[:, :r])
    print(f"[eig] {name}: theta {theta:.2e} residual {info['residual']:.2e} "
          f"iterations {info['eig_iterations']} lambda_r {info['lambda'][r - 1]:.6g} "
          f"lambda_r1 {info['lambda'][r]:.6g} warnings {info['warnings']}", flush=True)
    assert "not_converged" not in info["warnings"]
    assert info["residual"] <= 1e-8
    assert theta <= 1e-6, theta
    assert np.abs(V.T @ V - np.eye(r)).max() <= 1e-12
    # Ritz values of the wanted pairs equal the eigenvalues to the residual's order
    assert np.allclose(info["lambda"][:r], w[:r], rtol=1e-8, atol=1e-9 * w[-1])
    if name == "near_zero":
        assert info["eig_iterations"] == 2       # one step shrinks the rest by ~1e-7
    else:
        assert info["eig_iterations"] > 3


def test_batched_solves_one_workgroup_per_problem():
    # six problems of the same subspace width in one call take the one-workgroup-per-problem
    # form of the iteration; each must match its own eigh like the single calls above
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose_batched
    reqs, refs = [], []
    rng = np.random.default_rng(11)
    for k, name in enumerate(["gap_0.99", "bulk_edge", "near_zero"] * 2):
        n, _, lam_fn = CASES[name]
        n -= 37 * k                          # uneven sizes
        r = 8                                # one subspace width for the whole call
        lam = lam_fn(n, r)
        N = _spd(n, lam, seed=100 + k)
        m = 500
        Y = torch.from_numpy(rng.standard_normal((n, m))).cuda().T
        W = torch.from_numpy(rng.random((n, m)) < 0.8).cuda().T
        Nt = torch.from_numpy(np.ascontiguousarray(N.T)).cuda()
        reqs.append(Request(Y=Y, W=W, r=r, num_submatrices=0, seed=1, gram="f64", N=Nt,
                            flags=_lib.FINALIZE_ONLY))
        refs.append((N, r, name))
    out = decompose_batched(reqs)
    torch.cuda.synchronize()
    for res, (N, r, name) in zip(out, refs):
        V, info = res.V.cpu().numpy(), res.info()
        E = np.linalg.eigh(N)[1]
        theta = metrics.principal_angle_max(V, E[:, :r])
        print(f"[eig batched] {name} n={N.shape[0]}: theta {theta:.2e} iterations "
              f"{info['eig_iterations']} residual {info['residual']:.2e}", flush=True)
        assert "not_converged" not in info["warnings"]
        assert theta <= 1e-6
        assert np.abs(V.T @ V - np.eye(r)).max() <= 1e-12
