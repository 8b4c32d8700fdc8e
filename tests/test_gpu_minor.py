"""Step a4: the minor vector by inverse iteration (one vector per trial, no eigen taps)
against the full Jacobi eigen-decomposition (taken when the eigen taps are requested) and
against the FP64 oracle, for l across the range of both Jacobi kernels."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import lower_N, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("l,dt", [(3, np.float64), (6, np.float32), (9, np.float32),
                                  (12, np.float64), (15, np.float32), (17, np.float32)])
def test_inverse_iteration_matches_jacobi_and_oracle(l, dt):
    import torch
    from paper_1411_0814_amd import _lib, decompose
    gram = "f32" if dt == np.float32 else "f64"
    r = l - 1
    p = synth.paper_synthetic(4001, 120, r, 0.93, 1e-3, 300 + l, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=1500, seed_rsm=l, gram=gram)
    Y, W = to_device(p)
    N_inv = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
    N_jac = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
    a = decompose(Y, W, r, p.num_submatrices, p.seed_rsm, l=l, gram=gram, N=N_inv,
                  flags=_lib.N_ACCUMULATE)
    b = decompose(Y, W, r, p.num_submatrices, p.seed_rsm, l=l, gram=gram, N=N_jac,
                  flags=_lib.N_ACCUMULATE, taps=True)
    ia, ib = a.info(), b.info()
    assert ia["accepted"] == ib["accepted"] > 0
    Na, Nb = lower_N(N_inv), lower_N(N_jac)
    ora = rsm.rsm(p.Y, p.W, r, p.num_submatrices, seed=p.seed_rsm, l=l, with_e=False)
    scale = np.max(np.abs(ora.N))
    err_inv = np.max(np.abs(Na - ora.N)) / scale
    err_jac = np.max(np.abs(Nb - ora.N)) / scale
    if dt == np.float64:
        # FP64 Grams: both eigen-solvers are accurate to rounding
        assert np.max(np.abs(Na - Nb)) <= 1e-10 * scale
    else:
        # FP32 Grams: both are limited by the Gram's rounding, to the same degree
        assert err_inv <= 2.0 * err_jac + 1e-9, (err_inv, err_jac)
    assert err_inv <= (1e-9 if dt == np.float64 else 1e-4), err_inv
    Va, Ua = a.V.cpu().numpy(), a.U.cpu().numpy()
    assert metrics.principal_angle_max(Va, b.V.cpu().numpy()) <= 1e-5
    assert metrics.principal_angle_max(Va, ora.V) <= 1e-4
    assert metrics.rel_rms_known(p.W, Ua, Va, ora.U, ora.V) <= 1e-5
