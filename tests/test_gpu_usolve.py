"""Step a7 (U-hat, eq.(solve.barU)) on its own: given the V-hat the GPU found, every row's
least-squares solution equals the oracle's row-by-row solve with that same V-hat, for
ranks on both ways of forming the normal equations (one thread per row, and the FP64
matrix-core product), ragged m and n, FP32 and FP64 Y, rows with too few known entries."""
import numpy as np
import pytest

import synth
from oracle import rsm
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

# (m, n, r, rho, dtype): m not a multiple of the 128- or 256-row workgroup, n not a multiple of the
# 16-column stage; every 7th row is thinned to r - 2 known entries (underdetermined)
CASES = [(3001, 203, 2, 0.7, np.float32), (2999, 150, 5, 0.8, np.float64),
         (3001, 203, 6, 0.8, np.float32), (4097, 97, 8, 0.75, np.float32),
         (3001, 99, 9, 0.8, np.float64), (3001, 130, 12, 0.85, np.float64),
         (2500, 75, 13, 0.9, np.float64), (1500, 50, 14, 0.95, np.float32),
         (2001, 61, 16, 0.95, np.float32), (1000, 40, 16, 0.97, np.float64)]


@pytest.mark.parametrize("m,n,r,rho,dt", CASES)
def test_u_rows_equal_oracle_solve_with_gpu_v(m, n, r, rho, dt):
    from paper_1411_0814_amd import decompose
    gram = "f32" if dt == np.float32 else "f64"
    p = synth.paper_synthetic(m, n, r, rho, 1e-3, 100 + r, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=max(8 * n, 600), seed_rsm=r, gram=gram)
    for i in range(3, m, 7):
        on = np.flatnonzero(p.Wt[:, i])
        p.Wt[on[max(r - 2, 0):], i] = 0
    Y, W = to_device(p)
    res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, gram=gram)
    info = res.info()
    V = res.V.cpu().numpy()
    U = res.U.cpu().numpy()
    Uref, under = rsm.solve_U(p.Y, p.W, V)
    assert info["rows_underdetermined"] == under
    known = int(np.asarray(p.W, dtype=bool).sum())
    assert info["known"] == known
    few = np.asarray(p.W, dtype=bool).sum(axis=1) < r
    assert np.all(U[few] == 0.0)
    scale = np.max(np.abs(Uref))
    err = np.max(np.abs(U - Uref)) / scale
    # both sides solve the same r x r systems in FP64; cond(A_i) of random masks is modest
    assert err <= 1e-9, err
