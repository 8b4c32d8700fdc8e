"""Split-BF16 Gram on the matrix cores (hi + lo products, FP32 accumulate) against the FP64
oracle: per-trial Grams within the split-BF16 error bound, bit-exact row counts, V-hat and
U-hat within the parity tolerances."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import gram_bound_ok, to_device

pytestmark = pytest.mark.gpu

U_SPLIT = 3 * 2.0 ** -16     # unit roundoff used for the split-BF16 dot-product bound


def _run(p, gram):
    from paper_1411_0814_amd import decompose
    Y, W = to_device(p)
    res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram, taps=True)
    return res, res.info()


# (m, n, r, rho, extra trials): 8 n trials fill whole 64-trial workgroups at these n; the
# extra 37 leave a ragged last group (and the last trial is among the checked Grams)
@pytest.mark.parametrize("m,n,r,rho,extra", [(6000, 120, 4, 0.8, 0), (5003, 200, 8, 0.85, 0),
                                             (3000, 64, 15, 0.95, 0), (4001, 150, 6, 0.8, 37)])
def test_split_bf16_parity(m, n, r, rho, extra):
    p = synth.paper_synthetic(m, n, r, rho, 1e-2, 21 + r, factor_dtype=np.float32,
                              y_dtype=np.float32, relative_sigma=True,
                              num_submatrices=8 * n + extra, seed_rsm=3 + r)
    res, info = _run(p, "bf16x2")
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
    cols = res.taps["cols"].cpu().numpy()
    rows = res.taps["rows"].cpu().numpy()
    assert np.array_equal(cols, ora.subsets)
    assert np.array_equal(rows, ora.rows)
    assert info["accepted"] == ora.accepted
    G = res.taps["gram"].cpu().numpy()
    Y64 = np.asarray(p.Y, dtype=np.float64)
    worst = 0.0
    for t in np.linspace(0, len(cols) - 1, 120).astype(int):
        R = rsm.qualifying_rows(p.W, cols[t])
        Z = Y64[np.ix_(R, cols[t])]
        ok, ratio = gram_bound_ok(G[t], Z, U_SPLIT)
        assert ok, (t, ratio)
        ref = Z.T @ Z
        worst = max(worst, float(np.max(np.abs(G[t] - ref)) / np.max(np.abs(ref))))
    # the lo terms matter: a single BF16 product would be off by about 2^-9 relative
    assert worst < 2e-5, worst
    V, U = res.V.cpu().numpy(), res.U.cpu().numpy()
    theta = metrics.principal_angle_max(V, ora.V)
    rms = metrics.rel_rms_known(p.W, U, V, ora.U, ora.V)
    print(f"[bf16x2 {m}x{n} r{r}] gram rel {worst:.2e} theta {theta:.2e} rms {rms:.2e}",
          flush=True)
    assert theta <= 1e-4, theta
    assert rms <= 1e-5, rms


def test_split_bf16_close_to_fp32():
    """The same problem with the FP32 Gram and the split-BF16 Gram: same rows, close V-hat."""
    p = synth.paper_synthetic(8000, 256, 6, 0.8, 1e-2, 5, factor_dtype=np.float32,
                              y_dtype=np.float32, relative_sigma=True, num_submatrices=3000,
                              seed_rsm=8)
    rb, ib = _run(p, "bf16x2")
    rf, i_f = _run(p, "f32")
    assert ib["rows_total"] == i_f["rows_total"]
    assert ib["accepted"] == i_f["accepted"]
    assert metrics.principal_angle_max(rb.V.cpu().numpy(), rf.V.cpu().numpy()) <= 1e-4
