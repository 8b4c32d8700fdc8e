"""Batched decompositions (uneven sizes in shared launches) against the same problems run
one at a time and against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

# (m, n, r, rho, dtype, gram, row_major): several groups of the Gram / U-hat launches, two
# problems sharing every key, a ragged n, a row-major input, and columns whose byte offsets
# are not multiples of 16 (m = 3001, 1803)
SPECS = [
    (3001, 150, 3, 0.75, np.float32, "f32", False),
    (2500, 96, 5, 0.8, np.float64, "f64", False),
    (4000, 200, 2, 0.7, np.float32, "f32", True),
    (1803, 70, 8, 0.85, np.float32, "f32", False),
    (3300, 150, 3, 0.72, np.float32, "f32", False),
    (2200, 130, 12, 0.9, np.float32, "f32", False),
]


def _problems():
    out = []
    for k, (m, n, r, rho, dt, gram, rowm) in enumerate(SPECS):
        p = synth.paper_synthetic(m, n, r, rho, 1e-3, 40 + k, factor_dtype=dt, y_dtype=dt,
                                  num_submatrices=6 * n, seed_rsm=900 + k, gram=gram)
        out.append((p, rowm))
    return out


def test_batched_equals_single_and_oracle():
    import torch
    from paper_1411_0814_amd import Request, decompose, decompose_batched
    probs = _problems()
    reqs = []
    for p, rowm in probs:
        Y, W = to_device(p, row_major=rowm)
        reqs.append(Request(Y=Y, W=W, r=p.r, num_submatrices=p.num_submatrices,
                            seed=p.seed_rsm, l=p.l, gram=p.gram))
    batched = decompose_batched(reqs)
    infos_b = [res.info() for res in batched]
    torch.cuda.synchronize()
    for k, ((p, rowm), req, rb, ib) in enumerate(zip(probs, reqs, batched, infos_b)):
        single = decompose(req.Y, req.W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, gram=p.gram)
        i1 = single.info()
        # integer results are identical; floating point up to the order of accumulation
        for key in ("accepted", "rows_total", "known", "uncovered", "rows_underdetermined"):
            assert ib[key] == i1[key], (k, key)
        Vb, V1 = rb.V.cpu().numpy(), single.V.cpu().numpy()
        Ub, U1 = rb.U.cpu().numpy(), single.U.cpu().numpy()
        assert metrics.principal_angle_max(Vb, V1) < 1e-8, k
        assert metrics.rel_rms_known(p.W, Ub, Vb, U1, V1) < 1e-8, k
        assert abs(ib["lambda"][p.r - 1] - i1["lambda"][p.r - 1]) <= 1e-6 * abs(i1["lambda"][p.r - 1]) + 1e-14
        # and against the oracle
        ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
        assert ib["accepted"] == ora.accepted
        assert ib["rows_total"] == int(ora.rows.sum())
        theta = metrics.principal_angle_max(Vb, ora.V)
        rms = metrics.rel_rms_known(p.W, Ub, Vb, ora.U, ora.V)
        assert theta <= 1e-4, (k, theta)
        assert rms <= 1e-5, (k, rms)


def test_batched_mixed_modes():
    """A batch mixing an accumulate-only half, an accumulate-and-finalise half and a plain
    problem: equal to the same halves run alone.  (Against the whole run the FP32 Gram
    differs in rounding: a trial's row walk depends on its place in its workgroup, which
    trial_begin shifts.)"""
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose, decompose_batched
    p = synth.paper_synthetic(2600, 120, 4, 0.8, 1e-3, 77, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=800, seed_rsm=5)
    q = synth.paper_synthetic(2000, 90, 3, 0.75, 1e-3, 78, factor_dtype=np.float32,
                              y_dtype=np.float32, num_submatrices=500, seed_rsm=6)
    Yp, Wp = to_device(p)
    Yq, Wq = to_device(q)
    whole = decompose(Yp, Wp, p.r, 800, p.seed_rsm, l=p.l)
    Ns = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
    decompose(Yp, Wp, p.r, 400, p.seed_rsm, l=p.l, N=Ns, flags=_lib.ACCUMULATE_ONLY)
    single = decompose(Yp, Wp, p.r, 400, p.seed_rsm, l=p.l, N=Ns, trial_begin=400,
                       flags=_lib.N_ACCUMULATE)
    N = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
    first = Request(Y=Yp, W=Wp, r=p.r, num_submatrices=400, seed=p.seed_rsm, l=p.l, N=N,
                    flags=_lib.ACCUMULATE_ONLY)
    other = Request(Y=Yq, W=Wq, r=q.r, num_submatrices=500, seed=q.seed_rsm, l=q.l)
    r1 = decompose_batched([first, other])
    assert r1[0].info()["accepted"] == 400
    second = Request(Y=Yp, W=Wp, r=p.r, num_submatrices=400, seed=p.seed_rsm, l=p.l, N=N,
                     trial_begin=400, flags=_lib.N_ACCUMULATE)
    r2 = decompose_batched([second, other])
    torch.cuda.synchronize()
    assert r2[0].info()["accepted"] == 400
    assert torch.abs(N - Ns).max().item() <= 1e-12 * torch.abs(Ns).max().item()
    Vb, Vs, Vw = (x.V.cpu().numpy() for x in (r2[0], single, whole))
    assert metrics.principal_angle_max(Vb, Vs) < 1e-10
    assert metrics.principal_angle_max(Vb, Vw) < 1e-6
    ora = rsm.rsm(q.Y, q.W, q.r, 500, seed=q.seed_rsm, l=q.l, with_e=False)
    for res in (r1[1], r2[1]):
        assert metrics.principal_angle_max(res.V.cpu().numpy(), ora.V) <= 1e-4
