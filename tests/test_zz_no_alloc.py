"""rsm_decompose_noalloc (workspace from the library's own per-device scratch array) against
rsm_decompose with a caller workspace: two calls in a row, the second on a smaller problem,
each equal to the workspace path bitwise in deterministic mode and within the parity
tolerances (largest principal angle 1e-4 rad, relative RMS on known entries 1e-5)
otherwise; both also against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

# (m, n, r, rho, data seed, Y dtype): the second problem is the smaller one
SPECS = [(2000, 200, 5, 0.7, 21, np.float64), (1200, 96, 4, 0.8, 22, np.float32)]


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_matches_workspace_path_twice_shrinking():
    import torch
    from paper_1411_0814_amd import _lib, decompose, decompose_noalloc, workspace_bytes, Request
    for k, (m, n, r, rho, seed, ydt) in enumerate(SPECS):
        p = synth.paper_synthetic(m, n, r, rho, 1e-3, seed, factor_dtype=ydt, y_dtype=ydt,
                                  num_submatrices=4 * n, seed_rsm=700 + k)
        Y, W = to_device(p)
        gram = "f64" if ydt == np.float64 else "f32"
        need = workspace_bytes([Request(Y=Y, W=W, r=r, num_submatrices=p.num_submatrices,
                                        seed=p.seed_rsm, l=p.l, gram=gram)])
        assert need <= _lib.NOALLOC_MAX_BYTES, need
        print(f"[noalloc] case {k}: {m}x{n} r={r} workspace {need} bytes", flush=True)
        for flags in (_lib.DETERMINISTIC, 0):
            a = decompose(Y, W, r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram, flags=flags)
            b = decompose_noalloc(Y, W, r, p.num_submatrices, p.seed_rsm, l=p.l, gram=gram,
                                  flags=flags)
            torch.cuda.synchronize()
            Va, Ua, Vb, Ub = (t.cpu().numpy() for t in (a.V, a.U, b.V, b.U))
            ia, ib = a.info(), b.info()
            assert ia["accepted"] == ib["accepted"] and ia["warnings"] == ib["warnings"]
            if flags:
                assert _same(Va, Vb) and _same(Ua, Ub), k
                assert ia["lambda"] == ib["lambda"], k
            theta = metrics.principal_angle_max(Vb, Va)
            rms = metrics.rel_rms_known(p.W, Ub, Vb, Ua, Va)
            print(f"[noalloc] case {k} flags {flags}: theta {theta:.2e} rms {rms:.2e}", flush=True)
            assert theta <= 1e-4 and rms <= 1e-5, (k, flags, theta, rms)
        ora = rsm.rsm(p.Y, p.W, r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
        assert metrics.principal_angle_max(Vb, ora.V) <= 1e-4
        assert metrics.rel_rms_known(p.W, Ub, Vb, ora.U, ora.V) <= 1e-5


def test_noalloc_rejects_a_problem_above_the_limit():
    import torch
    from paper_1411_0814_amd import RSMError, _lib, decompose_noalloc
    # 131072 x 1024 needs about 150 MiB of workspace, above the 64 MiB scratch
    Y = torch.zeros(1024, 131072, dtype=torch.float32, device="cuda").T
    W = torch.ones(1024, 131072, dtype=torch.bool, device="cuda").T
    with pytest.raises(RSMError) as e:
        decompose_noalloc(Y, W, 8, 8192, 1, l=9)
    assert e.value.code == _lib.E_SCRATCH
