"""The tile table and its autotuner: every tiled-Gram shape the table can select gives
per-trial Grams within the dot-product error bound and exact row counts, and the
autotuned batch still matches the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import gram_bound_ok, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _empty_table():
    from paper_1411_0814_amd import _lib
    _lib.tune_set([])
    yield
    _lib.tune_set([])


REGS, DMA, DMA2, GATHER, AUTO = 1, 2, 3, 4, 5
# (l, Y/Gram type, trials per workgroup, workgroup target, staging): both staging kernels,
# both thread counts, a single row split and many row splits
CASES = [(3, "f32", 256, 1, REGS), (6, "f32", 256, 8192, REGS), (9, "f32", 512, 8192, REGS),
         (10, "f32", 256, 64, REGS), (12, "f32", 256, 4096, REGS), (4, "f64", 256, 2048, REGS),
         (6, "f64", 512, 1, REGS), (3, "f32", 512, 1, DMA), (9, "f32", 256, 8192, DMA),
         (13, "f32", 512, 64, DMA), (17, "f32", 256, 4096, DMA), (17, "f32", 512, 1, DMA),
         (3, "f32", 1024, 1, DMA2), (9, "f32", 1024, 8192, DMA2), (12, "f32", 512, 64, DMA2),
         (17, "f32", 512, 4096, DMA2),
         # "f64/f32": FP64 sums of FP32 data
         (4, "f64/f32", 512, 1, DMA2), (14, "f64/f32", 512, 4096, DMA2),
         (17, "f64/f32", 256, 64, DMA2),
         # gathering the qualifying values (forced), and the per-problem choice
         (3, "f32", 1024, 1, GATHER), (12, "f32", 512, 4096, GATHER), (17, "f32", 512, 64, GATHER),
         (5, "f64/f32", 512, 8192, GATHER), (16, "f64/f32", 256, 1, GATHER),
         (9, "f32", 1024, 2048, AUTO), (15, "f64/f32", 256, 2048, AUTO),
         (4, "f64", 256, 2048, GATHER), (6, "f64", 512, 1, AUTO), (11, "f64", 256, 64, GATHER)]


@pytest.mark.parametrize("l,prec,threads,wgs,kernel", CASES)
def test_tuned_gram_shapes_exact_rows_and_bounded_gram(l, prec, threads, wgs, kernel):
    from paper_1411_0814_amd import _lib, decompose
    dt = np.float64 if prec == "f64" else np.float32
    gram = prec.split("/")[0]
    r = l - 1
    p = synth.paper_synthetic(5003, 160, r, 0.9, 1e-3, 60 + l, factor_dtype=dt, y_dtype=dt,
                              num_submatrices=700, seed_rsm=l, gram=gram)
    _lib.tune_set([{"l": l, "gram_prec": _lib.GRAM_MODES[gram],
                    "y_dtype": _lib.F64 if prec == "f64" else _lib.F32, "batched": 0,
                    "gram_threads": threads, "gram_wgs": wgs, "gram_kernel": kernel}])
    Y, W = to_device(p)
    res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=l, gram=gram, taps=True)
    cols = res.taps["cols"].cpu().numpy()
    rows = res.taps["rows"].cpu().numpy()
    G = res.taps["gram"].cpu().numpy()
    ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=l, with_e=False)
    assert np.array_equal(cols, ora.subsets)
    assert np.array_equal(rows, ora.rows)
    u = 2.0 ** -24 if gram == "f32" else 2.0 ** -53
    Y64 = np.asarray(p.Y, dtype=np.float64)
    for t in np.linspace(0, len(cols) - 1, 60).astype(int):
        R = rsm.qualifying_rows(p.W, cols[t])
        ok, ratio = gram_bound_ok(G[t], Y64[np.ix_(R, cols[t])], u)
        assert ok, (t, ratio)
    assert metrics.principal_angle_max(res.V.cpu().numpy(), ora.V) <= 1e-4


def test_autotune_installs_a_table_and_keeps_parity():
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose_batched, tune
    specs = [(4000, 150, 3, 0.8, 1), (3500, 120, 3, 0.75, 2), (3000, 200, 8, 0.9, 3)]
    probs, reqs = [], []
    for m, n, r, rho, seed in specs:
        p = synth.paper_synthetic(m, n, r, rho, 1e-3, seed, factor_dtype=np.float32,
                                  y_dtype=np.float32, num_submatrices=6 * n, seed_rsm=seed)
        Y, W = to_device(p)
        probs.append(p)
        reqs.append(Request(Y=Y, W=W, r=p.r, num_submatrices=p.num_submatrices,
                            seed=p.seed_rsm, l=p.l, gram="f32"))
    out = tune.autotune(reqs, wgs=(64, 1024), reps=1)
    keys = {(g["l"], g["batched"]) for g in out["groups"]}
    assert keys == {(4, 1), (9, 0)}
    assert tune.table() == out["entries"]
    for g in out["groups"]:
        assert g["best_ms"] <= g["builtin_ms"]
    res = decompose_batched(reqs)
    torch.cuda.synchronize()
    for p, rb in zip(probs, res):
        ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
        V, U = rb.V.cpu().numpy(), rb.U.cpu().numpy()
        assert metrics.principal_angle_max(V, ora.V) <= 1e-4
        assert metrics.rel_rms_known(p.W, U, V, ora.U, ora.V) <= 1e-5
    # the autotuner ran its candidates with scratch N: the inputs' requests are untouched
    assert all(q.N is None and not q.flags for q in reqs)


def test_library_loaded_first_still_uses_torchs_runtime():
    """A fresh process whose first library call precedes any torch use (here: the tile
    table) still runs decompositions on torch's streams."""
    import os
    import subprocess
    import sys
    code = (
        "import numpy as np\n"
        "from paper_1411_0814_amd import _lib\n"
        "_lib.tune_set([])\n"
        "import torch, synth\n"
        "from tests.gpu_util import to_device\n"
        "from paper_1411_0814_amd import decompose\n"
        "p = synth.paper_synthetic(3000, 100, 3, 0.85, 1e-3, 5, factor_dtype=np.float32,\n"
        "                          y_dtype=np.float32, num_submatrices=400, seed_rsm=2, gram='f32')\n"
        "Y, W = to_device(p)\n"
        "res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, gram='f32')\n"
        "print('accepted', res.info()['accepted'])\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.startswith("accepted"), out.stdout
