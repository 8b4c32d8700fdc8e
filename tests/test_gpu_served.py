"""The serving loop: continuous batching under a memory budget; each request's result is
the same alone and inside the mix."""
import numpy as np
import pytest

import synth
from oracle import metrics

pytestmark = pytest.mark.gpu


def _pool():
    from paper_1411_0814_amd import serve
    specs = [dict(m=3000, n=140, r=3, rho=0.8, seed=1), dict(m=2400, n=96, r=5, rho=0.85, seed=2),
             dict(m=4100, n=200, r=2, rho=0.7, seed=3), dict(m=1900, n=70, r=7, rho=0.9, seed=4)]
    pool = []
    for sp in specs:
        Y, W = synth.batched_device(sp)
        pool.append(serve.PoolItem(Y=Y, W=W, r=sp["r"], num_submatrices=5 * sp["n"],
                                   l=sp["r"] + 1))
    return pool


def test_served_results_equal_alone_and_budget_respected():
    import torch
    from paper_1411_0814_amd import decompose, serve
    pool = _pool()
    # a burst of requests (all arrive within ~20 ms) under a budget of three footprints, so
    # admission has to wait for memory and several batches overlap
    jobs = serve.poisson_trace(len(pool), qps=2000.0, seconds=0.02, seed=3)
    assert len(jobs) >= 20
    srv = serve.Server(pool, batching=True, max_inflight=2, keep_results=True)
    budget = 3 * max(it.footprint for it in pool)
    srv.budget = budget
    stats = srv.run(jobs)
    torch.cuda.synchronize()
    assert stats["completed"] == len(jobs)
    assert stats["peak_bytes"] <= budget
    assert stats["batches"] >= 2
    for j in jobs:
        it = pool[j.item]
        alone = decompose(it.Y, it.W, it.r, it.num_submatrices, j.seed, l=it.l)
        Va, Ua = alone.V.cpu().numpy(), alone.U.cpu().numpy()
        Vm, Um = j.result.V.cpu().numpy(), j.result.U.cpu().numpy()
        W = it.W.cpu().numpy()
        assert metrics.principal_angle_max(Vm, Va) <= 1e-4
        assert metrics.rel_rms_known(W, Um, Vm, Ua, Va) <= 1e-5
        assert j.result.info()["accepted"] == alone.info()["accepted"]
        assert j.done >= j.start >= j.arrival


def test_plain_fifo_serves_one_at_a_time():
    from paper_1411_0814_amd import serve
    pool = _pool()
    jobs = serve.poisson_trace(len(pool), qps=500.0, seconds=0.03, seed=4)
    stats = serve.Server(pool, batching=False, max_inflight=1).run(jobs)
    assert stats["completed"] == len(jobs)
    assert stats["mean_batch"] == 1.0
    starts = sorted(j.start for j in jobs)
    assert starts == [j.start for j in sorted(jobs, key=lambda j: j.arrival)]


def test_served_mix_of_column_and_row_sampling_bitwise_alone():
    """Rows-first (method M2) and column-first requests served together in deterministic
    mode: every result is bit for bit the one computed alone."""
    import torch
    from paper_1411_0814_amd import _lib, decompose, serve
    pool = _pool()
    det = _lib.DETERMINISTIC
    pool[0].flags = det | _lib.ROWS_FIRST
    pool[1].flags = det
    pool[2].flags = det | _lib.ROWS_FIRST
    pool[3].flags = det
    jobs = serve.poisson_trace(len(pool), qps=2000.0, seconds=0.02, seed=5)
    srv = serve.Server(pool, batching=True, max_inflight=2, keep_results=True)
    stats = srv.run(jobs)
    torch.cuda.synchronize()
    assert stats["completed"] == len(jobs) and stats["batches"] < len(jobs)
    assert {pool[j.item].flags for j in jobs} == {det, det | _lib.ROWS_FIRST}
    for j in jobs:
        it = pool[j.item]
        alone = decompose(it.Y, it.W, it.r, it.num_submatrices, j.seed, l=it.l,
                          flags=it.flags)
        torch.cuda.synchronize()
        assert torch.equal(alone.V, j.result.V)
        assert torch.equal(alone.U, j.result.U)


def test_sampled_results_kept_while_the_rest_is_released():
    # every request sampled, results otherwise dropped at completion (their memory goes back
    # to the streams' pools and is reused by the next batches): the kept V-hat and rows of
    # U-hat still equal the same request run alone
    import torch
    from paper_1411_0814_amd import decompose, serve
    pool = _pool()
    jobs = serve.poisson_trace(len(pool), qps=3000.0, seconds=0.03, seed=5)
    rows = [torch.arange(0, it.Y.shape[0], 7, device="cuda") for it in pool]
    sample = {j.rid: rows[j.item] for j in jobs}
    srv = serve.Server(pool, batching=True, max_inflight=3)
    srv.budget = 2 * max(it.footprint for it in pool)
    stats = srv.run(jobs, sample=sample)
    torch.cuda.synchronize()
    assert stats["completed"] == len(jobs) and stats["batches"] >= 3
    for j in jobs:
        assert j.result is None and j.kept is not None
        it = pool[j.item]
        alone = decompose(it.Y, it.W, it.r, it.num_submatrices, j.seed, l=it.l)
        Va, Ua = alone.V.cpu().numpy(), alone.U[rows[j.item]].cpu().numpy()
        Vm, Um = j.kept[0].cpu().numpy(), j.kept[1].cpu().numpy()
        Wr = it.W[rows[j.item]].cpu().numpy()
        assert metrics.principal_angle_max(Vm, Va) <= 1e-4
        assert metrics.rel_rms_known(Wr, Um, Vm, Ua, Va) <= 1e-5
