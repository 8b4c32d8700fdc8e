"""Host-side parts of the serving loop (no GPU): the admission footprint and the latency
statistics of a trace cut off before every request was served."""
import math

import torch

from paper_1411_0814_amd import Request, _lib, _problem, serve


def _item(m, n, r, I, flags=0, l=0):
    Y = torch.empty((n, m), dtype=torch.float32).T      # column-major, CPU (shape only)
    W = torch.empty((n, m), dtype=torch.bool).T
    return serve.PoolItem(Y=Y, W=W, r=r, num_submatrices=I, l=l, flags=flags)


def test_footprint_is_the_workspace_of_the_request_run_plus_factors():
    m, n, r, I = 4096, 300, 4, 1200
    for flags in (0, _lib.ROWS_FIRST, _lib.DETERMINISTIC):
        it = _item(m, n, r, I, flags=flags)
        req = Request(Y=it.Y, W=it.W, r=r, num_submatrices=I, seed=123, l=it.l, gram=it.gram,
                      flags=flags)
        expect = _lib.workspace_bytes([_problem(req)]) + 8 * r * (m + n) + 4096
        assert serve.footprint(it) == expect
    # rows-first sampling carves a row-major copy of Y and the per-trial Q_t rows besides
    # what it shares with column-first sampling: the footprint holds at least those
    plain = serve.footprint(_item(m, n, r, I))
    rows = serve.footprint(_item(m, n, r, I, flags=_lib.ROWS_FIRST))
    assert rows > plain
    assert rows >= 4 * m * n + 8 * I * n * r


def test_unserved_requests_bound_the_tail_from_below():
    # a trace whose last requests were never served: the statistics over all requests count
    # them at the stop time and say that the figures are lower bounds
    jobs = [serve.Job(rid=k, arrival=0.1 * k, item=0, seed=k) for k in range(10)]
    for j in jobs[:6]:
        j.done = j.arrival + 0.05
    lat = sorted([0.05] * 6 + [max(0.0, 1.5 - j.arrival) for j in jobs[6:]])
    stats = serve.latency_stats(jobs, t_stop=1.5)
    assert stats["completed"] == 6 and stats["unserved"] == 4
    assert math.isclose(stats["latency_ms"]["p50"], 50.0)
    assert stats["latency_all_ms"]["lower_bound"] is True
    import numpy as np
    assert math.isclose(stats["latency_all_ms"]["p99"], float(np.percentile(lat, 99)) * 1e3)
