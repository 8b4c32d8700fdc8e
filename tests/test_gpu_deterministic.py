"""Deterministic mode: a problem's results are bitwise the same run alone, inside a batch
of other problems and inside a served mix, and stay within the parity tolerances of the
FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import metrics, rsm
from tests.gpu_util import to_device

pytestmark = pytest.mark.gpu

SPECS = [(3001, 150, 3, 0.75, 11), (2500, 96, 5, 0.8, 12), (4000, 200, 2, 0.7, 13),
         (1803, 70, 8, 0.85, 14)]


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def _problems():
    out = []
    for k, (m, n, r, rho, seed) in enumerate(SPECS):
        out.append(synth.paper_synthetic(m, n, r, rho, 1e-3, seed, factor_dtype=np.float32,
                                         y_dtype=np.float32, num_submatrices=6 * n,
                                         seed_rsm=500 + k))
    return out


def test_alone_equals_batched_bitwise():
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose, decompose_batched
    det = _lib.DETERMINISTIC | _lib.N_ACCUMULATE
    probs = _problems()
    reqs, alone = [], []
    for p in probs:
        Y, W = to_device(p)
        N1 = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
        res = decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, N=N1, flags=det)
        alone.append((res, N1))
        Nb = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
        reqs.append(Request(Y=Y, W=W, r=p.r, num_submatrices=p.num_submatrices,
                            seed=p.seed_rsm, l=p.l, N=Nb, flags=det))
    # the same problems in one batch, in reverse order, next to a non-deterministic one
    extra = probs[0]
    Ye, We = to_device(extra)
    batch = list(reversed(reqs)) + [Request(Y=Ye, W=We, r=extra.r, num_submatrices=300,
                                            seed=1, l=extra.l)]
    out = decompose_batched(batch)
    torch.cuda.synchronize()
    for k, (p, (r1, N1)) in enumerate(zip(probs, alone)):
        rb = out[len(probs) - 1 - k]
        req = reqs[k]
        assert _same(N1.cpu().numpy(), req.N.cpu().numpy()), k
        assert _same(r1.V.cpu().numpy(), rb.V.cpu().numpy()), k
        assert _same(r1.U.cpu().numpy(), rb.U.cpu().numpy()), k
        i1, ib = r1.info(), rb.info()
        assert i1["lambda"] == ib["lambda"] and i1["residual"] == ib["residual"], k
        ora = rsm.rsm(p.Y, p.W, p.r, p.num_submatrices, seed=p.seed_rsm, l=p.l, with_e=False)
        Vb, Ub = rb.V.cpu().numpy(), rb.U.cpu().numpy()
        assert metrics.principal_angle_max(Vb, ora.V) <= 1e-4, k
        assert metrics.rel_rms_known(p.W, Ub, Vb, ora.U, ora.V) <= 1e-5, k
        # fixed point 2^-40 rounds each added term: against the FP64 accumulation of the same
        # terms the difference is at most I 2^-41 plus the FP64 rounding of the other order
        Y, W = to_device(p)
        Nf = torch.zeros(p.n, p.n, dtype=torch.float64, device="cuda")
        decompose(Y, W, p.r, p.num_submatrices, p.seed_rsm, l=p.l, N=Nf, flags=_lib.N_ACCUMULATE)
        # N is column-major on the device: its lower triangle is the tensor's upper one
        Nd, Nf = np.tril(N1.cpu().numpy().T), np.tril(Nf.cpu().numpy().T)
        scale = np.max(np.abs(Nf))
        err = np.max(np.abs(Nd - Nf))
        assert err <= p.num_submatrices * 2.0 ** -41 + 1e-12 * scale, (k, err)
        assert np.max(np.abs(Nd - np.tril(ora.N))) <= 1e-4 * scale, k


def test_served_mix_equals_alone_bitwise():
    import torch
    from paper_1411_0814_amd import _lib, decompose, serve
    pool = []
    for sp in [dict(m=3000, n=140, r=3, rho=0.8, seed=1), dict(m=2400, n=96, r=5, rho=0.85, seed=2),
               dict(m=1900, n=70, r=7, rho=0.9, seed=4)]:
        Y, W = synth.batched_device(sp)
        pool.append(serve.PoolItem(Y=Y, W=W, r=sp["r"], num_submatrices=5 * sp["n"],
                                   l=sp["r"] + 1, flags=_lib.DETERMINISTIC))
    jobs = serve.poisson_trace(len(pool), qps=2000.0, seconds=0.015, seed=9)
    assert len(jobs) >= 10
    srv = serve.Server(pool, batching=True, max_inflight=2, keep_results=True)
    stats = srv.run(jobs)
    torch.cuda.synchronize()
    assert stats["completed"] == len(jobs)
    assert stats["mean_batch"] > 1.0
    for j in jobs:
        it = pool[j.item]
        a = decompose(it.Y, it.W, it.r, it.num_submatrices, j.seed, l=it.l, flags=it.flags)
        assert _same(a.V.cpu().numpy(), j.result.V.cpu().numpy()), j.rid
        assert _same(a.U.cpu().numpy(), j.result.U.cpu().numpy()), j.rid


def test_large_batch_on_side_by_side_lanes_equals_alone_bitwise():
    """A call of 72 problems runs each step's launch groups (one per l for the Gram and
    minor steps, one per r for U-hat) side by side on several streams, joined back into
    the caller's stream before the next step: every problem's N, V-hat and U-hat are still
    bitwise those of the problem run alone."""
    import torch
    from paper_1411_0814_amd import Request, _lib, decompose, decompose_batched
    det = _lib.DETERMINISTIC | _lib.N_ACCUMULATE
    ranks = [2, 3, 5, 6, 8, 9]
    reqs, alone = [], []
    for k in range(72):
        r = ranks[k % len(ranks)]
        m, n = 900 + 37 * k, 40 + (k % 5) * 6
        p = synth.paper_synthetic(m, n, r, 0.85, 1e-3, 900 + k, factor_dtype=np.float32,
                                  y_dtype=np.float32, num_submatrices=4 * n, seed_rsm=k)
        Y, W = to_device(p)
        N1 = torch.zeros(n, n, dtype=torch.float64, device="cuda")
        alone.append((decompose(Y, W, r, p.num_submatrices, p.seed_rsm, l=p.l, N=N1,
                                flags=det), N1))
        reqs.append(Request(Y=Y, W=W, r=r, num_submatrices=p.num_submatrices,
                            seed=p.seed_rsm, l=p.l, flags=det,
                            N=torch.zeros(n, n, dtype=torch.float64, device="cuda")))
    out = decompose_batched(reqs)
    torch.cuda.synchronize()
    for k, ((r1, N1), rb, q) in enumerate(zip(alone, out, reqs)):
        assert _same(N1.cpu().numpy(), q.N.cpu().numpy()), k
        assert _same(r1.V.cpu().numpy(), rb.V.cpu().numpy()), k
        assert _same(r1.U.cpu().numpy(), rb.U.cpu().numpy()), k
    # the same call with its launch groups in order on the caller's stream
    from dataclasses import replace
    reqs_s = [replace(q, N=torch.zeros_like(q.N)) for q in reqs]
    reqs_s[5] = replace(reqs_s[5], flags=det | _lib.SERIAL_STEPS)
    out_s = decompose_batched(reqs_s)
    torch.cuda.synchronize()
    for k, ((r1, N1), rs, q) in enumerate(zip(alone, out_s, reqs_s)):
        assert _same(N1.cpu().numpy(), q.N.cpu().numpy()), k
        assert _same(r1.U.cpu().numpy(), rs.U.cpu().numpy()), k
