"""Entries of Y where W is 0 are unknown: every sum of the method (the Grams of the trials,
N, the normal equations of U-hat and the error of eq.(ep)) runs over known entries only, so
NaN stored there must leave every result bit for bit as it is with zeros there.  Also: the
U-hat rows of a problem do not depend on what other work, running at the same time on
other streams, left in the compute units' local memory (the U-hat solve once read a few
LDS slots past the last staged column, scaled by a zero weight: NaN left there by other
kernels zeroed whole blocks of rows)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _inputs(m, n, r, rho, seed):
    import torch
    Y, W = synth.batched_device(dict(m=m, n=n, r=r, rho=rho, seed=seed))
    # column-major (m, n) views, as synth returns them
    Y0 = torch.where(W.T, Y.T, torch.zeros((), device=Y.device)).contiguous().T
    Ynan = torch.where(W.T, Y.T, torch.full((), float("nan"), device=Y.device)).contiguous().T
    return Y0, Ynan, W


@pytest.mark.parametrize("gram,extra", [("f32", ""), ("f64", ""), ("bf16x2", ""),
                                        ("f32", "plain"), ("f64", "rows_first")])
def test_nan_at_unknown_entries_changes_nothing(gram, extra):
    import torch
    from paper_1411_0814_amd import _lib, decompose
    m, n, r = 3001, 151, 3            # n not a multiple of any column group
    Y0, Ynan, W = _inputs(m, n, r, 0.8, seed=21)
    rows_first = extra == "rows_first"
    flags = _lib.DETERMINISTIC | _lib.COMPUTE_ERROR | {
        "": 0, "plain": _lib.PLAIN_GRAM, "rows_first": _lib.ROWS_FIRST}[extra]
    trials = 600 if rows_first else 4 * n
    out = []
    for Y in (Y0, Ynan):
        res = decompose(Y, W, r, trials, 5, l=r + 1, gram=gram, flags=flags)
        out.append((res.V.cpu(), res.U.cpu(), res.info()))
    torch.cuda.synchronize()
    (V0, U0, i0), (V1, U1, i1) = out
    print(f"[unknown nan] {gram} {extra}: e {i0['e']:.3e} / {i1['e']:.3e} "
          f"warnings {i0['warnings']} / {i1['warnings']}", flush=True)
    assert torch.isfinite(V1).all() and torch.isfinite(U1).all()
    assert torch.equal(V0, V1) and torch.equal(U0, U1)
    assert i0["e"] == i1["e"] and np.isfinite(i1["e"])
    assert i0["warnings"] == i1["warnings"]
    assert i1["rows_underdetermined"] == 0


def test_u_rows_do_not_depend_on_other_streams_work():
    # stream B keeps the Gram stage busy on inputs whose unknown entries are NaN (its staging
    # leaves NaN all over the local memory of the compute units it ran on) while stream A
    # solves problems whose column count leaves a partial group of columns in the U-hat
    # solve; A's deterministic results must equal the same calls made alone, bit for bit
    import torch
    from paper_1411_0814_amd import _lib, decompose
    small = [(20011, 151, 3, 31), (20011, 161, 5, 32), (9001, 97, 2, 33), (9001, 250, 7, 34)]
    probs = []
    for m, n, r, seed in small:
        Y0, _, W = _inputs(m, n, r, 0.8, seed)
        probs.append((Y0, W, r, 3 * n))
    flags = _lib.DETERMINISTIC
    alone = []
    for Y, W, r, I in probs:
        res = decompose(Y, W, r, I, 7, l=r + 1, flags=flags)
        alone.append(res.U.cpu())
    torch.cuda.synchronize()
    _, Ynan, Wb = _inputs(30011, 600, 6, 0.7, seed=35)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    keep = []
    for rep in range(6):
        with torch.cuda.stream(sb):
            for _ in range(3):
                keep.append(decompose(Ynan, Wb, 6, 1200, rep, l=7, gram="f32", stream=sb))
        with torch.cuda.stream(sa):
            for k, (Y, W, r, I) in enumerate(probs):
                keep.append((k, decompose(Y, W, r, I, 7, l=r + 1, flags=flags, stream=sa)))
    torch.cuda.synchronize()
    bad = []
    for item in keep:
        if isinstance(item, tuple):
            k, res = item
            if not torch.equal(res.U.cpu(), alone[k]) or res.info()["rows_underdetermined"]:
                bad.append((k, res.info()["rows_underdetermined"]))
        else:
            assert torch.isfinite(item.V).all()
    assert not bad, bad
