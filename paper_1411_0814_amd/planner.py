"""Step 1 of the algorithm (Section IV-A): how many sub-matrices to draw.

Theorem 3's bound on the trial count and Lemma 1's bracket of the binomial distribution
function are computed by the library (`rsm_lemma1_c`, `rsm_trials_bound`,
`rsm_plan_trials` in include/rsm.h, host code); this module only marshals the arguments
and turns RSM_E_ARG into ValueError.
"""
from __future__ import annotations

import ctypes as C

from . import _lib


def _call(fn, *args, out):
    code = fn(*args, C.byref(out))
    if code == _lib.E_ARG:
        raise ValueError(f"{fn.__name__}: argument out of range")
    _lib.check(code, fn.__name__)
    return out.value


def lemma1_C(n: int, rho: float, k: int) -> float:
    """C_{n,rho}(k) of Lemma 1: C(k) <= P(X <= k) <= C(k + 1) for X ~ B(n, rho)."""
    return _call(_lib.lib().rsm_lemma1_c, int(n), float(rho), int(k), out=C.c_double())


def trials_bound_rows_first(m: int, n: int, rho: float, r: int, k: int, eps: float) -> float:
    """Theorem 3 as stated (row-first sampling, k > r rows per trial)."""
    return _call(_lib.lib().rsm_trials_bound, int(m), int(n), float(rho), int(r), int(k),
                 float(eps), 1, out=C.c_double())


def trials_bound(m: int, n: int, rho: float, r: int, l: int | None = None,
                 eps: float = 0.99) -> float:
    """Theorem 3 for column-first sampling (method M1, l > r columns per trial)."""
    return _call(_lib.lib().rsm_trials_bound, int(m), int(n), float(rho), int(r),
                 int(l or 0), float(eps), 0, out=C.c_double())


def plan_trials(m: int, n: int, rho: float, r: int, l: int | None = None,
                eps: float = 0.99, rows_first: bool = False) -> int:
    """Step 1: the number of sub-matrices I to draw for visiting probability eps."""
    return _call(_lib.lib().rsm_plan_trials, int(m), int(n), float(rho), int(r), int(l or 0),
                 float(eps), 1 if rows_first else 0, out=C.c_int64())
