"""Step 1 of the algorithm (Section IV-A): how many sub-matrices to draw.

Theorem 3 bounds the number of trials I after which every known entry of Y has been in
some sub-matrix with probability at least eps, using Lemma 1's normal-approximation bounds
C_{n,rho}(k) on the binomial distribution function.  The theorem is stated for row-first
sampling (k rows, the columns known on all of them: about n rho^k columns); for column-first
sampling (method M1: l columns, the rows known on all of them: about m rho^l rows) the same
argument applies to Y^T, i.e. with m and n exchanged and l in place of k.

Host-side scalar code: no device work.
"""
from __future__ import annotations

import math


def _kl(x: float, rho: float) -> float:
    """phi(x, rho) of Lemma 1: the Kullback-Leibler divergence of Bernoulli(x) from
    Bernoulli(rho)."""
    a = 0.0 if x <= 0.0 else x * math.log(x / rho)
    b = 0.0 if x >= 1.0 else (1.0 - x) * math.log((1.0 - x) / (1.0 - rho))
    return a + b


def lemma1_C(n: int, rho: float, k: int) -> float:
    """C_{n,rho}(k) of Lemma 1: (1 - rho)^n at k = 0, 1 - rho^n at k = n, otherwise the
    standard normal distribution function at sgn(k/n - rho) sqrt(2 n phi(k/n, rho)).
    For a binomial X ~ B(n, rho) it brackets the distribution function:
    C(k) <= P(X <= k) <= C(k + 1)."""
    if not (0.0 < rho < 1.0) or n < 1 or k < 0 or k > n:
        raise ValueError("need 0 < rho < 1, n >= 1, 0 <= k <= n")
    if k == 0:
        return (1.0 - rho) ** n
    if k == n:
        return 1.0 - rho ** n
    x = k / n
    z = math.copysign(1.0, x - rho) * math.sqrt(2.0 * n * _kl(x, rho))
    return 0.5 * math.erfc(-z / math.sqrt(2.0))


def trials_bound_rows_first(m: int, n: int, rho: float, r: int, k: int, eps: float) -> float:
    """Theorem 3 as stated (row-first sampling, k > r rows per trial): at most
    m n rho / (k (r + 1) (1 - C_{n, rho^k}(r + 2))) ln(1 / (1 - eps)) trials make every
    known entry visited with probability >= eps."""
    if k <= r or not (0.0 < eps < 1.0):
        raise ValueError("need k > r and 0 < eps < 1")
    if r + 2 > n:
        raise ValueError("need r + 2 <= n")
    p = rho ** k
    tail = 1.0 - lemma1_C(n, p, r + 2)
    if tail <= 0.0:
        return math.inf
    return m * n * rho / (k * (r + 1) * tail) * math.log(1.0 / (1.0 - eps))


def trials_bound(m: int, n: int, rho: float, r: int, l: int | None = None,
                 eps: float = 0.99) -> float:
    """Theorem 3 for column-first sampling (method M1, l > r columns per trial): the bound
    of the rows-first form applied to Y^T."""
    l = r + 1 if l is None else l
    return trials_bound_rows_first(n, m, rho, r, l, eps)


def plan_trials(m: int, n: int, rho: float, r: int, l: int | None = None,
                eps: float = 0.99) -> int:
    """Step 1: the number of sub-matrices I to draw for visiting probability eps (the
    bound of Theorem 3, rounded up)."""
    b = trials_bound(m, n, rho, r, l, eps)
    if not math.isfinite(b):
        raise ValueError("no sub-matrix with more than r rows is likely at this density")
    return int(math.ceil(b))
