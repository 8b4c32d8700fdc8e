"""Column-subset draws for the RSM trials (oracle side; test infrastructure only).

The paper (Section III-A, method M1, and Section IV-A, step 2) picks the l columns of
every trial at random without saying how.  The reading adopted here is a uniform
l-subset of [0, n) drawn without replacement, made a pure function of (seed, trial)
so that any implementation draws the very same subsets:

* Philox4x64 with 10 rounds, the counter-based generator of Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).  Key = (seed, 0);
  counter = (block, trial, 0, 0).  The 64-bit words u_0, u_1, ... of a trial are the
  four output words of block 0, then of block 1, and so on.
* Floyd's sampling algorithm (Bentley and Floyd, "A sample of brilliance",
  CACM 30(9), 1987): for i = 0..l-1 let j = n-l+i and x = floor(u_i * (j+1) / 2^64)
  (the high word of the 128-bit product, a value in [0, j]); insert j if x is already
  in the set, else insert x.  The set is returned sorted ascending.

This module is written from those published definitions and shares nothing with the
device implementation.  It is vectorised over trials with numpy uint64 arithmetic;
the 64x64 -> 128-bit product is assembled from 32-bit halves.
"""
from __future__ import annotations

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Philox4x64 round multipliers and Weyl key increments (SC'11, Table 2 / Section 5).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
PHILOX_ROUNDS = 10


def mulhilo64(a: np.ndarray, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Full 128-bit product of uint64 arrays, returned as (high word, low word)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)  # < 3 * 2^32, no overflow
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # numpy integer arrays wrap modulo 2^64
    return hi, lo


def philox4x64_10(counter, key) -> np.ndarray:
    """Philox4x64-10 block function.

    counter: array (..., 4) of uint64; key: array (..., 2) of uint64 (broadcast).
    Returns the (..., 4) output block.  Each round multiplies words 0 and 2 by the two
    round constants and mixes the halves with words 1 and 3 and the round key; the key
    is advanced by the Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c = np.array(counter, dtype=np.uint64, copy=True)
        k = np.array(key, dtype=np.uint64, copy=True)
        c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
        k0, k1 = np.broadcast_to(k[..., 0], c0.shape).copy(), np.broadcast_to(k[..., 1], c0.shape).copy()
        for rnd in range(PHILOX_ROUNDS):
            if rnd:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = mulhilo64(PHILOX_M0, c0)
            hi1, lo1 = mulhilo64(PHILOX_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        return np.stack([c0, c1, c2, c3], axis=-1)


def trial_words(seed: int, trials: np.ndarray, count: int) -> np.ndarray:
    """The first `count` 64-bit words of each trial's stream: shape (len(trials), count)."""
    trials = np.asarray(trials, dtype=np.uint64).reshape(-1)
    nblocks = (count + 3) // 4
    key = np.array([np.uint64(seed), np.uint64(0)], dtype=np.uint64)
    words = np.empty((trials.size, nblocks * 4), dtype=np.uint64)
    for b in range(nblocks):
        ctr = np.zeros((trials.size, 4), dtype=np.uint64)
        ctr[:, 0] = np.uint64(b)
        ctr[:, 1] = trials
        words[:, 4 * b:4 * b + 4] = philox4x64_10(ctr, key)
    return words[:, :count]


def floyd_subsets(words: np.ndarray, n: int, l: int) -> np.ndarray:
    """Floyd's uniform l-subset of [0, n) for every row of `words` (T, l); sorted (T, l) int64."""
    if not (1 <= l <= n):
        raise ValueError("need 1 <= l <= n")
    words = np.asarray(words, dtype=np.uint64)
    T = words.shape[0]
    chosen = np.empty((T, l), dtype=np.int64)
    with np.errstate(over="ignore"):
        for i in range(l):
            j = n - l + i
            x, _ = mulhilo64(words[:, i], np.uint64(j + 1))
            x = x.astype(np.int64)
            seen = (chosen[:, :i] == x[:, None]).any(axis=1) if i else np.zeros(T, dtype=bool)
            chosen[:, i] = np.where(seen, j, x)
    chosen.sort(axis=1)
    return chosen


def draw_subsets(seed: int, n: int, l: int, num_trials: int, trial_begin: int = 0) -> np.ndarray:
    """Column subsets C_t for t = trial_begin .. trial_begin + num_trials - 1, shape (num_trials, l)."""
    trials = np.arange(trial_begin, trial_begin + num_trials, dtype=np.uint64)
    return floyd_subsets(trial_words(seed, trials, l), n, l)
