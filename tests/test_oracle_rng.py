"""Pins of the oracle's subset generator (Philox4x64-10 + Floyd)."""
import itertools
import math

import numpy as np
import pytest

from oracle import rng


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((0, 7, 0, 0), (5, 0)),
    ((3, 123456789, 0, 0), (0xDEADBEEFCAFEF00D, 0)),
    ((2**64 - 2, 2**63 + 5, 17, 2**64 - 1), (2**64 - 1, 2**64 - 1)),
])
def test_philox_known_answer_vs_numpy(counter, key):
    # numpy's Philox bit generator is Philox4x64-10 and advances its 256-bit counter by
    # one *before* producing a block, so block(counter + 1) == numpy(counter).random_raw(4).
    c = list(counter)
    ref = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                           key=np.array(key, dtype=np.uint64)).random_raw(4)
    c1 = np.array(c, dtype=object)
    # add one to the 256-bit little-endian counter
    carry = 1
    out = []
    for w in c1:
        s = int(w) + carry
        out.append(s & (2**64 - 1))
        carry = s >> 64
    got = rng.philox4x64_10(np.array(out, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert [int(x) for x in got] == [int(x) for x in ref]


def test_mulhilo_matches_python_ints():
    g = np.random.default_rng(0)
    a = g.integers(0, 2**64 - 1, size=1000, dtype=np.uint64, endpoint=True)
    b = g.integers(0, 2**64 - 1, size=1000, dtype=np.uint64, endpoint=True)
    a[:4] = [0, 1, 2**64 - 1, 2**63]
    b[:4] = [2**64 - 1, 2**64 - 1, 2**64 - 1, 2]
    hi, lo = rng.mulhilo64(a, b)
    for x, y, h, l_ in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l_) == p & (2**64 - 1)


def test_trial_words_are_the_block_stream():
    w = rng.trial_words(42, np.array([9]), 10)[0]
    blocks = [rng.philox4x64_10(np.array([b, 9, 0, 0], dtype=np.uint64),
                                np.array([42, 0], dtype=np.uint64)) for b in range(3)]
    flat = np.concatenate(blocks)[:10]
    assert np.array_equal(w, flat)


@pytest.mark.parametrize("n,l", [(10, 1), (10, 10), (200, 6), (1024, 9), (37, 17)])
def test_floyd_subsets_valid(n, l):
    S = rng.draw_subsets(7, n, l, 2000)
    assert S.shape == (2000, l)
    assert S.min() >= 0 and S.max() < n
    assert np.all(np.diff(S, axis=1) > 0)          # sorted and distinct


def test_floyd_uniform_chi_square():
    n, l, draws = 8, 3, 100_000
    S = rng.draw_subsets(11, n, l, draws)
    subsets = list(itertools.combinations(range(n), l))
    index = {s: k for k, s in enumerate(subsets)}
    counts = np.zeros(len(subsets))
    for row in map(tuple, S):
        counts[index[row]] += 1
    expected = draws / len(subsets)
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    dof = len(subsets) - 1
    # 55 degrees of freedom: P(chi2 > 100) ~ 2e-4
    assert chi2 < 100.0, chi2
    # and not suspiciously perfect
    assert chi2 > 20.0, chi2
    # every element equally likely to be chosen
    per_elem = np.bincount(S.ravel(), minlength=n) / (draws * l / n)
    assert np.all(np.abs(per_elem - 1.0) < 0.02)
    assert math.comb(n, l) == len(subsets) == dof + 1


def test_floyd_small_cases_exhaustive():
    # x = floor(u * (j+1) / 2^64) with u spanning the range must hit every value 0..j,
    # and Floyd must then reach every l-subset: enumerate with hand-built words.
    n, l = 5, 2
    reached = set()
    grid = [0, 2**62, 2**63, 3 * 2**62, 2**64 - 1]
    for u0 in grid:
        for u1 in grid:
            words = np.array([[u0, u1]], dtype=np.uint64)
            reached.add(tuple(rng.floyd_subsets(words, n, l)[0]))
    assert reached == set(itertools.combinations(range(n), l))


def test_subsets_depend_only_on_seed_and_trial():
    a = rng.draw_subsets(3, 300, 7, 50, trial_begin=0)
    b = rng.draw_subsets(3, 300, 7, 30, trial_begin=20)
    assert np.array_equal(a[20:], b)
    c = rng.draw_subsets(4, 300, 7, 50)
    assert not np.array_equal(a, c)
