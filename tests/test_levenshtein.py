"""Pins of the ground-truth edit distance (the textbook Levenshtein recurrence)."""
import functools
import itertools

import numpy as np
import pytest

import oracle


def _recursive(a, b):
    # Levenshtein's definition, by exhaustive recursion (tiny inputs only)
    @functools.lru_cache(maxsize=None)
    def d(i, j):
        if i == 0:
            return j
        if j == 0:
            return i
        return min(d(i - 1, j) + 1, d(i, j - 1) + 1, d(i - 1, j - 1) + (a[i - 1] != b[j - 1]))
    return d(len(a), len(b))


@pytest.mark.parametrize("a,b,expect", [
    ("", "", 0), ("", "ACGT", 4), ("ACGT", "ACGT", 0), ("ACGT", "AGT", 1),
    ("ACGT", "TGCA", 4), ("GATTACA", "GCATGCT", 4), ("AAAA", "TTTT", 4), ("ACAC", "CACA", 2),
])
def test_known_values(a, b, expect):
    assert oracle.edit_distance(a, b) == expect


def test_exhaustive_small_vs_recursion():
    seqs = ["".join(s) for n in range(0, 4) for s in itertools.product("ACGT", repeat=n)]
    for a in seqs[::3]:
        for b in seqs:
            assert oracle.edit_distance(a, b) == _recursive(a, b)


def test_banded_matches_full_and_metric_axioms():
    rng = np.random.default_rng(1)
    for _ in range(300):
        n = int(rng.integers(1, 30))
        a = rng.integers(0, 4, n).astype(np.uint8)
        b = a.copy()
        for _ in range(int(rng.integers(0, 6))):
            b[rng.integers(0, n)] = rng.integers(0, 4)
        b = np.roll(b, int(rng.integers(-2, 3)))
        c = rng.integers(0, 4, n).astype(np.uint8)
        dab = oracle.edit_distance(a, b)
        assert dab == oracle.edit_distance(b, a)
        assert oracle.edit_distance(a, c) <= dab + oracle.edit_distance(b, c)
        for k in (0, 1, 2, 4, 8, 40):
            got = oracle.edit_distance_banded(a, b, k)
            assert got == (dab if dab <= k else -1)
