"""Pins of the oracle's window-width variant (Suppl. Sec. 6.1, Fig. 4 compares
window widths): W = 4 is the filter itself, W = 1 has a closed form, E = 0
gives the Hamming distance, and an independent matrix implementation agrees
on every small case."""
import itertools

import numpy as np
import pytest

import oracle


def test_width4_is_the_filter():
    rng = np.random.default_rng(11)
    for _ in range(400):
        m = int(rng.integers(0, 60))
        E = int(rng.integers(0, 8))
        P = rng.integers(0, 4, m).astype(np.uint8)
        T = P.copy()
        T[rng.random(m) < 0.15] = rng.integers(0, 4)
        assert oracle.shouji_pair_w(P, T, E, 4) == oracle.shouji_pair(P, T, E)


def test_width1_closed_form():
    # one column per window: S[i] = 0 iff some diagonal |d| <= E matches at
    # column i, i.e. T[i] occurs in P[i-E .. i+E]
    rng = np.random.default_rng(12)
    for _ in range(400):
        m = int(rng.integers(0, 50))
        E = int(rng.integers(0, 6))
        P = rng.integers(0, 4, m).astype(np.uint8)
        T = rng.integers(0, 4, m).astype(np.uint8)
        want = sum(1 for i in range(m) if not any(P[q] == T[i] for q in range(max(0, i - E), min(m, i + E + 1))))
        c, S = oracle.shouji_pair_w(P, T, E, 1)
        assert c == want


@pytest.mark.parametrize("W", [1, 2, 3, 5, 6, 8, 12])
def test_E0_is_hamming(W):
    rng = np.random.default_rng(13 + W)
    for _ in range(300):
        m = int(rng.integers(0, 40))
        P = rng.integers(0, 4, m).astype(np.uint8)
        T = rng.integers(0, 4, m).astype(np.uint8)
        assert oracle.shouji_pair_w(P, T, 0, W)[0] == int((P != T).sum())


def _matrix_w(Pseq, Tseq, E, W):
    """Independent version over the explicit m x m map (rows pattern, columns
    text, Eq. 1) with W-column windows and Algorithm 1's order (text index -
    pattern index = +j before -j, main last)."""
    m = len(Tseq)

    def cell(r, c):
        if 0 <= r < m and 0 <= c < m and abs(c - r) <= E:
            return 0 if Pseq[r] == Tseq[c] else 1
        return 1

    order = [x for j in range(1, E + 1) for x in (j, -j)] + [0]
    S = [1] * (m + W)
    for w in range(m):
        best, bkey = None, None
        for k in order:
            seg = [cell(c - k, c) for c in range(w, w + W)]
            key = (seg.count(0), seg[0] == 0)
            if bkey is None or key > bkey:
                best, bkey = seg, key
        if best.count(0) > S[w:w + W].count(0):
            S[w:w + W] = best
    return sum(S[:m])


@pytest.mark.parametrize("W", [1, 2, 3, 5, 6])
def test_exhaustive_tiny_vs_matrix(W):
    seqs = [s for n in (3, 4) for s in itertools.product(range(3), repeat=n)]
    for E in range(0, 5):
        for a in seqs:
            for b in seqs:
                if len(a) != len(b):
                    continue
                got = oracle.shouji_pair_w(np.array(a, np.uint8), np.array(b, np.uint8), E, W)[0]
                assert got == _matrix_w(a, b, E, W), (a, b, E, W)


def test_random_vs_matrix():
    rng = np.random.default_rng(14)
    for _ in range(300):
        m = int(rng.integers(1, 16))
        E = int(rng.integers(0, 5))
        W = int(rng.integers(1, 9))
        a = tuple(int(x) for x in rng.integers(0, 2, m))
        b = tuple(int(x) for x in rng.integers(0, 2, m))
        got = oracle.shouji_pair_w(np.array(a, np.uint8), np.array(b, np.uint8), E, W)[0]
        assert got == _matrix_w(a, b, E, W), (a, b, E, W)


def test_batch_w_matches_pairwise():
    rng = np.random.default_rng(15)
    n, stride = 200, 40
    P = rng.integers(0, 4, (n, stride)).astype(np.uint8)
    T = P.copy()
    T[rng.random((n, stride)) < 0.1] = 1
    L = rng.integers(0, stride + 1, n).astype(np.int32)
    L[::17] = stride + 1
    for W in (2, 4, 7):
        acc, pc = oracle.shouji_batch_w(P, T, L, 3, W)
        for p in range(n):
            if L[p] > stride:
                assert acc[p] == 0xFF and pc[p] == -1
                continue
            c, _ = oracle.shouji_pair_w(P[p, :L[p]], T[p, :L[p]], 3, W)
            assert pc[p] == c and acc[p] == (1 if c <= 3 else 0)


def test_width2_equals_width1():
    # With 2-column windows a zero of S is never overwritten (a copy into
    # S[i..i+1] needs more zeros than S holds there, and S[i+1] is still 1),
    # and window i picks a segment with a zero at column i whenever one exists
    # (most zeros first, then a leading zero).  So S[i] = 0 exactly when some
    # diagonal matches at column i: the W = 1 vector, for every input.
    rng = np.random.default_rng(16)
    for _ in range(500):
        m = int(rng.integers(0, 50))
        E = int(rng.integers(0, 7))
        P = rng.integers(0, 4, m).astype(np.uint8)
        T = P.copy()
        T[rng.random(m) < 0.3] = rng.integers(0, 4)
        c1, S1 = oracle.shouji_pair_w(P, T, E, 1)
        c2, S2 = oracle.shouji_pair_w(P, T, E, 2)
        assert c1 == c2 and S1 == S2
