"""Pins of the oracle's local / glocal counting and of pairs with different
read and reference lengths (Sec. 2.2.3; Suppl. Sec. 8, Fig. 6(c)).

Local filtering ignores the runs of ones before the first zero and after the
last zero of the Shouji bit-vector; glocal filtering ignores one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
from golden_io import read_sections

GLOBAL, LOCAL, GSTART, GEND = oracle.GLOBAL, oracle.LOCAL, oracle.GLOCAL_START, oracle.GLOCAL_END


def test_fig6c_local_count_is_two():
    g = read_sections("fig6c_local.txt")[""]
    E = int(g["E"])
    assert len(g["read"]) == 68 and len(g["reference"]) == 100
    count, S = oracle.shouji_pair2(g["read"], g["reference"], E, LOCAL)
    assert count == int(g["local_edits"])
    # the read covers reference positions 4..71: past its end every cell is
    # a mismatch, so the vector ends in a run of ones from position 72 on
    assert S[72:] == "1" * 28
    # the printed (character-dropping) vector also ends in its longest run of ones
    assert g["shouji"].rstrip("1").endswith("0") and len(g["shouji"]) - len(g["shouji"].rstrip("1")) >= 28
    # the global count of the same vector includes that run
    gcount, _ = oracle.shouji_pair2(g["read"], g["reference"], E, GLOBAL)
    assert gcount == S.count("1") and gcount >= 28


def _runs(S):
    z = [j for j, b in enumerate(S) if b == "0"]
    if not z:
        return 0, 0
    return z[0], len(S) - 1 - z[-1]


def test_modes_remove_exactly_the_end_runs():
    rng = np.random.default_rng(5)
    for _ in range(300):
        mT = int(rng.integers(0, 60))
        mP = int(rng.integers(0, 60))
        E = int(rng.integers(0, 8))
        P = rng.integers(0, 4, mP).astype(np.uint8)
        T = rng.integers(0, 4, mT).astype(np.uint8)
        g, S = oracle.shouji_pair2(P, T, E, GLOBAL)
        lead, trail = _runs(S)
        assert g == S.count("1")
        assert oracle.shouji_pair2(P, T, E, LOCAL)[0] == g - lead - trail
        assert oracle.shouji_pair2(P, T, E, GSTART)[0] == g - lead
        assert oracle.shouji_pair2(P, T, E, GEND)[0] == g - trail


def test_equal_lengths_global_is_the_plain_filter():
    # Fig. 6(c) pins the diagonal order, the tie rule and the strict update of
    # the two-length form (its stated local count of 2 comes out only with
    # them).  With equal lengths and global counting the plain filter must be
    # the same function, so that pin holds for the plain filter too: compare
    # every vector, on pairs built to reach order-sensitive ties (a two-letter
    # alphabet, tandem repeats, insertions and deletions).
    rng = np.random.default_rng(6)
    for m in (1, 4, 17, 100):
        for E in (0, 2, 5):
            P = rng.integers(0, 4, m).astype(np.uint8)
            T = P.copy()
            T[rng.integers(0, m, 3)] = rng.integers(0, 4, 3)
            assert oracle.shouji_pair2(P, T, E, GLOBAL) == oracle.shouji_pair(P, T, E)
    n, m = 4000, 60
    P = np.zeros((n, m), np.uint8)
    T = np.zeros((n, m), np.uint8)
    for k in range(n):
        alpha = 2 if k % 2 else 4
        unit = rng.integers(0, alpha, int(rng.integers(1, 4)))
        a = np.resize(unit, m) if k % 3 == 0 else rng.integers(0, alpha, m)
        b = list(a)
        for _ in range(int(rng.integers(0, 6))):
            op, pos = int(rng.integers(0, 3)), int(rng.integers(0, len(b) + 1))
            if op == 0 and pos < len(b):
                b[pos] = int(rng.integers(0, alpha))
            elif op == 1:
                b.insert(pos, int(rng.integers(0, alpha)))
            elif pos < len(b):
                del b[pos]
        b = (b + list(rng.integers(0, alpha, m)))[:m]
        P[k], T[k] = a, b
    L = np.full(n, m, np.int32)
    for E in (1, 2, 3, 5, 8):
        acc, pc = oracle.shouji_batch(P, T, L, E=E)
        acc2, pc2 = oracle.shouji_batch2(P, T, L, L, E=E, mode=GLOBAL)
        assert np.array_equal(pc, pc2) and np.array_equal(acc, acc2)
    for k in range(0, n, 40):
        for E in (2, 5):
            assert oracle.shouji_pair2(P[k], T[k], E, GLOBAL) == oracle.shouji_pair(P[k], T[k], E)


def test_read_embedded_in_reference_closed_form():
    # read over {A, C}, reference = X + read + Y with X, Y over {G, T}: every
    # cell off the read's copy is a mismatch, so S is zero exactly on the copy
    # [k, k + mP) when the copy is on a diagonal |k| <= E (mP >= 4)
    rng = np.random.default_rng(7)
    for _ in range(200):
        mP = int(rng.integers(4, 40))
        E = int(rng.integers(0, 6))
        k = int(rng.integers(0, E + 1))
        tail = int(rng.integers(0, 12))
        P = rng.integers(0, 2, mP).astype(np.uint8)
        T = np.concatenate([rng.integers(2, 4, k), P, rng.integers(2, 4, tail)]).astype(np.uint8)
        mT = len(T)
        c, S = oracle.shouji_pair2(P, T, E, GLOBAL)
        assert S == "1" * k + "0" * mP + "1" * tail
        assert c == mT - mP
        assert oracle.shouji_pair2(P, T, E, LOCAL)[0] == 0
        assert oracle.shouji_pair2(P, T, E, GSTART)[0] == tail
        assert oracle.shouji_pair2(P, T, E, GEND)[0] == k


def test_no_common_base_keeps_every_one():
    for mP, mT in ((5, 9), (9, 5), (0, 7), (7, 0)):
        P = np.zeros(mP, np.uint8)          # all A
        T = np.full(mT, 3, np.uint8)        # all T
        for mode in (GLOBAL, LOCAL, GSTART, GEND):
            assert oracle.shouji_pair2(P, T, 3, mode)[0] == mT


def _matrix2(Pseq, Tseq, E, mode):
    """Independent version over the explicit mP x mT map, indexed (pattern row,
    text column) as in Eq. 1, for the counting modes.  Windows are text
    columns; Algorithm 1's order (text index - pattern index = +j before -j,
    main last); S over the text's positions; the mode drops end runs."""
    mP, mT = len(Pseq), len(Tseq)

    def cell(r, c):
        if 0 <= r < mP and 0 <= c < mT and abs(c - r) <= E:
            return 0 if Pseq[r] == Tseq[c] else 1
        return 1

    order = [x for j in range(1, E + 1) for x in (j, -j)] + [0]
    S = [1] * (mT + 3)
    for w in range(mT):
        best, bkey = None, None
        for k in order:
            seg = [cell(c - k, c) for c in range(w, w + 4)]
            key = (seg.count(0), seg[0] == 0)
            if bkey is None or key > bkey:
                best, bkey = seg, key
        if best.count(0) > S[w:w + 4].count(0):
            S[w:w + 4] = best
    S = S[:mT]
    lo, hi = 0, mT
    if 0 in S:
        first = S.index(0)
        last = mT - 1 - S[::-1].index(0)
        if mode in (LOCAL, GSTART):
            lo = first
        if mode in (LOCAL, GEND):
            hi = last + 1
    return sum(S[lo:hi])


@pytest.mark.parametrize("mode", [GLOBAL, LOCAL, GSTART, GEND])
def test_exhaustive_tiny_unequal_lengths_vs_matrix(mode):
    # every pair of sequences of lengths 0..3 over three letters, every E <= 4
    seqs = [s for n in range(4) for s in itertools.product(range(3), repeat=n)]
    for E in range(5):
        for a in seqs:
            for b in seqs:
                got = oracle.shouji_pair2(np.array(a, np.uint8), np.array(b, np.uint8), E, mode)[0]
                assert got == _matrix2(a, b, E, mode), (a, b, E, mode)


def test_random_unequal_lengths_vs_matrix():
    rng = np.random.default_rng(8)
    for _ in range(400):
        mP, mT = int(rng.integers(0, 14)), int(rng.integers(0, 14))
        E = int(rng.integers(0, 5))
        a = tuple(int(x) for x in rng.integers(0, 2, mP))
        b = tuple(int(x) for x in rng.integers(0, 2, mT))
        mode = int(rng.integers(0, 4))
        got = oracle.shouji_pair2(np.array(a, np.uint8), np.array(b, np.uint8), E, mode)[0]
        assert got == _matrix2(a, b, E, mode), (a, b, E, mode)


def test_batch2_matches_pairwise_and_marks_invalid():
    rng = np.random.default_rng(9)
    n, stride = 300, 50
    P = rng.integers(0, 4, (n, stride)).astype(np.uint8)
    T = rng.integers(0, 4, (n, stride)).astype(np.uint8)
    LP = rng.integers(0, stride + 1, n).astype(np.int32)
    LT = rng.integers(0, stride + 1, n).astype(np.int32)
    Ep = rng.integers(0, 8, n).astype(np.int32)
    LP[::37] = stride + 1
    LT[5::41] = -1
    Ep[7::43] = -2
    for mode in (GLOBAL, LOCAL, GSTART, GEND):
        acc, pc = oracle.shouji_batch2(P, T, LP, LT, E_per_pair=Ep, mode=mode)
        for p in range(n):
            if LP[p] > stride or LT[p] < 0 or Ep[p] < 0:
                assert acc[p] == 0xFF and pc[p] == -1
                continue
            c, _ = oracle.shouji_pair2(P[p, :LP[p]], T[p, :LT[p]], int(Ep[p]), mode)
            assert pc[p] == c and acc[p] == (1 if c <= Ep[p] else 0)
