"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties the oracle to something other than itself:
  * the worked examples printed in the paper (Fig. 1; Fig. 6(a)(b));
  * proven invariants of the method (E = 0 reduces to Hamming distance, equal
    sequences give no ones, every one of S is a forced mismatch or a copied
    diagonal bit, E >= m always accepts);
  * an independent implementation, written here over the full m x m matrix of
    Eq. 1 with matrix (row, column) indexing, compared exhaustively on tiny
    inputs and on random small ones.
"""
import itertools

import numpy as np
import pytest

import oracle
import syninput
from golden_io import read_sections


def _edit_distance_str(a, b):
    # plain string edit distance, used only to compare garbled printed rows
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def _is_subsequence(short, long):
    it = iter(long)
    return all(c in it for c in short)


# ---------------------------------------------------------------- Fig. 1

def test_fig1_three_edits_and_common_subsequences():
    g = read_sections("fig1.txt")[""]
    E = int(g["E"])
    ones, S = oracle.shouji_pair(g["pattern"], g["text"], E)
    # Sec. 2.2.1: the pattern differs from the text by three edits, and the
    # caption's three common subsequences are the zero streaks of S.
    assert ones == int(g["edits"])
    zeros = set()
    for rng in g["common"].split(","):
        lo, hi = (int(x) for x in rng.strip().split("-"))
        zeros.update(range(lo, hi + 1))
    assert {j for j, c in enumerate(S) if c == "0"} == zeros
    assert ones <= E  # accepted


def test_fig1_convention_matters():
    # With pattern and text swapped (the other reading of the row/column roles)
    # the popcount is no longer the stated three edits: the example fixes the
    # convention of Eq. 1 (rows pattern, columns text).
    g = read_sections("fig1.txt")[""]
    ones_swapped, _ = oracle.shouji_pair(g["text"], g["pattern"], int(g["E"]))
    assert ones_swapped != int(g["edits"])


# ---------------------------------------------------------------- Fig. 6

@pytest.fixture(scope="module")
def fig6():
    return read_sections("fig6_global.txt")


def _printed_row(sec, d):
    if d == 0:
        return sec["main"]
    return sec["upper%d" % d] if d > 0 else sec["lower%d" % (-d)]


def test_fig6_diagonals_follow_eq1(fig6):
    # The printed diagonal rows lost characters in extraction; recompute each
    # row and check it is closer (edit distance) to the printed row than the
    # row of the swapped convention, for at least 15 of the 16 off-diagonal rows.
    closer = 0
    total = 0
    for tag in ("a", "b"):
        sec = fig6[tag]
        P, T = sec["read"], sec["reference"]
        for d in (-4, -3, -2, -1, 1, 2, 3, 4):
            printed = _printed_row(sec, d).replace("-", "")
            ours = oracle.map_row(P, T, d)
            swapped = oracle.map_row(T, P, d)
            # drop the out-of-range columns, printed as '-'
            if d > 0:
                ours, swapped = ours[d:], swapped[d:]
            else:
                ours, swapped = ours[:d], swapped[:d]
            total += 1
            closer += _edit_distance_str(ours, printed) < _edit_distance_str(swapped, printed)
    assert total == 16 and closer >= 15


def test_fig6_main_diagonal(fig6):
    # The main diagonal is the plain mismatch vector; the printed row is that
    # vector with a few characters dropped.
    for tag in ("a", "b"):
        sec = fig6[tag]
        ours = oracle.map_row(sec["read"], sec["reference"], 0)
        printed = sec["main"]
        assert _edit_distance_str(ours, printed) <= 100 - len(printed) + 10


def test_fig6b_shouji_vector(fig6):
    sec = fig6["b"]
    ones, S = oracle.shouji_pair(sec["read"], sec["reference"], int(sec["E"]))
    printed = sec["shouji"]
    # Printed vector holds four ones; the extraction only dropped characters,
    # so the printed row must be a subsequence of the oracle's vector.
    assert ones == printed.count("1") == 4
    assert _is_subsequence(printed, S)
    assert ones <= 4  # accepted


def test_fig6a_shouji_vector(fig6):
    sec = fig6["a"]
    ones, S = oracle.shouji_pair(sec["read"], sec["reference"], int(sec["E"]))
    printed = sec["shouji"]
    # The printed (garbled) vector shows three ones; the pair is accepted at E=4
    # in the figure.  Soft pin: accepted, within one of the printed count, and
    # at most one edit beyond the dropped characters.
    assert ones <= 4
    assert abs(ones - printed.count("1")) <= 1
    assert _edit_distance_str(S, printed) <= (100 - len(printed)) + 1


# ---------------------------------------------------------------- invariants

def _random_pairs(n, m, seed, E=2, p_unrelated=0.3):
    return syninput.generate(n, m, E=E, seed=seed, p_unrelated=p_unrelated)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 16, 33, 100])
def test_E0_is_hamming(m):
    # With E = 0 the only candidate is the main diagonal, so S equals the
    # mismatch vector: popcount = Hamming distance, accept iff equal.
    p = _random_pairs(400, m, seed=11 + m)
    acc, pc = oracle.shouji_batch(p.P, p.T, p.lengths, E=0)
    ham = (p.P[:, :m] != p.T[:, :m]).sum(axis=1)
    assert np.array_equal(pc.astype(np.int64), ham)
    assert np.array_equal(acc == 1, ham == 0)


@pytest.mark.parametrize("E", [0, 1, 2, 5, 10, 40])
def test_identical_pairs_have_no_ones(E):
    p = _random_pairs(300, 64, seed=5)
    acc, pc = oracle.shouji_batch(p.P, p.P, p.lengths, E=E)
    assert (pc == 0).all() and (acc == 1).all()


@pytest.mark.parametrize("m,E", [(8, 1), (20, 2), (50, 5), (100, 3)])
def test_ones_bounded_by_length_and_forced(m, E):
    # popcount <= m; every position where all 2E+1 diagonals mismatch stays one.
    p = _random_pairs(200, m, seed=m * 7 + E, E=E, p_unrelated=0.5)
    acc, pc = oracle.shouji_batch(p.P, p.T, p.lengths, E=E)
    for k in range(p.n):
        P, T = p.P[k, :m], p.T[k, :m]
        forced = 0
        for j in range(m):
            if all(not (0 <= j - d < m and P[j - d] == T[j]) for d in range(-E, E + 1)):
                forced += 1
        assert forced <= pc[k] <= m
    assert np.array_equal(acc == 1, pc <= E)


def test_E_at_least_m_accepts():
    p = _random_pairs(200, 12, seed=3, p_unrelated=1.0)
    acc, pc = oracle.shouji_batch(p.P, p.T, p.lengths, E=12)
    assert (acc == 1).all()


def test_invalid_lengths_and_empty():
    P = np.zeros((3, 8), dtype=np.uint8)
    acc, pc = oracle.shouji_batch(P, P, np.array([0, 9, -1], dtype=np.int32), E=1)
    assert acc.tolist() == [1, 0xFF, 0xFF] and pc.tolist() == [0, -1, -1]


# ------------------------------------------------ independent implementation

def _matrix_shouji(Pseq, Tseq, E):
    """Shouji over the explicit m x m neighbourhood map (Eq. 1).

    N[r][c] = 0 iff pattern[r] == text[c]; only |r - c| <= E is in the map.
    Window w covers text columns w..w+3.  A diagonal is the set of cells with
    c - r = k; its 4-bit segment in window w is the cells (c - k, c) for the
    4 columns, cells outside the map being 1.  The winner has the most zeros,
    then a leading zero, then comes first in Algorithm 1's order: for j = 1..E
    its "lower" diagonal j, whose text index exceeds the pattern index by j
    (Algorithm 1 indexes the map by text row, pattern column: k = +j here),
    before its "upper" diagonal j (k = -j), and the main diagonal last.
    S[w..w+3] takes the winner if it has strictly more zeros.
    """
    m = len(Tseq)
    Nmat = [[1] * m for _ in range(m)]
    for r in range(m):
        for c in range(max(0, r - E), min(m, r + E + 1)):
            Nmat[r][c] = 0 if Pseq[r] == Tseq[c] else 1

    def seg(k, w):
        out = []
        for c in range(w, w + 4):
            r = c - k
            out.append(Nmat[r][c] if (0 <= r < m and c < m and abs(r - c) <= E) else 1)
        return out

    names = []
    for k in range(1, E + 1):
        names += [k, -k]
    names.append(0)
    S = [1] * (m + 3)
    for w in range(m):
        cands = [seg(k, w) for k in names]
        keys = [(4 - sum(z), z[0] == 0) for z in cands]
        best = max(keys)
        Z = cands[keys.index(best)]
        if Z.count(0) > S[w:w + 4].count(0):
            S[w:w + 4] = Z
    return sum(S[:m])


def _batch_vs_matrix(pairs, E):
    P = np.array([a for a, _ in pairs], dtype=np.uint8)
    T = np.array([b for _, b in pairs], dtype=np.uint8)
    L = np.full(len(pairs), P.shape[1], dtype=np.int32)
    _, pc = oracle.shouji_batch(P, T, L, E=E)
    for k, (a, b) in enumerate(pairs):
        assert pc[k] == _matrix_shouji(a, b, E), (a, b, E)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_exhaustive_tiny_vs_matrix(m):
    seqs = list(itertools.product(range(4), repeat=m))
    pairs = [(a, b) for a in seqs for b in seqs]
    for E in range(0, m + 2):
        _batch_vs_matrix(pairs, E)


def test_exhaustive_m4_binary_alphabet_vs_matrix():
    # all 2^4 x 2^4 pairs over two letters (many ties), every E
    seqs = list(itertools.product(range(2), repeat=4))
    pairs = [(a, b) for a in seqs for b in seqs]
    for E in range(0, 6):
        _batch_vs_matrix(pairs, E)


@pytest.mark.parametrize("m", [4, 5, 6, 9, 13, 20])
def test_random_small_vs_matrix(m):
    rng = np.random.default_rng(100 + m)
    for E in (0, 1, 2, 3, m // 2):
        pairs = []
        for _ in range(150):
            a = rng.integers(0, 4, m)
            if rng.random() < 0.5:
                b = a.copy()
                for _ in range(rng.integers(0, 3)):
                    b[rng.integers(0, m)] = rng.integers(0, 4)
                b = np.roll(b, rng.integers(-1, 2))
            else:
                b = rng.integers(0, 2, m)  # low complexity
                a = rng.integers(0, 2, m)
            pairs.append((tuple(int(x) for x in a), tuple(int(x) for x in b)))
        _batch_vs_matrix(pairs, E)


def test_reading_a_and_b_differ_only_on_main_lead_ties():
    # Sanity of the sensitivity-study flag: readings agree at E = 0.
    p = _random_pairs(500, 40, seed=9)
    _, pb = oracle.shouji_batch(p.P, p.T, p.lengths, E=0, reading=oracle.READING_B)
    _, pa = oracle.shouji_batch(p.P, p.T, p.lengths, E=0, reading=oracle.READING_A)
    assert np.array_equal(pa, pb)
