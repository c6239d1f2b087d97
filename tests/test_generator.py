"""Checks of the seeded synthetic input generator (shared by both sides)."""
import numpy as np

import oracle
import syninput


def test_deterministic_and_shaped():
    a = syninput.generate(1000, 100, E=3, seed=7)
    b = syninput.generate(1000, 100, E=3, seed=7)
    c = syninput.generate(1000, 100, E=3, seed=8)
    assert np.array_equal(a.P, b.P) and np.array_equal(a.T, b.T)
    assert not np.array_equal(a.P, c.P)
    assert a.P.max() <= 3 and a.T.max() <= 3
    assert (a.lengths == 100).all() and (a.E == 3).all()


def test_prefix_stable():
    # pair p's content depends only on (seed, p): a smaller batch is a prefix
    a = syninput.generate(500, 64, 300, E=None, seed=3)
    b = syninput.generate(200, 64, 300, E=None, seed=3)
    assert np.array_equal(a.P[:200], b.P) and np.array_equal(a.lengths[:200], b.lengths)


def test_mixed_lengths_and_thresholds():
    p = syninput.generate(20000, 64, 300, E=None, r_max=0.10, seed=3000)
    assert p.lengths.min() == 64 and p.lengths.max() == 300
    assert (p.E >= 0).all() and (p.E <= np.floor(0.10 * p.lengths)).all()
    # padding beyond each length is zero
    k = int(np.argmin(p.lengths))
    assert (p.P[k, p.lengths[k]:] == 0).all()


def test_related_pairs_are_close():
    # related pairs: at most 2E edits, plus the re-padding at the end after
    # insertions and deletions (bounded by the same count)
    p = syninput.generate(2000, 100, E=2, seed=0, p_unrelated=0.0)
    d = np.array([oracle.edit_distance(p.P[k], p.T[k]) for k in range(300)])
    assert d.max() <= 8
    u = syninput.generate(300, 100, E=2, seed=0, p_unrelated=1.0)
    du = np.array([oracle.edit_distance(u.P[k], u.T[k]) for k in range(50)])
    assert du.min() > 30


def test_tandem_repeats_present():
    p = syninput.generate(2000, 250, E=5, seed=2005, p_repeat=1.0)
    # a periodic block of >= 20% of the read: some period q<=6 with many P[j]==P[j+q]
    runs = 0
    for k in range(200):
        r = p.P[k]
        best = max(int((r[:-q] == r[q:]).sum()) for q in range(1, 7))
        runs += best >= 0.2 * 250
    assert runs == 200
