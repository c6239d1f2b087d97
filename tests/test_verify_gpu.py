"""GPU verifier (banded edit distance of filtered pairs) against the CPU
oracle's banded edit distance, exact on every pair."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import syninput

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_07858_amd as m
    m.lib()
    return m


def _dev(sj, p, max_len):
    d = torch.device("cuda:0")
    return (torch.from_numpy(sj.pack_words(p.P, max_len)).to(d),
            torch.from_numpy(sj.pack_words(p.T, max_len)).to(d),
            torch.from_numpy(np.ascontiguousarray(p.lengths, dtype=np.int32)).to(d))


@pytest.mark.parametrize("E", [0, 1, 2, 5, 8, 13, 24, 31])
def test_distances_vs_oracle(sj, E):
    # edits k ~ U{0..2E} (20% unrelated): distances on both sides of E
    p = syninput.generate(8000, 60, 180, E=max(E, 1), seed=600 + E)
    r, t, L = _dev(sj, p, 180)
    print("verify E=%d n=%d" % (E, p.n), flush=True)
    got = sj.shouji_verify(r, t, L, E, max_len=180)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.int32)
    want = oracle.edit_distance_batch(p.P, p.T, p.lengths, k=E)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "mismatches at %s: gpu %s oracle %s (m %s)" % (
        bad[:6], got[bad[:6]], want[bad[:6]], p.lengths[bad[:6]])
    assert (want >= 0).any() and (want == -1).any()


def test_only_accepted_pairs_are_verified(sj):
    p = syninput.generate(20_000, 100, E=5, seed=1005)
    r, t, L = _dev(sj, p, 100)
    acc, _ = sj.shouji_filter(r, t, L, 5, max_len=100)
    dist = sj.shouji_verify(r, t, L, 5, filter_accept=acc, max_len=100)
    torch.cuda.synchronize()
    a = acc.cpu().numpy()
    d = dist.cpu().numpy().astype(np.int32)
    want = oracle.edit_distance_batch(p.P, p.T, p.lengths, k=5)
    assert (d[a != 1] == -2).all()
    assert np.array_equal(d[a == 1], want[a == 1])
    # every pair the filter rejected that is within E is a false reject, the
    # rest of the accepted ones above E are false accepts: both are counted
    # by the pipeline, and a similar pair is rarely rejected
    fr = int(((a != 1) & (want >= 0)).sum())
    assert fr <= 0.05 * max(1, int((want >= 0).sum()))


def test_edge_cases(sj):
    d = torch.device("cuda:0")
    n, max_len = 9, 40
    P = np.random.default_rng(1).integers(0, 4, (n, max_len)).astype(np.uint8)
    T = P.copy()
    L = np.full(n, max_len, np.int32)
    T[1, 7] = (T[1, 7] + 1) % 4                       # one substitution
    T[2, 5:] = P[2, 4:-1]                             # one insertion + a trailing change
    L[3] = 0                                          # empty pair
    L[4] = 1
    T[4, 0] = (P[4, 0] + 2) % 4                       # one base, different
    L[5] = max_len + 1                                # invalid
    L[6] = -1                                         # invalid
    T[7] = (P[7] + 1) % 4                             # nothing matches
    r = torch.from_numpy(sj.pack_words(P, max_len)).to(d)
    t = torch.from_numpy(sj.pack_words(T, max_len)).to(d)
    Ld = torch.from_numpy(L).to(d)
    for E in (0, 1, 3, 31):
        got = sj.shouji_verify(r, t, Ld, E, max_len=max_len).cpu().numpy().astype(np.int32)
        ok = (L >= 0) & (L <= max_len)
        want = oracle.edit_distance_batch(P[ok], T[ok], L[ok], k=E)
        assert np.array_equal(got[ok], want), E
        assert (got[~ok] == -3).all()
        assert got[0] == 0 and got[3] == 0
        assert got[1] == (1 if E >= 1 else -1)


def test_argument_errors(sj):
    d = torch.device("cuda:0")
    r = torch.zeros((4, 10), dtype=torch.int32, device=d)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_verify(r, r, None, -1, max_len=64)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_verify(r, r, None, 32, max_len=64)


@pytest.mark.parametrize("E", [3, 7, 11, 20])
def test_long_mixed_lengths_and_odd_counts(sj, E):
    # lengths 1..1024 (64-word rows) and an odd number of pairs: the last lane
    # of the two-pairs-per-lane band holds one pair; pairs with 0..3 bases
    p = syninput.generate(3001, 1, 1024, E=E, seed=700 + E)
    r, t, L = _dev(sj, p, 1024)
    print("verify long E=%d n=%d" % (E, p.n), flush=True)
    got = sj.shouji_verify(r, t, L, E, max_len=1024)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.int32)
    want = oracle.edit_distance_batch(p.P, p.T, p.lengths, k=E)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "mismatches at %s: gpu %s oracle %s (m %s)" % (
        bad[:6], got[bad[:6]], want[bad[:6]], p.lengths[bad[:6]])


def test_two_letter_alphabet_every_threshold(sj):
    # many near-ties of the recurrence: codes 0/1 only, every E in 0..31
    p = syninput.generate(2000, 20, 140, E=6, seed=777)
    p.P[:] &= 1
    p.T[:] &= 1
    r, t, L = _dev(sj, p, 140)
    for E in range(32):
        got = sj.shouji_verify(r, t, L, E, max_len=140).cpu().numpy().astype(np.int32)
        want = oracle.edit_distance_batch(p.P, p.T, p.lengths, k=E)
        assert np.array_equal(got, want), E
