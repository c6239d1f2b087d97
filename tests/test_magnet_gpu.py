"""GPU MAGNET filter (Suppl. Sec. 7.1, Algorithms 3-4) against the CPU oracle,
exact on every accept bit and popcount."""
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


def _dev(sj, P, T, L, max_len):
    d = torch.device("cuda:0")
    return (torch.from_numpy(sj.pack_words(P, max_len)).to(d),
            torch.from_numpy(sj.pack_words(T, max_len)).to(d),
            None if L is None else torch.from_numpy(np.ascontiguousarray(L, dtype=np.int32)).to(d))


def _compare(sj, P, T, L, E, max_len, tag=""):
    r, t, Ld = _dev(sj, P, T, L, max_len)
    print("magnet %s E=%d n=%d max_len=%d" % (tag, E, P.shape[0], max_len), flush=True)
    acc, pc = sj.shouji_filter_magnet(r, t, Ld, E, max_len=max_len)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy()
    pc = pc.cpu().numpy()
    Lh = np.full(P.shape[0], max_len, np.int32) if L is None else L
    wa, wp = oracle.magnet_batch(P, T, Lh, E)
    bad = np.nonzero((acc != wa) | (pc != wp))[0]
    assert bad.size == 0, "E=%d mismatches at %s: gpu %s/%s oracle %s/%s (m %s)" % (
        E, bad[:6], acc[bad[:6]], pc[bad[:6]], wa[bad[:6]], wp[bad[:6]], Lh[bad[:6]])
    return acc, pc


@pytest.mark.parametrize("E", [0, 1, 2, 3, 5, 8, 10])
def test_m100_vs_oracle(sj, E):
    p = syninput.generate(20_077, 100, E=max(E, 1), seed=1100 + E)
    acc, pc = _compare(sj, p.P, p.T, p.lengths, E, 100, "m100")
    assert (acc == 1).any() and (acc == 0).any()


@pytest.mark.parametrize("E", [5, 15, 25])
def test_m250_vs_oracle(sj, E):
    # max_len 250: both sequences' words in LDS at E = 5, the read's only at
    # E = 15 and 25 (the stack takes the rest)
    p = syninput.generate(4_000, 250, E=E, seed=1150 + E)
    acc, pc = _compare(sj, p.P, p.T, p.lengths, E, 250, "m250")
    assert (acc == 1).any() and (acc == 0).any()


@pytest.mark.parametrize("E", [0, 4, 13, 20, 31])
def test_mixed_lengths_vs_oracle(sj, E):
    p = syninput.generate(6000, 40, 300, E=min(max(E, 1), 25), seed=1200 + E)
    _compare(sj, p.P, p.T, p.lengths, E, 300, "mixed")


def test_ties_two_letters(sj):
    # a two-letter alphabet: many equally long runs on several diagonals
    rng = np.random.default_rng(1300)
    n, ml = 8000, 70
    P = rng.integers(0, 2, (n, ml)).astype(np.uint8)
    T = P.copy()
    T[rng.random((n, ml)) < 0.1] ^= 1
    L = rng.integers(0, ml + 1, n).astype(np.int32)
    for E in (0, 1, 2, 5, 9):
        _compare(sj, P, T, L, E, ml, "binary")


def test_indels_and_periodic(sj):
    # single insertions / deletions (MAGNET's false rejects) and periodic
    # texts with substitutions (the oracle's closed forms), in one batch
    rng = np.random.default_rng(1400)
    n, m = 3000, 90
    T = rng.integers(0, 4, (n, m)).astype(np.uint8)
    P = T.copy()
    for i in range(n):
        k = int(rng.integers(1, m - 1))
        kind = i % 3
        if kind == 0:
            P[i] = np.concatenate([T[i, :k], rng.integers(0, 4, 1), T[i, k:m - 1]])
        elif kind == 1:
            P[i] = np.concatenate([T[i, :k], T[i, k + 1:], rng.integers(0, 4, 1)])
        else:
            T[i] = np.resize(np.arange(4, dtype=np.uint8), m)
            P[i] = T[i]
            pos = rng.choice(np.arange(2, m - 2), size=int(rng.integers(0, 6)), replace=False)
            P[i, pos] = (T[i, pos] + 2) % 4
    for E in (1, 2, 3, 6):
        _compare(sj, P, T, np.full(n, m, np.int32), E, m, "indels")


def test_edge_cases(sj):
    n, max_len = 12, 37
    rng = np.random.default_rng(1500)
    P = rng.integers(0, 4, (n, max_len)).astype(np.uint8)
    T = P.copy()
    L = np.full(n, max_len, np.int32)
    T[1, 7] = (T[1, 7] + 1) % 4
    L[2] = 0
    L[3] = 1
    L[4] = 2
    L[5] = max_len + 1                                # invalid
    L[6] = -4                                         # invalid
    T[7] = (P[7] + 1) % 4                             # nothing matches on the main diagonal
    T[8, 9:] = P[8, 8:-1]                             # one insertion
    L[9] = 16                                         # one full word
    L[10] = 17
    T[11] = (P[11] + 1) % 4
    P[11] = 0
    T[11] = 1                                         # no zero on any diagonal
    r, t, Ld = _dev(sj, P, T, L, max_len)
    ok = (L >= 0) & (L <= max_len)
    for E in (0, 1, 3, 20, 31, 36, 37, 1000):
        if min(E, max_len - 1) > 31:
            with pytest.raises(sj.ShoujiError):
                sj.shouji_filter_magnet(r, t, Ld, E, max_len=max_len)
            continue
        acc, pc = sj.shouji_filter_magnet(r, t, Ld, E, max_len=max_len)
        acc = acc.cpu().numpy()
        pc = pc.cpu().numpy()
        wa, wp = oracle.magnet_batch(P[ok], T[ok], L[ok], E)
        assert np.array_equal(acc[ok], wa) and np.array_equal(pc[ok], wp), E
        assert (acc[~ok] == 0xFF).all() and (pc[~ok] == -1).all()
        assert pc[0] == 0 and pc[2] == 0 and acc[2] == 1


def test_large_E_clamped(sj):
    # max_len <= 32: E above the clamp (E >= m) accepts every pair
    rng = np.random.default_rng(1600)
    n, ml = 2000, 32
    P = rng.integers(0, 4, (n, ml)).astype(np.uint8)
    T = rng.integers(0, 4, (n, ml)).astype(np.uint8)
    L = rng.integers(0, ml + 1, n).astype(np.int32)
    for E in (31, 32, 40, 100):
        acc, pc = _compare(sj, P, T, L, E, ml, "clamp")
        if E >= ml:
            assert (acc == 1).all()


def test_ragged_count_no_lengths_and_long(sj):
    rng = np.random.default_rng(1700)
    for n in (1, 255, 257, 1000):
        P = rng.integers(0, 4, (n, 50)).astype(np.uint8)
        T = P.copy()
        T[rng.random((n, 50)) < 0.05] = 2
        _compare(sj, P, T, None, 3, 50, "ragged")
    # the longest sequences
    p = syninput.generate(300, 900, 1024, E=20, seed=1701)
    _compare(sj, p.P, p.T, p.lengths, 20, 1024, "long")


def test_argument_errors(sj):
    d = torch.device("cuda:0")
    r = torch.zeros((4, 10), dtype=torch.int32, device=d)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_filter_magnet(r, r, None, -1, max_len=64)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_filter_magnet(r, r, None, 40, max_len=64)
