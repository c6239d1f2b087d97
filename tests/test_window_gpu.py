"""GPU window-width variant (Suppl. Sec. 6.1, Fig. 4: widths other than 4)
against the CPU oracle's window-width filter, exact on every accept bit and
count; W = 4 also equals the plain kernel."""
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
            torch.from_numpy(np.ascontiguousarray(L, dtype=np.int32)).to(d))


def _compare(sj, P, T, L, E, W, max_len):
    r, t, Ld = _dev(sj, P, T, L, max_len)
    print("window E=%d W=%d n=%d max_len=%d" % (E, W, len(L), max_len), flush=True)
    acc, pc = sj.shouji_filter_window(r, t, Ld, E, W, max_len=max_len)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy()
    pc = pc.cpu().numpy()
    wa, wp = oracle.shouji_batch_w(P, T, L, E, W)
    bad = np.nonzero((acc != wa) | (pc != wp))[0]
    assert bad.size == 0, "E=%d W=%d mismatches at %s: gpu %s/%s oracle %s/%s" % (
        E, W, bad[:6], acc[bad[:6]], pc[bad[:6]], wa[bad[:6]], wp[bad[:6]])
    return acc, pc


@pytest.mark.parametrize("W", [1, 2, 3, 4, 5, 6, 8, 12, 16])
@pytest.mark.parametrize("E", [0, 2, 5, 10])
def test_widths_vs_oracle(sj, W, E):
    p = syninput.generate(3000, 40, 130, E=max(E, 1), seed=700 + 17 * W + E)
    _compare(sj, p.P, p.T, p.lengths, E, W, 130)


@pytest.mark.parametrize("E", [13, 20, 31, 45])
def test_wide_bands(sj, E):
    # compiled bands 16, 24 and 31; E above the longest length clamps to m - 1
    max_len = 32 if E == 45 else 150
    p = syninput.generate(1500, 20, max_len, E=min(E, 10), seed=800 + E)
    for W in (3, 4, 7):
        _compare(sj, p.P, p.T, p.lengths, E, W, max_len)


def test_width4_equals_plain(sj):
    p = syninput.generate(20_000, 100, E=5, seed=901)
    r, t, Ld = _dev(sj, p.P, p.T, p.lengths, 100)
    for E in (0, 3, 5, 9):
        a1, c1 = sj.shouji_filter_window(r, t, Ld, E, 4, max_len=100)
        a2, c2 = sj.shouji_filter(r, t, Ld, E, max_len=100)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2) and torch.equal(c1, c2), E


def test_edge_cases(sj):
    n, max_len = 10, 37
    rng = np.random.default_rng(3)
    P = rng.integers(0, 4, (n, max_len)).astype(np.uint8)
    T = P.copy()
    L = np.full(n, max_len, np.int32)
    T[1, 7] = (T[1, 7] + 1) % 4
    L[2] = 0
    L[3] = 1
    L[4] = 2
    L[5] = max_len + 1                                # invalid
    L[6] = -4                                         # invalid
    T[7] = (P[7] + 1) % 4
    T[8, 9:] = P[8, 8:-1]                             # one insertion
    L[9] = 16                                         # one full word
    r, t, Ld = _dev(sj, P, T, L, max_len)
    ok = (L >= 0) & (L <= max_len)
    for W in (1, 4, 5, 16):
        for E in (0, 1, 3, 31):
            acc, pc = sj.shouji_filter_window(r, t, Ld, E, W, max_len=max_len)
            acc = acc.cpu().numpy()
            pc = pc.cpu().numpy()
            wa, wp = oracle.shouji_batch_w(P[ok], T[ok], L[ok], E, W)
            assert np.array_equal(acc[ok], wa) and np.array_equal(pc[ok], wp), (W, E)
            assert (acc[~ok] == 0xFF).all() and (pc[~ok] == -1).all()
            assert pc[0] == 0 and pc[2] == 0 and acc[2] == 1


def test_ragged_count_and_no_lengths(sj):
    # pair counts that leave partial workgroups, and the lengths pointer absent
    rng = np.random.default_rng(5)
    for n in (1, 255, 257, 1000):
        P = rng.integers(0, 4, (n, 50)).astype(np.uint8)
        T = P.copy()
        T[rng.random((n, 50)) < 0.06] = 2
        d = torch.device("cuda:0")
        r = torch.from_numpy(sj.pack_words(P, 50)).to(d)
        t = torch.from_numpy(sj.pack_words(T, 50)).to(d)
        acc, pc = sj.shouji_filter_window(r, t, None, 3, 6, max_len=50)
        wa, wp = oracle.shouji_batch_w(P, T, np.full(n, 50, np.int32), 3, 6)
        assert np.array_equal(acc.cpu().numpy(), wa) and np.array_equal(pc.cpu().numpy(), wp), n


def test_longest_sequences_and_widest_rings(sj):
    # lengths up to 1,024 (11-bit counts), the widest window with E = 31 (the
    # largest LDS rings, past 64 KB per wavefront), W = 1 with E = 0, pair
    # counts that leave a partial wavefront of 2,048 pairs, and lengths mixed
    # inside wavefronts
    max_len = 1024
    rng = np.random.default_rng(11)
    n = 2048 + 77
    P = rng.integers(0, 4, (n, max_len)).astype(np.uint8)
    T = P.copy()
    T[rng.random((n, max_len)) < 0.004] = 1
    for i in range(0, n, 7):
        T[i] = np.roll(T[i], 1)
    L = rng.integers(900, max_len + 1, n).astype(np.int32)
    L[::5] = max_len
    r, t, Ld = _dev(sj, P, T, L, max_len)
    for W, E in ((16, 31), (1, 0), (9, 31), (12, 7)):
        print("window W=%d E=%d n=%d max_len=%d" % (W, E, n, max_len), flush=True)
        acc, pc = sj.shouji_filter_window(r, t, Ld, E, W, max_len=max_len)
        torch.cuda.synchronize()
        wa, wp = oracle.shouji_batch_w(P, T, L, E, W)
        assert np.array_equal(acc.cpu().numpy(), wa) and np.array_equal(pc.cpu().numpy(), wp), (W, E)
        if W == 1:
            assert (pc.cpu().numpy() > 255).any()   # counts past 8 bits


def test_argument_errors(sj):
    d = torch.device("cuda:0")
    r = torch.zeros((4, 10), dtype=torch.int32, device=d)
    for W in (0, 17, -1):
        with pytest.raises(sj.ShoujiError):
            sj.shouji_filter_window(r, r, None, 2, W, max_len=64)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_filter_window(r, r, None, -1, 4, max_len=64)
    with pytest.raises(sj.ShoujiError):
        sj.shouji_filter_window(r, r, None, 40, 4, max_len=64)
