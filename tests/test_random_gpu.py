"""Seeded random shapes for every entry point (plain with a padded leading
dimension, window widths, MAGNET, batched, two-length, verifier, relayout
followed by the filter), each compared with the oracle on every pair."""
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


def _pairs(rng, n, max_len):
    """Random pairs of random lengths: reads, and references that are the read
    with a few substitutions, insertions and deletions, or unrelated."""
    P = rng.integers(0, 4, (n, max_len)).astype(np.uint8)
    T = P.copy()
    sub = rng.random((n, max_len)) < rng.uniform(0, 0.08)
    T[sub] = rng.integers(0, 4, int(sub.sum())).astype(np.uint8)
    shift = rng.integers(-3, 4, n)
    for i in np.nonzero(shift)[0]:
        T[i] = np.roll(T[i], int(shift[i]))
    unrelated = rng.random(n) < 0.2
    T[unrelated] = rng.integers(0, 4, (int(unrelated.sum()), max_len)).astype(np.uint8)
    return P, T


@pytest.mark.parametrize("seed", range(10))
def test_batched_random(sj, seed):
    rng = np.random.default_rng(7100 + seed)
    n = int(rng.integers(1, 30_000))
    max_len = int(rng.integers(1, 600))
    P, T = _pairs(rng, n, max_len)
    L = rng.integers(0, max_len + 1, n).astype(np.int32)
    if seed % 3 == 0:
        L[:] = max_len
    E = rng.integers(0, 32, n).astype(np.int32)
    E[rng.random(n) < 0.01] = -1                     # invalid thresholds get sentinels
    cfg = [None, (4, 2), (8, 4), (16, 1), (32, 2)][seed % 5]
    print("case seed=%d n=%d max_len=%d config=%s" % (seed, n, max_len, cfg), flush=True)
    d = torch.device("cuda:0")
    r = torch.from_numpy(sj.pack_words(P, max_len)).to(d)
    t = torch.from_numpy(sj.pack_words(T, max_len)).to(d)
    acc, pc = sj.shouji_filter_batched(r, t, torch.from_numpy(L).to(d), torch.from_numpy(E).to(d),
                                       max_len=max_len, config=cfg)
    torch.cuda.synchronize()
    ga, gp = acc.cpu().numpy(), pc.cpu().numpy()
    bad = E < 0
    assert (ga[bad] == 0xFF).all() and (gp[bad] == -1).all()
    ea, ep = oracle.shouji_batch(P[~bad], T[~bad], L[~bad], E_per_pair=E[~bad])
    assert np.array_equal(ga[~bad], ea) and np.array_equal(gp[~bad], ep)


@pytest.mark.parametrize("seed", range(8))
def test_local_random(sj, seed):
    rng = np.random.default_rng(7200 + seed)
    n = int(rng.integers(1, 6_000))
    max_len = int(rng.integers(4, 300))
    E = int(rng.integers(0, min(12, max_len)))
    mode = seed % 4
    P, T = _pairs(rng, n, max_len)
    if seed % 2:
        LP = np.full(n, int(rng.integers(1, max_len + 1)), np.int32)   # reads of one length
    else:
        LP = rng.integers(0, max_len + 1, n).astype(np.int32)
    LT = rng.integers(0, max_len + 1, n).astype(np.int32)
    print("case seed=%d n=%d max_len=%d E=%d mode=%d" % (seed, n, max_len, E, mode), flush=True)
    d = torch.device("cuda:0")
    r = torch.from_numpy(sj.pack_words(P, max_len)).to(d)
    t = torch.from_numpy(sj.pack_words(T, max_len)).to(d)
    acc, pc = sj.shouji_filter_local(r, t, torch.from_numpy(LP).to(d), torch.from_numpy(LT).to(d), E,
                                     mode=mode, max_len=max_len)
    torch.cuda.synchronize()
    ea, ep = oracle.shouji_batch2(P, T, LP, LT, E=E, mode=mode)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)


@pytest.mark.parametrize("seed", range(8))
def test_verify_random(sj, seed):
    rng = np.random.default_rng(7300 + seed)
    n = int(rng.integers(1, 12_000))
    max_len = int(rng.integers(1, 400))
    E = int(rng.integers(0, 32))
    P, T = _pairs(rng, n, max_len)
    L = rng.integers(0, max_len + 1, n).astype(np.int32)
    print("case seed=%d n=%d max_len=%d E=%d" % (seed, n, max_len, E), flush=True)
    d = torch.device("cuda:0")
    r = torch.from_numpy(sj.pack_words(P, max_len)).to(d)
    t = torch.from_numpy(sj.pack_words(T, max_len)).to(d)
    Ld = torch.from_numpy(L).to(d)
    want = oracle.edit_distance_batch(P, T, L, k=E)
    got = sj.shouji_verify(r, t, Ld, E, max_len=max_len)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().astype(np.int32), want)
    # only the pairs a filter accepted
    acc = torch.from_numpy((rng.random(n) < 0.6).astype(np.uint8)).to(d)
    got = sj.shouji_verify(r, t, Ld, E, filter_accept=acc, max_len=max_len)
    torch.cuda.synchronize()
    exp = np.where(acc.cpu().numpy() == 1, want, -2)
    assert np.array_equal(got.cpu().numpy().astype(np.int32), exp)


def _padded(sj, rng, X, max_len, ld):
    """Word-major words of X in the first n columns of an [nwords, ld] tensor
    whose other columns hold random words (never read: pairs beyond n_pairs)."""
    n = X.shape[0]
    w = sj.pack_words(X, max_len)
    buf = rng.integers(-2**31, 2**31, (w.shape[0], ld)).astype(np.int32)
    buf[:, :n] = w
    return torch.from_numpy(buf).to(torch.device("cuda:0"))


@pytest.mark.parametrize("seed", range(12))
def test_plain_random(sj, seed):
    """The plain entry point with a leading dimension above n_pairs, with and
    without lengths, E drawn over 0..31 (clamped to max_len - 1 where larger)."""
    rng = np.random.default_rng(7400 + seed)
    n = int(rng.integers(1, 40_000))
    max_len = int(rng.integers(1, 500))
    E = int(rng.integers(0, 32))
    ld = n + int(rng.integers(0, 3)) * int(rng.integers(1, 700))
    P, T = _pairs(rng, n, max_len)
    with_lengths = seed % 3 != 0
    L = rng.integers(0, max_len + 1, n).astype(np.int32) if with_lengths else np.full(n, max_len, np.int32)
    print("case seed=%d n=%d ld=%d max_len=%d E=%d lengths=%d" % (seed, n, ld, max_len, E, with_lengths),
          flush=True)
    r = _padded(sj, rng, P, max_len, ld)
    t = _padded(sj, rng, T, max_len, ld)
    Ld = torch.from_numpy(L).to(r.device) if with_lengths else None
    acc, pc = sj.shouji_filter(r, t, Ld, E, n_pairs=n, max_len=max_len)
    torch.cuda.synchronize()
    ea, ep = oracle.shouji_batch(P, T, L, E=E)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)


@pytest.mark.parametrize("seed", range(8))
def test_window_random(sj, seed):
    rng = np.random.default_rng(7500 + seed)
    n = int(rng.integers(1, 8_000))
    max_len = int(rng.integers(1, 300))
    E = int(rng.integers(0, 32))
    W = int(rng.integers(1, 17))
    P, T = _pairs(rng, n, max_len)
    L = rng.integers(0, max_len + 1, n).astype(np.int32)
    print("case seed=%d n=%d max_len=%d E=%d W=%d" % (seed, n, max_len, E, W), flush=True)
    d = torch.device("cuda:0")
    acc, pc = sj.shouji_filter_window(torch.from_numpy(sj.pack_words(P, max_len)).to(d),
                                      torch.from_numpy(sj.pack_words(T, max_len)).to(d),
                                      torch.from_numpy(L).to(d), E, W, max_len=max_len)
    torch.cuda.synchronize()
    ea, ep = oracle.shouji_batch_w(P, T, L, E, W)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)


@pytest.mark.parametrize("seed", range(8))
def test_magnet_random(sj, seed):
    rng = np.random.default_rng(7600 + seed)
    n = int(rng.integers(1, 8_000))
    max_len = int(rng.integers(1, 300))
    E = int(rng.integers(0, 32))
    P, T = _pairs(rng, n, max_len)
    with_lengths = seed % 2 == 0
    L = rng.integers(0, max_len + 1, n).astype(np.int32) if with_lengths else np.full(n, max_len, np.int32)
    print("case seed=%d n=%d max_len=%d E=%d lengths=%d" % (seed, n, max_len, E, with_lengths), flush=True)
    d = torch.device("cuda:0")
    acc, pc = sj.shouji_filter_magnet(torch.from_numpy(sj.pack_words(P, max_len)).to(d),
                                      torch.from_numpy(sj.pack_words(T, max_len)).to(d),
                                      torch.from_numpy(L).to(d) if with_lengths else None, E, max_len=max_len)
    torch.cuda.synchronize()
    ea, ep = oracle.magnet_batch(P, T, L, E)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)


@pytest.mark.parametrize("seed", range(6))
def test_relayout_then_filter_random(sj, seed):
    """Pair-major words with spare words per sequence, relaid into a padded
    word-major layout, then filtered: every pair equal to the oracle."""
    rng = np.random.default_rng(7700 + seed)
    n = int(rng.integers(1, 30_000))
    max_len = int(rng.integers(1, 400))
    E = int(rng.integers(0, 32))
    wps = (max_len + 31) // 32 + int(rng.integers(0, 3))
    ld = n + int(rng.integers(0, 300))
    P, T = _pairs(rng, n, max_len)
    L = rng.integers(0, max_len + 1, n).astype(np.int32)
    print("case seed=%d n=%d max_len=%d wps=%d ld=%d E=%d" % (seed, n, max_len, wps, ld, E), flush=True)
    d = torch.device("cuda:0")
    r = sj.relayout_pair_major(torch.from_numpy(sj.pack_pair_major(P, max_len, wps).view(np.int64)).to(d),
                               max_len, ld=ld)
    t = sj.relayout_pair_major(torch.from_numpy(sj.pack_pair_major(T, max_len, wps).view(np.int64)).to(d),
                               max_len, ld=ld)
    assert torch.equal(r[:, :n].cpu(), torch.from_numpy(sj.pack_words(P, max_len)))
    acc, pc = sj.shouji_filter(r, t, torch.from_numpy(L).to(d), E, n_pairs=n, max_len=max_len)
    torch.cuda.synchronize()
    ea, ep = oracle.shouji_batch(P, T, L, E=E)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)
