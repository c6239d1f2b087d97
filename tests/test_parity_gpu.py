"""GPU parity: the HIP filter against the CPU oracle, bit-exact on every
accept bit and popcount, through the C ABI.

Sizes: small enough for the oracle to finish in seconds, spanning several
wavefront tiles (1024 pairs each) with a ragged tail; and the full sizes in
one launch each: 2M pairs at m=100 for every E in 0..10 and 2M pairs at
m=250 for E in {0, 5, ..., 25}, every output compared (E=5 at m=100 is the
bench's workload and launch).
"""
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


def _run(sj, p, E, max_len, ld=None, with_lengths=True, pop=True):
    dev = torch.device("cuda:0")
    reads = torch.from_numpy(sj.pack_words(p.P, max_len, ld=ld)).to(dev)
    refs = torch.from_numpy(sj.pack_words(p.T, max_len, ld=ld)).to(dev)
    lens = torch.from_numpy(np.ascontiguousarray(p.lengths, dtype=np.int32)).to(dev) if with_lengths else None
    acc, pc = sj.shouji_filter(reads, refs, lens, E, n_pairs=p.n, max_len=max_len, want_popcount=pop)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), (pc.cpu().numpy() if pc is not None else None)


def _check(sj, p, E, max_len, **kw):
    print("case n=%d max_len=%d E=%d %s" % (p.n, max_len, E, kw), flush=True)
    ga, gp = _run(sj, p, E, max_len, **kw)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=E)
    bad = np.nonzero((ga != ea) | (gp != ep))[0]
    assert bad.size == 0, "mismatches at %s (gpu %s/%s oracle %s/%s)" % (
        bad[:8], ga[bad[:8]], gp[bad[:8]], ea[bad[:8]], ep[bad[:8]])
    return ga, gp


def test_config0_full(sj):
    p = syninput.config0()
    _check(sj, p, 2, 100)


@pytest.mark.parametrize("E", list(range(0, 11)))
def test_config1_slices(sj, E):
    p = syninput.config1(E, n=20_000 + 77)
    _check(sj, p, E, 100)


@pytest.mark.parametrize("E", [0, 5, 10, 15, 20, 25])
def test_config2_slices(sj, E):
    p = syninput.config2(E, n=6_000 + 13)
    _check(sj, p, E, 250)


@pytest.mark.parametrize("E", [0, 1, 3, 8, 17, 30, 31])
def test_mixed_lengths(sj, E):
    p = syninput.generate(9_000, 64, 300, E=E, seed=77 + E)
    _check(sj, p, E, 300)


def test_mixed_short_lengths_and_low_complexity(sj):
    # lengths 0..40 (m < 4 included), two-letter alphabet: many ties
    p = syninput.generate(5_000, 0, 40, E=3, seed=5)
    p.P[:] &= 1
    p.T[:] &= 1
    for E in (0, 1, 2, 3, 6, 31):
        _check(sj, p, E, 40)
    with pytest.raises(sj.ShoujiError):
        _run(sj, p, 32, 40)        # clamped E (min(E, max_len-1)) above the maximum


def test_tiny_and_ragged_batches(sj):
    for n in (1, 2, 63, 64, 65, 2047, 2048, 2049):
        p = syninput.generate(n, 100, E=3, seed=n)
        _check(sj, p, 3, 100)


def test_no_lengths_and_padded_ld(sj):
    p = syninput.generate(3_000, 100, E=4, seed=9)
    ga, gp = _run(sj, p, 4, 100, ld=3_333, with_lengths=False)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=4)
    assert np.array_equal(ga, ea) and np.array_equal(gp, ep)


@pytest.mark.parametrize("m,E", [(250, 13), (250, 14), (250, 15), (250, 20), (250, 22), (250, 23), (250, 25),
                                 (100, 0), (100, 5), (100, 10), (37, 31), (1024, 12)])
def test_no_lengths_every_threshold(sj, m, E):
    # without a length array the kernel keeps only the pattern ring in LDS
    # and computes the boundary masks from the positions (two wavefronts per
    # SIMD up to E = 22); ragged pair counts leave a partial last wavefront
    n = 2_500 + 3 * E + m if m < 1024 else 1_100
    p = syninput.generate(n, m, E=min(max(E, 1), 25), seed=9000 + 31 * m + E,
                          p_repeat=0.3 if m == 250 else 0.0)
    print("case no lengths n=%d m=%d E=%d" % (p.n, m, E), flush=True)
    ga, gp = _run(sj, p, E, m, with_lengths=False)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=E)
    bad = np.nonzero((ga != ea) | (gp != ep))[0]
    assert bad.size == 0, "mismatches at %s (gpu %s/%s oracle %s/%s)" % (
        bad[:8], ga[bad[:8]], gp[bad[:8]], ea[bad[:8]], ep[bad[:8]])
    # the same pairs with their (all equal) lengths passed: the other kernel
    la, lp = _run(sj, p, E, m, with_lengths=True)
    assert np.array_equal(la, ga) and np.array_equal(lp, gp)


def test_E_clamped_and_large(sj):
    p = syninput.generate(2_100, 20, E=3, seed=4)
    _check(sj, p, 19, 20)
    _check(sj, p, 500, 20)     # clamped to m-1 internally, decision uses E=500


def test_max_len_1024(sj):
    p = syninput.generate(2_500, 1000, 1024, E=10, seed=8)
    _check(sj, p, 10, 1024)


@pytest.mark.parametrize("E", [2, 20])
def test_invalid_lengths_get_sentinels(sj, E):
    # the valid pairs all have max_len bases: each group takes the one-length
    # path while its invalid pairs get the sentinels (E = 20: quarter layout)
    p = syninput.generate(3_000, 100, E=E, seed=3)
    p.lengths[::7] = 101
    p.lengths[3::11] = -5
    _check(sj, p, E, 100)


def test_identical_pairs(sj):
    p = syninput.generate(4_096, 150, E=6, seed=2)
    p.T[:] = p.P
    ga, gp = _run(sj, p, 6, 150)
    assert (gp == 0).all() and (ga == 1).all()


def test_deterministic(sj):
    p = syninput.config1(7, n=10_000)
    a1, p1 = _run(sj, p, 7, 100)
    a2, p2 = _run(sj, p, 7, 100)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_headline_full_size(sj):
    # m=100, E=5, 2M pairs: the bench's workload and launch, every output compared
    p = syninput.config1(5)
    _check(sj, p, 5, 100)


@pytest.mark.parametrize("E", list(range(0, 11)))
def test_config1_full_size(sj, E):
    # m=100, 2M pairs at every E of the sweep: every output against the oracle
    p = syninput.config1(E)
    _check(sj, p, E, 100)


@pytest.mark.parametrize("m,E", [(100, 0), (100, 5), (100, 10), (250, 15), (250, 22)])
def test_no_lengths_full_size_equals_lengths(sj, m, E):
    # 2M pairs: the ring-only kernel (no length array) against the kernel with
    # lengths, whose full-size outputs are checked against the oracle above
    p = syninput.generate(2_000_000, m, E=E, seed=9500 + E, p_repeat=0.3 if m == 250 else 0.0)
    print("case full size no lengths m=%d E=%d" % (m, E), flush=True)
    d = torch.device("cuda:0")
    reads = sj.pack_words_device(p.P, m)
    refs = sj.pack_words_device(p.T, m)
    lens = torch.from_numpy(p.lengths).to(d)
    a1, p1 = sj.shouji_filter(reads, refs, lens, E, max_len=m)
    a0, p0 = sj.shouji_filter(reads, refs, None, E, max_len=m)
    torch.cuda.synchronize()
    assert torch.equal(a0, a1) and torch.equal(p0, p1)
    # and the oracle on a strided sample
    idx = np.arange(0, p.n, 997)
    ea, ep = oracle.shouji_batch(p.P[idx], p.T[idx], p.lengths[idx], E=E)
    assert np.array_equal(a0.cpu().numpy()[idx], ea) and np.array_equal(p0.cpu().numpy()[idx], ep)


@pytest.mark.parametrize("E", [0, 5, 10, 15, 20, 25])
def test_config2_full_size(sj, E):
    # m=250, 2M pairs with tandem repeats, in one launch: every accept bit and
    # popcount against the oracle, and the properties that hold at any size
    # (decision = popcount <= E, popcount in [0, m], identical pairs have
    # popcount 0)
    p = syninput.config2(E)
    print("case config2 full n=%d E=%d" % (p.n, E), flush=True)
    ga, gp = _run(sj, p, E, 250)
    assert ((gp >= 0) & (gp <= 250)).all()
    assert np.array_equal(ga, (gp <= E).astype(np.uint8))
    same = (p.P == p.T).all(axis=1)
    assert (gp[same] == 0).all() and same.any()
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=E)
    bad = np.nonzero((ga != ea) | (gp != ep))[0]
    assert bad.size == 0, "%d mismatches, first at %s" % (bad.size, bad[:8])
    print("config2 E=%d: %d pairs compared, 0 mismatches" % (E, p.n), flush=True)


def test_empty_sequences(sj):
    # every pair of length 0 (max_len 0 and max_len 100), and max_len 0 with
    # no lengths: nothing to filter, popcount 0, accepted at every E
    d = torch.device("cuda:0")
    n = 3000
    for max_len in (0, 100):
        words = max(1, (max_len + 15) // 16)
        r = torch.zeros((words, n), dtype=torch.int32, device=d)
        L = torch.zeros(n, dtype=torch.int32, device=d)
        for E in (0, 3):
            print("case empty max_len=%d E=%d" % (max_len, E), flush=True)
            acc, pc = sj.shouji_filter(r, r, L, E, max_len=max_len)
            torch.cuda.synchronize()
            assert (acc.cpu().numpy() == 1).all() and (pc.cpu().numpy() == 0).all()
    r = torch.zeros((1, n), dtype=torch.int32, device=d)
    acc, pc = sj.shouji_filter(r, r, None, 2, max_len=0)
    torch.cuda.synchronize()
    assert (acc.cpu().numpy() == 1).all() and (pc.cpu().numpy() == 0).all()


def test_lengths_around_word_and_block_edges(sj):
    # lengths that end at and next to a 16-base word, an 8-window block and a
    # 16-window iteration (tail iterations of 1..8 windows, blocks of 2 and 4)
    for m in (1, 2, 3, 4, 5, 8, 9, 15, 16, 17, 18, 20, 24, 31, 32, 33, 34, 36, 40, 47, 48, 49, 97, 98, 99, 100,
              101, 104, 112, 113):
        p = syninput.generate(2_100, m, E=min(3, max(m - 1, 0)), seed=900 + m)
        for E in (0, 1, 5):
            _check(sj, p, E, m)


def test_no_lengths_around_word_and_block_edges(sj):
    # the kernel without a length array computes its boundary masks from the
    # positions: the same word, block and iteration edges as above, at
    # thresholds that clamp to m-1 for the shortest pairs
    for m in (1, 2, 3, 4, 5, 8, 9, 15, 16, 17, 18, 20, 24, 31, 32, 33, 34, 36, 40, 47, 48, 49, 97, 98, 99, 100,
              101, 104, 112, 113):
        p = syninput.generate(1_500, m, E=min(3, max(m - 1, 0)), seed=1900 + m)
        for E in (0, 1, 5, 20):
            _check(sj, p, E, m, with_lengths=False)


@pytest.mark.parametrize("E", [14, 20, 29, 30, 31])
def test_quarter_layout_edges(sj, E):
    # thresholds above 13 (with a length array) and above 22 (without) run the
    # layout of four 16-lane groups with iterations of 32 windows: lengths at
    # and next to those iterations' edges, a ragged wavefront (1,100 pairs),
    # thresholds that clamp to m-1 for short pairs
    for m in (1, 2, 3, 4, 31, 32, 33, 63, 64, 65, 96, 97, 250, 511, 512, 513, 1024):
        p = syninput.generate(1_100, m, E=min(E, max(m - 1, 0)), seed=5100 + m + 7 * E)
        for with_lengths in (True, False):
            _check(sj, p, E, m, with_lengths=with_lengths)


@pytest.mark.parametrize("E", [14, 23, 31])
def test_quarter_layout_mixed_lengths(sj, E):
    # mixed lengths inside every wavefront of 512 pairs: per-pair boundary
    # masks from the length planes
    p = syninput.generate(7_000, 40, 700, E=E, seed=5300 + E, p_repeat=0.3)
    _check(sj, p, E, 700)


@pytest.mark.parametrize("E", [3, 13, 14, 22, 31])
def test_one_length_below_max_len(sj, E):
    # wavefronts whose valid pairs share one length below max_len take their
    # boundary masks from the positions, bounded by that length: a group of
    # length m, a group of m and m-1 (per-pair masks), a ragged group of m-1,
    # in both layouts (E <= 13: 1,024 pairs per wavefront, above: 512)
    for m, max_len in ((90, 100), (33, 64), (200, 250)):
        p = syninput.generate(3_000, m, E=min(E, m - 1), seed=7000 + m + E)
        _check(sj, p, E, max_len)
        p.lengths[1536:] = m - 1
        _check(sj, p, E, max_len)


def test_concurrent_launches_share_the_pacing_table(sj):
    # launches on three streams at once, two in the quarter layout (whose
    # wavefronts post their progress in a table per SIMD and read their SIMD
    # neighbour's) and one in the two-half layout: the posts only steer issue
    # priority, so every output still equals the oracle's
    dev = torch.device("cuda:0")
    cases = [(syninput.generate(30_000, 250, E=20, seed=8100, p_repeat=0.3), 20, 250),
             (syninput.generate(30_000, 180, 250, E=25, seed=8101), 25, 250),
             (syninput.generate(30_000, 100, E=5, seed=8102), 5, 100)]
    prepared = []
    for p, E, max_len in cases:
        reads = torch.from_numpy(sj.pack_words(p.P, max_len)).to(dev)
        refs = torch.from_numpy(sj.pack_words(p.T, max_len)).to(dev)
        lens = torch.from_numpy(np.ascontiguousarray(p.lengths, dtype=np.int32)).to(dev)
        ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=E)
        prepared.append((reads, refs, lens, E, max_len, p.n, ea, ep))
    streams = [torch.cuda.Stream() for _ in cases]
    torch.cuda.synchronize()
    for rep in range(3):
        print("concurrent rep %d" % rep, flush=True)
        outs = []
        for st, (reads, refs, lens, E, max_len, n, _, _) in zip(streams, prepared):
            with torch.cuda.stream(st):
                outs.append(sj.shouji_filter(reads, refs, lens, E, n_pairs=n, max_len=max_len, stream=st))
        torch.cuda.synchronize()
        for (a, c), (_, _, _, E, _, _, ea, ep) in zip(outs, prepared):
            assert np.array_equal(a.cpu().numpy(), ea), "accept, E=%d rep %d" % (E, rep)
            assert np.array_equal(c.cpu().numpy(), ep), "popcount, E=%d rep %d" % (E, rep)


@pytest.mark.parametrize("seed", range(24))
def test_random_shapes(sj, seed):
    # random batch sizes, maximum lengths and thresholds, with four length
    # patterns: every pair max_len (also without the length array), one
    # length below max_len for all, one length per block of 512 pairs (each
    # wavefront's group of one length in either layout, a different one per
    # group), and lengths mixed inside every group
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(1, 5_000))
    max_len = int(rng.integers(1, 400))
    E = int(rng.integers(0, 32))
    pattern = seed % 4
    p = syninput.generate(n, max_len, E=min(E, max(max_len - 1, 0)), seed=9100 + seed)
    if pattern == 1:
        p.lengths[:] = int(rng.integers(0, max_len + 1))
    elif pattern == 2:
        for b in range(0, n, 512):
            p.lengths[b:b + 512] = int(rng.integers(0, max_len + 1))
    elif pattern == 3:
        p.lengths[:] = rng.integers(0, max_len + 1, n)
    print("case seed=%d n=%d max_len=%d E=%d pattern=%d" % (seed, n, max_len, E, pattern), flush=True)
    _check(sj, p, E, max_len)
    if pattern == 0:
        _check(sj, p, E, max_len, with_lengths=False)
