"""GPU parity of the batched form (mixed lengths, one threshold per pair):
bit-exact against the CPU oracle, equal to the plain form, identical for
every tuning config, and stable under graph capture and replay."""
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
            torch.from_numpy(np.ascontiguousarray(p.lengths, dtype=np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(p.E, dtype=np.int32)).to(d))


def _check(sj, p, max_len, config=None):
    print("batched n=%d max_len=%d config=%s" % (p.n, max_len, config), flush=True)
    r, t, L, E = _dev(sj, p, max_len)
    acc, pc = sj.shouji_filter_batched(r, t, L, E, max_len=max_len, config=config)
    torch.cuda.synchronize()
    ga, gp = acc.cpu().numpy(), pc.cpu().numpy()
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    bad = np.nonzero((ga != ea) | (gp != ep))[0]
    assert bad.size == 0, "mismatches at %s: gpu %s/%s oracle %s/%s (m %s E %s)" % (
        bad[:6], ga[bad[:6]], gp[bad[:6]], ea[bad[:6]], ep[bad[:6]], p.lengths[bad[:6]], p.E[bad[:6]])
    return ga, gp


def test_mixed_lengths_per_pair_E(sj):
    # lengths 64..300, E_p = floor(r m), r ~ U[0, 0.1]: the mixed workload shape
    p = syninput.generate(60_000, 64, 300, E=None, r_max=0.10, seed=3000)
    _check(sj, p, 300)


@pytest.mark.parametrize("config", [None, (4, 2)])
def test_longest_lengths_and_largest_thresholds(sj, config):
    # lengths 500..1024 (up to 64 words) with E_p up to 31: every bin of the
    # E > 13 class and the largest length buckets.  Bin width 4 gives the
    # most bins (8,224): one histogram copy per workgroup, and more bins than
    # the LDS-staged scatter holds, so the direct scatter runs
    p = syninput.generate(3_000, 500, 1024, E=None, r_max=0.031, seed=3100)
    assert p.E.max() >= 25 and p.lengths.max() > 1000
    _check(sj, p, 1024, config=config)


@pytest.mark.parametrize("max_len", [216, 220, 728, 732])
def test_bin_counts_at_the_staged_scatter_limits(sj, max_len):
    # bin width 4: (ceil(max_len/4) + 1) * 32 bins = 1,760 / 1,792 / 5,856 /
    # 5,888, on both sides of what the staged scatter holds beside its scan's
    # static LDS with chunks of 16,384 pairs (1,791 bins) and of 8,192 (5,887)
    p = syninput.generate(4_000, max_len - 60, max_len, E=None, r_max=min(0.10, 31.0 / max_len),
                          seed=3200 + max_len)
    assert p.E.max() <= 31
    _check(sj, p, max_len, config=(4, 2))


@pytest.mark.parametrize("config", [(4, 2), (8, 4), (16, 1), (32, 4)])
def test_every_config_exact(sj, config):
    p = syninput.generate(20_000, 30, 200, E=None, r_max=0.15, seed=31)
    _check(sj, p, 200, config=config)


def test_short_lengths_large_E_and_sentinels(sj):
    p = syninput.generate(12_000, 0, 48, E=None, r_max=0.9, seed=7)
    p.E[::13] = -1                    # invalid threshold
    p.E[5::17] = 40                   # clamps to m-1 (<= 47): large but valid only if <= 31
    p.lengths[3::19] = 49             # beyond max_len
    r, t, L, E = _dev(sj, p, 48)
    acc, pc = sj.shouji_filter_batched(r, t, L, E, max_len=48)
    torch.cuda.synchronize()
    ga, gp = acc.cpu().numpy(), pc.cpu().numpy()
    Eeff = np.minimum(p.E, np.maximum(p.lengths - 1, 0))
    invalid = (p.E < 0) | (p.lengths > 48) | (Eeff > 31)
    assert (ga[invalid] == 0xFF).all() and (gp[invalid] == -1).all()
    ok = ~invalid
    ea, ep = oracle.shouji_batch(p.P[ok], p.T[ok], p.lengths[ok], E_per_pair=p.E[ok])
    assert np.array_equal(ga[ok], ea) and np.array_equal(gp[ok], ep)


def test_equals_plain_for_uniform_E(sj):
    p = syninput.generate(30_000, 100, E=6, seed=66)
    r, t, L, E = _dev(sj, p, 100)
    ba, bp = sj.shouji_filter_batched(r, t, L, E, max_len=100)
    pa, pp = sj.shouji_filter(r, t, L, 6, max_len=100)
    torch.cuda.synchronize()
    assert torch.equal(ba, pa) and torch.equal(bp, pp)


def test_tiny_batches(sj):
    for n in (1, 2, 1023, 1025):
        p = syninput.generate(n, 64, 300, E=None, seed=n)
        _check(sj, p, 300)


def test_autotuner_returns_a_config(sj):
    p = syninput.generate(50_000, 64, 300, E=None, seed=3)
    r, t, L, E = _dev(sj, p, 300)
    (bw, wpg), ms = sj.tune_batched(r, t, L, E, max_len=300)
    assert bw in (4, 8, 16, 32) and wpg in (1, 2, 4) and ms > 0
    _check(sj, p, 300)               # config None now uses the tuned choice


def test_graph_capture_replays(sj):
    p = syninput.generate(40_000, 64, 300, E=None, seed=99)
    r, t, L, E = _dev(sj, p, 300)
    ws = torch.empty(sj.batched_workspace_bytes(p.n, 300), dtype=torch.uint8, device="cuda:0")
    acc = torch.empty(p.n, dtype=torch.uint8, device="cuda:0")
    pc = torch.empty(p.n, dtype=torch.int16, device="cuda:0")
    ref_a, ref_p = sj.shouji_filter_batched(r, t, L, E, max_len=300, workspace=ws)
    ref_a, ref_p = ref_a.clone(), ref_p.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up on the capture stream
        sj.shouji_filter_batched(r, t, L, E, acc, pc, max_len=300, workspace=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sj.shouji_filter_batched(r, t, L, E, acc, pc, max_len=300, workspace=ws,
                                 stream=torch.cuda.current_stream())
    for it in range(3):
        acc.fill_(7)
        pc.fill_(-7)
        junk = torch.randn(1000, device="cuda:0").sum()   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(acc, ref_a) and torch.equal(pc, ref_p), "replay %d" % it
        del junk


def test_full_size(sj):
    # the full mixed workload: 8M pairs, lengths 64..300, E_p = floor(r m),
    # unsorted, in one call with the tuned configuration: every accept bit and
    # popcount against the oracle, and on every pair accept = popcount <= E_p,
    # popcount in [0, m]
    p = syninput.config3()
    max_len = 300
    print("batched full n=%d" % p.n, flush=True)
    d = torch.device("cuda:0")
    r = sj.pack_words_device(p.P, max_len)
    t = sj.pack_words_device(p.T, max_len)
    L = torch.from_numpy(p.lengths).to(d)
    E = torch.from_numpy(p.E).to(d)
    acc, pc = sj.shouji_filter_batched(r, t, L, E, max_len=max_len)
    torch.cuda.synchronize()
    ga, gp = acc.cpu().numpy(), pc.cpu().numpy().astype(np.int32)
    del r, t
    assert ((gp >= 0) & (gp <= p.lengths)).all()
    assert np.array_equal(ga, (gp <= p.E).astype(np.uint8))
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    bad = np.nonzero((ga != ea) | (gp != ep))[0]
    assert bad.size == 0, "%d mismatches, first at %s" % (bad.size, bad[:8])
    print("batched full: %d pairs compared, 0 mismatches" % p.n, flush=True)


def test_no_lengths_per_pair_E(sj):
    # lengths = NULL: every pair has max_len bases; per-pair thresholds across
    # both E classes and a ragged pair count
    p = syninput.generate(5_003, 150, E=None, r_max=0.2, seed=3200)
    assert (p.lengths == 150).all() and p.E.max() > 13
    d = torch.device("cuda:0")
    r = torch.from_numpy(sj.pack_words(p.P, 150)).to(d)
    t = torch.from_numpy(sj.pack_words(p.T, 150)).to(d)
    E = torch.from_numpy(p.E).to(d)
    print("batched no lengths n=%d" % p.n, flush=True)
    acc, pc = sj.shouji_filter_batched(r, t, None, E, max_len=150)
    torch.cuda.synchronize()
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)
