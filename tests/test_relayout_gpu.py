"""Relayout of pair-major 64-bit words into the filters' layout (shouji_relayout_pair_major)."""
import numpy as np
import pytest
import torch

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


@pytest.mark.parametrize("n,m,max_len,extra_words,ld", [
    (3_000, 100, 100, 0, None), (3_000, 100, 128, 2, 3_333), (1, 1, 1, 0, None), (1_025, 250, 250, 1, None),
    (777, 33, 48, 0, 800), (4_096, 300, 300, 0, None), (257, 1024, 1024, 3, None)])
def test_relayout_equals_the_host_packer(sj, n, m, max_len, extra_words, ld):
    print("case n=%d m=%d max_len=%d extra=%d ld=%s" % (n, m, max_len, extra_words, ld), flush=True)
    rng = np.random.default_rng(n + m)
    codes = rng.integers(0, 4, size=(n, m), dtype=np.uint8)
    pm = sj.pack_pair_major(codes, max_len, words_per_seq=(max_len + 31) // 32 + extra_words)
    src = torch.from_numpy(pm.view(np.int64)).cuda()
    out = sj.relayout_pair_major(src, max_len, ld=ld)
    torch.cuda.synchronize()
    want = sj.pack_words(codes, max_len, ld=ld)
    assert np.array_equal(out.cpu().numpy(), want)


def test_filter_on_relayout_matches_the_oracle(sj):
    p = syninput.generate(5_000, 100, E=5, seed=77)
    reads = sj.relayout_pair_major(torch.from_numpy(sj.pack_pair_major(p.P, 100).view(np.int64)).cuda(), 100)
    refs = sj.relayout_pair_major(torch.from_numpy(sj.pack_pair_major(p.T, 100).view(np.int64)).cuda(), 100)
    lens = torch.from_numpy(p.lengths).cuda()
    acc, pc = sj.shouji_filter(reads, refs, lens, 5, max_len=100)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E=5)
    assert np.array_equal(acc.cpu().numpy(), ea) and np.array_equal(pc.cpu().numpy(), ep)
