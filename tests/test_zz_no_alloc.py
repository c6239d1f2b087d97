"""GPU test of shouji_filter_batched_noalloc: the batched form with the
library's own scratch array in place of a caller workspace gives, through the
C ABI, exactly the outputs of shouji_filter_batched with a workspace, on two
calls in a row (the second smaller, so that it runs on scratch the first call
left filled)."""
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


def _inputs(sj, n, seed, max_len=300):
    p = syninput.generate(n, 64, max_len, E=None, r_max=0.10, seed=seed)
    d = torch.device("cuda:0")
    return p, (sj.pack_words_device(p.P, max_len), sj.pack_words_device(p.T, max_len),
               torch.from_numpy(p.lengths).to(d), torch.from_numpy(p.E).to(d))


def test_noalloc_equals_workspace_form_on_two_calls(sj):
    max_len = 300
    for n, seed in ((700_000, 3600), (45_001, 3601)):
        print("noalloc n=%d seed=%d" % (n, seed), flush=True)
        p, (r, t, L, E) = _inputs(sj, n, seed, max_len)
        assert sj.batched_workspace_bytes(n, max_len) <= sj.NOALLOC_SCRATCH_BYTES
        d = r.device
        a0 = torch.full((n,), 0xEE, dtype=torch.uint8, device=d)
        c0 = torch.full((n,), -7, dtype=torch.int16, device=d)
        sj.shouji_filter_batched_noalloc(r, t, L, E, a0, c0, max_len=max_len)
        a1, c1 = sj.shouji_filter_batched(r, t, L, E, max_len=max_len)
        torch.cuda.synchronize()
        assert torch.equal(a0, a1) and torch.equal(c0, c1)
        if n < 100_000:
            ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
            assert np.array_equal(a0.cpu().numpy(), ea) and np.array_equal(c0.cpu().numpy(), ep)
