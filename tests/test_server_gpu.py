"""GPU tests of the serving form: requests cut across batches and batches
shared by requests give the oracle's results bit-exactly; each request's
results are identical when served alone and inside a concurrent mix; invalid
pairs get the sentinels; the memory budget decides the number of batch slots."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import syninput

pytestmark = pytest.mark.gpu

MAX_LEN = 300


@pytest.fixture(scope="module")
def sj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_07858_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def work(sj):
    # mixed lengths 64..300, E_p = floor(r m) with r ~ U[0, 0.1]; references laid
    # out in a shuffled pool with gaps (unaligned offsets)
    p = syninput.generate(40_000, 64, MAX_LEN, E=None, r_max=0.10, seed=4000)
    codes, off = syninput.reference_pool(p, seed=4001, base_len=1000)
    pool = torch.from_numpy(sj.pack_pool(codes).view(np.int32)).to("cuda:0")
    reads = sj.pack_pairs(p.P, MAX_LEN)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    return dict(p=p, pool=pool, pool_bases=codes.size, off=off, reads=reads, ea=ea, ep=ep)


def _server(sj, w, **kw):
    return sj.Server(w["pool"], w["pool_bases"], MAX_LEN, **kw)


def _submit(srv, w, lo, hi):
    p = w["p"]
    return srv.submit(w["reads"][lo:hi], w["off"][lo:hi], p.lengths[lo:hi], p.E[lo:hi])


def _expect(w, lo, hi, acc, pc):
    ea, ep = w["ea"][lo:hi], w["ep"][lo:hi]
    bad = np.nonzero((acc != ea) | (pc != ep))[0]
    assert bad.size == 0, "range %d:%d mismatches at %s: server %s/%s oracle %s/%s" % (
        lo, hi, bad[:6], acc[bad[:6]], pc[bad[:6]], ea[bad[:6]], ep[bad[:6]])


def _cuts(n, sizes):
    out, lo = [], 0
    for s in sizes:
        if lo >= n:
            break
        out.append((lo, min(n, lo + s)))
        lo += s
    if lo < n:
        out.append((lo, n))
    return out


def test_requests_across_batches_match_oracle(sj, work):
    # batch capacity 4096: requests smaller than, equal to and larger than a
    # batch, so batches hold several requests and requests span batches
    n = work["p"].n
    cuts = _cuts(n, [1, 2, 17, 1000, 4095, 4096, 4097, 9000, 3, 250, 8192, 64])
    print("server: %d requests, batch 4096, 3 slots" % len(cuts), flush=True)
    with _server(sj, work, slots=3, max_batch_pairs=4096) as srv:
        tickets = [_submit(srv, work, lo, hi) for lo, hi in cuts]
        for (lo, hi), t in zip(cuts, tickets):
            acc, pc, ms = srv.wait(t)
            assert ms >= 0.0
            _expect(work, lo, hi, acc, pc)
        st = srv.stats()
    assert st["pairs_done"] == n and st["requests_done"] == len(cuts)
    assert st["batches"] >= (n + 4095) // 4096 and st["queued_pairs"] == 0


def test_alone_vs_mix_identical(sj, work):
    # each probe request is served alone on an idle server, then again inside
    # a mix of other requests submitted concurrently from three threads
    probes = [(100, 101), (2000, 2600), (10_000, 17_000), (30_000, 30_005), (5, 9000)]
    with _server(sj, work, slots=2, max_batch_pairs=8192) as srv:
        alone = []
        for lo, hi in probes:
            acc, pc, _ = srv.wait(_submit(srv, work, lo, hi))
            alone.append((acc.copy(), pc.copy()))
        results = {}
        errors = []

        def client(k):
            try:
                rng = np.random.default_rng(9 + k)
                local = []
                for i in range(12):
                    if i % 3 == 0:
                        j = (k + i // 3) % len(probes)
                        local.append(("probe", j, _submit(srv, work, *probes[j])))
                    lo = int(rng.integers(0, work["p"].n - 1))
                    hi = min(work["p"].n, lo + int(rng.integers(1, 6000)))
                    local.append(("other", (lo, hi), _submit(srv, work, lo, hi)))
                for kind, key, t in local:
                    acc, pc, _ = srv.wait(t)
                    if kind == "probe":
                        results.setdefault(key, []).append((acc, pc))
                    else:
                        _expect(work, key[0], key[1], acc, pc)
            except Exception as e:  # reported in the main thread
                errors.append(e)

        threads = [threading.Thread(target=client, args=(k,)) for k in range(3)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errors, errors
    assert results, "no probe request ran in the mix"
    for j, runs in results.items():
        lo, hi = probes[j]
        for acc, pc in runs:
            assert np.array_equal(acc, alone[j][0]) and np.array_equal(pc, alone[j][1])
        _expect(work, lo, hi, alone[j][0], alone[j][1])


def test_invalid_pairs_get_sentinels(sj, work):
    p = work["p"]
    lo, hi = 0, 3000
    offs = work["off"][lo:hi].copy()
    lens = p.lengths[lo:hi].copy()
    E = p.E[lo:hi].copy()
    offs[::37] = -5                                   # before the pool
    offs[1::41] = work["pool_bases"] + 3              # past the pool
    offs[2::43] = work["pool_bases"] - 10             # runs off the end
    lens[3::47] = MAX_LEN + 1                         # longer than max_len
    E[4::53] = -1                                     # negative threshold
    E[5::59] = 40                                     # clamped E above 31
    bad = np.zeros(hi - lo, dtype=bool)
    bad[::37] = True
    bad[1::41] = True
    bad[2::43] |= lens[2::43] > 10
    bad[3::47] = True
    bad[4::53] = True
    bad[5::59] |= np.minimum(40, lens[5::59] - 1) > 31
    with _server(sj, work, slots=1, max_batch_pairs=1024) as srv:
        acc, pc, _ = srv.wait(srv.submit(work["reads"][lo:hi], offs, lens, E))
    assert (acc[bad] == 0xFF).all() and (pc[bad] == -1).all()
    good = ~bad
    ea, ep = oracle.shouji_batch(p.P[lo:hi][good], p.T[lo:hi][good], lens[good], E_per_pair=E[good])
    assert np.array_equal(acc[good], ea) and np.array_equal(pc[good], ep)


def test_short_read_rows_and_empty_request(sj, work):
    # a request whose reads use fewer words than the server's max_len needs
    p = syninput.generate(5000, 20, 80, E=None, r_max=0.1, seed=77)
    codes, off = syninput.reference_pool(p, seed=78)
    pool = torch.from_numpy(sj.pack_pool(codes).view(np.int32)).to("cuda:0")
    reads = sj.pack_pairs(p.P, 80)                    # 5 words per read
    with sj.Server(pool, codes.size, MAX_LEN, slots=2, max_batch_pairs=2048) as srv:
        t0 = srv.submit(np.zeros((0, 5), np.uint32), np.zeros(0, np.int64), np.zeros(0, np.int32), 0)
        t1 = srv.submit(reads, off, p.lengths, p.E)
        a0, p0, _ = srv.wait(t0)
        acc, pc, _ = srv.wait(t1)
    assert a0.size == 0 and p0.size == 0
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    assert np.array_equal(acc, ea) and np.array_equal(pc, ep)


def test_memory_budget_sets_slots(sj, work):
    per = sj.server_slot_bytes(4096, MAX_LEN)
    with pytest.raises(sj.ShoujiError) as e:
        _server(sj, work, slots=4, max_batch_pairs=4096, memory_budget=per - 1)
    assert e.value.code == -5
    with _server(sj, work, slots=5, max_batch_pairs=4096, memory_budget=2 * per + 100) as srv:
        assert srv.stats()["slots"] == 2
        t = _submit(srv, work, 0, 20_000)
        acc, pc, _ = srv.wait(t)
    _expect(work, 0, 20_000, acc, pc)


def _pinned(a):
    t = torch.empty(a.shape, dtype=getattr(torch, {"uint32": "int32"}.get(a.dtype.name, a.dtype.name)),
                    pin_memory=True)
    v = t.numpy().view(a.dtype)
    v[...] = a
    return t, v


def test_pinned_and_pageable_requests_share_batches(sj, work):
    # pinned requests move by DMA in place, pageable ones through the staging
    # buffers; alternating them puts both kinds in the same batches
    p = work["p"]
    cuts = _cuts(p.n, [3000, 1, 2500, 777, 5000, 64, 4096, 12_000])
    keep = []
    with _server(sj, work, slots=2, max_batch_pairs=6000) as srv:
        tickets = []
        for i, (lo, hi) in enumerate(cuts):
            if i % 2 == 0:
                bufs = [_pinned(a) for a in (work["reads"][lo:hi], work["off"][lo:hi],
                                             p.lengths[lo:hi], p.E[lo:hi],
                                             np.zeros(hi - lo, np.uint8), np.zeros(hi - lo, np.int16))]
                keep.append(bufs)
                r, o, L, E, a, c = [v for _, v in bufs]
                tickets.append(srv.submit(r, o, L, E, pinned=True, out_accept=a, out_popcount=c))
            else:
                tickets.append(_submit(srv, work, lo, hi))
        for (lo, hi), t in zip(cuts, tickets):
            acc, pc, _ = srv.wait(t)
            _expect(work, lo, hi, acc, pc)
    with pytest.raises(ValueError):
        srv2 = _server(sj, work, slots=1, max_batch_pairs=64)
        try:
            srv2.submit(work["reads"][:4], work["off"][:4], p.lengths[:4], p.E[:4], pinned=True)
        finally:
            srv2.close()


def test_packed_reads_in_every_mix_of_formats(sj, work):
    # packed requests (pinned and pageable) are cut across batches at any
    # pair, and share batches with row requests (pinned and pageable)
    p = work["p"]
    words, wo = sj.pack_reads_packed(p.P, p.lengths, MAX_LEN)
    cuts = _cuts(p.n, [2500, 1, 7000, 333, 4096, 5000, 64, 9000, 3, 4095])
    keep = []
    print("server: packed and row requests, %d requests, batch 4096" % len(cuts), flush=True)
    with _server(sj, work, slots=2, max_batch_pairs=4096) as srv:
        tickets = []
        for i, (lo, hi) in enumerate(cuts):
            kind = i % 4
            if kind == 0:
                t = srv.submit(words[wo[lo]:wo[hi]], work["off"][lo:hi], p.lengths[lo:hi], p.E[lo:hi],
                               packed=True)
            elif kind == 2:
                t = _submit(srv, work, lo, hi)
            else:
                r = words[wo[lo]:wo[hi]] if kind == 1 else work["reads"][lo:hi]
                bufs = [_pinned(a) for a in (r, work["off"][lo:hi], p.lengths[lo:hi], p.E[lo:hi],
                                             np.zeros(hi - lo, np.uint8), np.zeros(hi - lo, np.int16))]
                keep.append(bufs)
                r, o, L, E, a, c = [v for _, v in bufs]
                t = srv.submit(r, o, L, E, pinned=True, packed=kind == 1, out_accept=a, out_popcount=c)
            tickets.append(t)
        for (lo, hi), t in zip(cuts, tickets):
            acc, pc, _ = srv.wait(t)
            _expect(work, lo, hi, acc, pc)
        st = srv.stats()
    assert st["pairs_done"] == p.n and st["queued_pairs"] == 0


def test_packed_reads_with_invalid_and_empty_lengths(sj, work):
    # a length outside [1, max_len] takes no words of the packed reads; the
    # pairs after it still find theirs
    p = work["p"]
    lo, hi = 0, 3000
    lens = p.lengths[lo:hi].copy()
    lens[3::47] = MAX_LEN + 1
    lens[4::53] = -2
    lens[5::59] = 0
    words, _ = sj.pack_reads_packed(p.P[lo:hi], lens, MAX_LEN)
    with _server(sj, work, slots=2, max_batch_pairs=1000) as srv:
        acc, pc, _ = srv.wait(srv.submit(words, work["off"][lo:hi], lens, p.E[lo:hi], packed=True))
        with pytest.raises(ValueError):
            srv.submit(words[:-1], work["off"][lo:hi], lens, p.E[lo:hi], packed=True)
        # the library's own check, past the binding's: a word count short of
        # what the lengths need is refused and nothing is queued
        import ctypes
        offs = np.ascontiguousarray(work["off"][lo:hi], dtype=np.int64)
        Ep = np.ascontiguousarray(p.E[lo:hi], dtype=np.int32)
        oa = np.empty(hi - lo, np.uint8)
        req = sj.Request(words.ctypes.data, 1, offs.ctypes.data, lens.ctypes.data, Ep.ctypes.data,
                         oa.ctypes.data, None, hi - lo, sj.REQUEST_PACKED, words.size - 1)
        t = ctypes.c_uint64()
        assert sj.lib().shouji_server_submit(srv._h, ctypes.byref(req), ctypes.byref(t)) == -2
        assert b"packed reads hold" in sj.lib().shouji_last_error()
        assert srv.stats()["queued_pairs"] == 0
    bad = (lens < 0) | (lens > MAX_LEN)
    assert (acc[bad] == 0xFF).all() and (pc[bad] == -1).all()
    good = ~bad
    ea, ep = oracle.shouji_batch(p.P[lo:hi][good], p.T[lo:hi][good], lens[good], E_per_pair=p.E[lo:hi][good])
    assert np.array_equal(acc[good], ea) and np.array_equal(pc[good], ep)


def test_many_tiny_requests_of_every_format(sj, work):
    # hundreds of 1..40-pair requests per batch, in every request format:
    # small pinned parts are staged like pageable ones, large ones go by DMA
    p = work["p"]
    words, wo = sj.pack_reads_packed(p.P, p.lengths, MAX_LEN)
    rng = np.random.default_rng(4100)
    sizes = [int(s) for s in rng.integers(1, 41, 600)] + [2048, 5000]
    cuts = _cuts(p.n, sizes)[:len(sizes)]
    keep = []
    print("server: %d tiny requests, batch 4096" % len(cuts), flush=True)
    with _server(sj, work, slots=3, max_batch_pairs=4096) as srv:
        tickets = []
        for i, (lo, hi) in enumerate(cuts):
            kind = i % 4
            if kind == 0:
                t = srv.submit(words[wo[lo]:wo[hi]], work["off"][lo:hi], p.lengths[lo:hi], p.E[lo:hi],
                               packed=True)
            elif kind == 2:
                t = _submit(srv, work, lo, hi)
            else:
                r = words[wo[lo]:wo[hi]] if kind == 1 else work["reads"][lo:hi]
                bufs = [_pinned(a) for a in (r, work["off"][lo:hi], p.lengths[lo:hi], p.E[lo:hi],
                                             np.zeros(hi - lo, np.uint8), np.zeros(hi - lo, np.int16))]
                keep.append(bufs)
                r, o, L, E, a, c = [v for _, v in bufs]
                t = srv.submit(r, o, L, E, pinned=True, packed=kind == 1, out_accept=a, out_popcount=c)
            tickets.append(t)
        for (lo, hi), t in zip(cuts, tickets):
            acc, pc, _ = srv.wait(t)
            _expect(work, lo, hi, acc, pc)


def test_longest_reads(sj):
    # max_len 1024 (64-word rows), lengths 500..1024, E_p up to 31, packed and
    # row requests in the same batches
    p = syninput.generate(2_000, 500, 1024, E=None, r_max=0.031, seed=4200)
    codes, off = syninput.reference_pool(p, seed=4201, base_len=1000)
    pool = torch.from_numpy(sj.pack_pool(codes).view(np.int32)).to("cuda:0")
    rows = sj.pack_pairs(p.P, 1024)
    words, wo = sj.pack_reads_packed(p.P, p.lengths, 1024)
    ea, ep = oracle.shouji_batch(p.P, p.T, p.lengths, E_per_pair=p.E)
    with sj.Server(pool, codes.size, 1024, slots=2, max_batch_pairs=700) as srv:
        t0 = srv.submit(words[wo[0]:wo[1000]], off[:1000], p.lengths[:1000], p.E[:1000], packed=True)
        t1 = srv.submit(rows[1000:], off[1000:], p.lengths[1000:], p.E[1000:])
        a0, c0, _ = srv.wait(t0)
        a1, c1, _ = srv.wait(t1)
    acc, pc = np.concatenate([a0, a1]), np.concatenate([c0, c1])
    assert np.array_equal(acc, ea) and np.array_equal(pc, ep)


def test_fill_wait_trickled_stream(sj, work):
    # requests trickle in while batches are in flight: with a fill wait a free
    # slot holds a part-filled batch for more requests (never with nothing in
    # flight); every result is the same.  The batch counts depend on host
    # timing and are printed, not compared
    import time
    cuts = _cuts(12_000, [150] * 80)
    batches = {}
    for wait in (0, 3000):
        print("server: %d trickled requests, fill_wait_us %d" % (len(cuts), wait), flush=True)
        with _server(sj, work, slots=2, max_batch_pairs=4096, fill_wait_us=wait) as srv:
            tickets = []
            for lo, hi in cuts:
                tickets.append(_submit(srv, work, lo, hi))
                time.sleep(0.0002)
            for (lo, hi), t in zip(cuts, tickets):
                acc, pc, ms = srv.wait(t)
                assert ms >= 0.0
                _expect(work, lo, hi, acc, pc)
            st = srv.stats()
        assert st["pairs_done"] == 12_000 and st["queued_pairs"] == 0
        batches[wait] = st["batches"]
    print("batches:", batches, flush=True)
