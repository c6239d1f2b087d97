"""Host-side checks of the C ABI library (no GPU needed: no kernel is launched)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1809_07858_amd as sj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names.update(re.findall(r"\b(shouji_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = sj.lib()
    names = _declared_symbols()
    assert "shouji_filter" in names
    for name in names:
        assert hasattr(L, name), name


def test_version_and_empty_error():
    assert sj.lib().shouji_version() >= 10000


def _call(**kw):
    a = dict(reads=ctypes.c_void_p(16), refs=ctypes.c_void_p(16), lengths=None, E=2,
             out_accept=ctypes.c_void_p(16), out_popcount=None, n_pairs=10, max_len=100,
             ld=10, stream=None)
    a.update(kw)
    return sj.lib().shouji_filter(a["reads"], a["refs"], a["lengths"], a["E"], a["out_accept"],
                                  a["out_popcount"], a["n_pairs"], a["max_len"], a["ld"], a["stream"])


def test_argument_errors_are_reported_before_launch():
    assert _call(n_pairs=-1) == -2
    assert _call(E=-1) == -2
    assert _call(max_len=2000) == -3
    assert _call(max_len=-1) == -3
    assert _call(E=40, max_len=100) == -3          # clamped E still above 31
    assert _call(reads=None) == -1
    assert _call(out_accept=None) == -1
    assert _call(ld=5) == -2
    assert b"ld" in sj.lib().shouji_last_error()
    # zero pairs is a successful no-op, even with NULL pointers
    assert _call(n_pairs=0, reads=None, refs=None, out_accept=None) == 0
    assert sj.lib().shouji_last_error() == b""


def test_pack_words_layout():
    rng = np.random.default_rng(0)
    codes = rng.integers(0, 4, (37, 50)).astype(np.uint8)
    w = sj.pack_words(codes, 50, ld=40).view(np.uint32)
    assert w.shape == (4, 40)
    for p in range(37):
        for j in range(50):
            assert (int(w[j // 16, p]) >> (2 * (j % 16))) & 3 == codes[p, j]
    assert (w[:, 37:] == 0).all()
    assert (w[3, :37] >> 4 == 0).all()   # bases 50..63 of the last word are zero


def test_server_argument_errors_are_reported_without_a_device():
    L = sj.lib()
    h = ctypes.c_void_p()
    assert L.shouji_server_create(None, ctypes.byref(h)) == -1
    cfg = sj.ServerConfig(None, 1000, 100, 2, 1024, 0, 0)
    assert L.shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -2      # no pool
    cfg = sj.ServerConfig(16, 1000, 2000, 2, 1024, 0, 0)
    assert L.shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -3      # max_len
    cfg = sj.ServerConfig(16, 1000, 100, 0, 1024, 0, 0)
    assert L.shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -2      # slots
    assert b"slots" in L.shouji_last_error()
    cfg = sj.ServerConfig(16, 1000, 300, 2, 1 << 40, 0, 0)
    assert L.shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -3      # batch words
    for wait in (-1, 1000001):
        cfg = sj.ServerConfig(16, 1000, 100, 2, 1024, 0, 0, wait)
        assert L.shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -3  # fill wait
        assert b"fill_wait_us" in L.shouji_last_error()
    assert ctypes.sizeof(sj.ServerConfig) == 48
    t = ctypes.c_uint64()
    assert L.shouji_server_submit(None, None, ctypes.byref(t)) == -1
    assert L.shouji_server_wait(None, 1, None) == -1
    assert L.shouji_server_destroy(None) == 0
    assert sj.server_slot_bytes(1 << 20, 300) > (1 << 20) * 19 * 4 * 3
    with pytest.raises(sj.ShoujiError):
        sj.server_slot_bytes(0, 300)
    with pytest.raises(sj.ShoujiError):
        sj.server_slot_bytes(100, 5000)


def test_pool_and_pair_packing_layout():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 4, (7, 45), dtype=np.uint8)
    pp = sj.pack_pairs(c, 45)
    assert pp.shape == (7, 3) and pp.dtype == np.uint32
    flat = c.ravel()
    pool = sj.pack_pool(flat)
    for b in range(flat.size):
        assert (int(pool[b // 16]) >> (2 * (b % 16))) & 3 == flat[b]
    for p in range(7):
        for j in range(45):
            assert (int(pp[p, j // 16]) >> (2 * (j % 16))) & 3 == c[p, j]


def test_packed_read_layout():
    # reads back to back, ceil(m/16) words each, none for a length outside
    # [1, max_len]; read p is the first words of its row in the row layout
    rng = np.random.default_rng(2)
    c = rng.integers(0, 4, (9, 70), dtype=np.uint8)
    lens = np.array([70, 1, 16, 17, 0, -3, 71, 33, 48], dtype=np.int32)
    words, off = sj.pack_reads_packed(c, lens, 70)
    k = [5, 1, 1, 2, 0, 0, 0, 3, 3]
    assert list(np.diff(off)) == k and off[0] == 0 and words.size == sum(k)
    assert words.dtype == np.uint32
    rows = sj.pack_pairs(c, 70)
    for p in range(9):
        assert np.array_equal(words[off[p]:off[p + 1]], rows[p, :k[p]])
    assert list(sj.packed_read_words(lens, 70)) == k


def test_batched_pair_count_limit():
    # the binning indexes pairs in 32 bits: above 2^31 - 1 pairs the batched
    # form refuses the call before anything is enqueued
    L = sj.lib()
    big = 1 << 31
    assert L.shouji_batched_workspace_bytes(big, 300) == -3
    assert b"limit" in L.shouji_last_error()
    assert L.shouji_batched_workspace_bytes(big - 1, 16) > 0
    vp = ctypes.c_void_p(16)
    rc = L.shouji_filter_batched(vp, vp, None, vp, vp, None, big, 300, big, vp, 1 << 40, None, None)
    assert rc == -3


def test_request_struct_carries_the_packed_word_count():
    # read_words sits after flags (8-byte aligned): the struct is 80 bytes
    assert sj.Request.flags.offset == 64
    assert sj.Request.read_words.offset == 72
    assert ctypes.sizeof(sj.Request) == 80


def test_noalloc_batched_refuses_sizes_beyond_its_scratch():
    # sizes are checked before the device is touched: more pairs than the
    # library's scratch array holds is SHOUJI_ERR_RANGE, naming the limit
    L = sj.lib()
    vp = ctypes.c_void_p(16)
    n = 2_000_000
    assert sj.batched_workspace_bytes(n, 300) > sj.NOALLOC_SCRATCH_BYTES
    assert L.shouji_filter_batched_noalloc(vp, vp, None, vp, vp, None, n, 300, n, None, None) == -3
    assert b"scratch" in L.shouji_last_error()
    assert L.shouji_filter_batched_noalloc(vp, vp, None, vp, vp, None, -1, 300, 0, None, None) == -2
    assert L.shouji_filter_batched_noalloc(vp, vp, None, vp, vp, None, 10, 5000, 10, None, None) == -3
    assert L.shouji_filter_batched_noalloc(None, None, None, None, None, None, 0, 300, 0, None, None) == 0


def _relayout(**kw):
    a = dict(src=ctypes.c_void_p(16), wps=4, n=10, max_len=100, dst=ctypes.c_void_p(16), ld=10, stream=None)
    a.update(kw)
    return sj.lib().shouji_relayout_pair_major(a["src"], a["wps"], a["n"], a["max_len"], a["dst"], a["ld"],
                                               a["stream"])


def test_relayout_argument_errors_are_reported_before_launch():
    assert _relayout(wps=3) == -2                  # 100 bases need 4 words of 32
    assert b"words_per_seq" in sj.lib().shouji_last_error()
    assert _relayout(n=-1) == -2
    assert _relayout(max_len=2000) == -3
    assert _relayout(src=None) == -1
    assert _relayout(dst=None) == -1
    assert _relayout(ld=9) == -2
    assert _relayout(n=0, src=None, dst=None) == 0  # nothing to do
    assert _relayout(max_len=0, wps=0, src=None, dst=None) == 0


def test_pair_major_words_are_two_rows_of_the_filter_layout():
    # a 64-bit word w of a pair (32 bases) is rows 2w (low half) and 2w+1 (high
    # half) of the word-major 16-base layout: the relayout's expected output
    rng = np.random.default_rng(5)
    for m, max_len in ((100, 100), (33, 64), (250, 300), (16, 16), (1, 1)):
        codes = rng.integers(0, 4, size=(37, m), dtype=np.uint8)
        pm = sj.pack_pair_major(codes, max_len)
        assert pm.shape == (37, (max_len + 31) // 32) and pm.dtype == np.uint64
        wm = sj.pack_words(codes, max_len).view(np.uint32)
        nr = wm.shape[0]
        for r in range(nr):
            half = (pm[:, r // 2] >> np.uint64(32 * (r % 2))) & np.uint64(0xFFFFFFFF)
            assert np.array_equal(half.astype(np.uint32), wm[r])
        # rows past ceil(max_len/16) are zero in the last 64-bit word
        if nr % 2:
            assert not np.any(pm[:, -1] >> np.uint64(32))
    # base j of a sequence: bits 2(j%32).. of word j/32
    codes = np.zeros((1, 64), dtype=np.uint8)
    codes[0, 33] = 3
    assert sj.pack_pair_major(codes)[0, 1] == np.uint64(3 << 2)
