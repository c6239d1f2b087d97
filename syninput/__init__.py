"""Seeded synthetic read/reference pairs shaped like the paper's workloads.

This module is shared by the CPU oracle's tests and the GPU path's tests and
bench.  It holds no step of the filter: only random sequences, tandem repeats
and random edits (see gen.c for the recipe).  The paper's real datasets
(Sec. 3.1, Tables 5-8: 30 M mrFAST candidate pairs per set, read lengths 100,
150 and 250) are stood in for by these inputs.

Base codes are uint8 0..3; rows are padded with zeros to `stride` codes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libsyngen.so")
_lib = None


def build():
    """Compile gen.c into _build/libsyngen.so (gcc, OpenMP)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           os.path.join(_HERE, "gen.c"), "-o", tmp, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.syn_generate.restype = ctypes.c_int
        lib.syn_generate.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p]
        lib.syn_pool.restype = ctypes.c_int
        lib.syn_pool.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


class Pairs:
    """A batch of pairs: P (reads), T (references) as uint8 codes [n, stride]."""

    def __init__(self, P, T, lengths, E):
        self.P, self.T, self.lengths, self.E = P, T, lengths, E

    @property
    def n(self):
        return int(self.lengths.shape[0])

    def slice(self, lo, hi):
        return Pairs(self.P[lo:hi], self.T[lo:hi], self.lengths[lo:hi], self.E[lo:hi])


def generate(n, m_min, m_max=None, E=None, r_max=0.10, seed=0, p_unrelated=0.2,
             p_repeat=0.0, stride=None):
    """Generate n pairs.  E fixed (int) or None for per-pair E_p = floor(r*m), r~U[0,r_max]."""
    m_max = m_min if m_max is None else m_max
    stride = m_max if stride is None else stride
    P = np.zeros((n, stride), dtype=np.uint8)
    T = np.zeros((n, stride), dtype=np.uint8)
    L = np.zeros(n, dtype=np.int32)
    Ep = np.zeros(n, dtype=np.int32)
    rc = _load().syn_generate(seed, n, m_min, m_max, stride, -1 if E is None else int(E),
                              float(r_max), float(p_unrelated), float(p_repeat),
                              P.ctypes.data, T.ctypes.data, L.ctypes.data, Ep.ctypes.data)
    if rc != 0:
        raise ValueError("syn_generate rejected its arguments")
    return Pairs(P, T, L, Ep)


def pool(length, seed=0):
    """A pool of `length` uniform random base codes."""
    out = np.empty(length, dtype=np.uint8)
    if _load().syn_pool(seed, length, out.ctypes.data) != 0:
        raise ValueError("bad pool length")
    return out


# Workload presets (sizes from the benchmark configurations; seeds fixed).
def config0():
    """10,000 pairs, m=100, E=2, 20% unrelated, seed 0."""
    return generate(10_000, 100, E=2, seed=0)


def config1(E, n=2_000_000):
    """m=100, threshold E in 0..10, edits k~U{0..2E}, 20% unrelated, seed 1000+E."""
    return generate(n, 100, E=E, seed=1000 + E)


def config2(E, n=2_000_000):
    """m=250, E in {0,5,...,25}, 30% of reads with a tandem repeat, seed 2000+E."""
    return generate(n, 250, E=E, seed=2000 + E, p_repeat=0.3)


def config3(n=8_000_000):
    """Mixed lengths 64..300, per-pair E_p=floor(r*m) with r~U[0,0.10], seed 3000."""
    return generate(n, 64, 300, E=None, r_max=0.10, seed=3000)


def reference_pool(pairs, seed=0, max_gap=7, base_len=0):
    """Lay the references of `pairs` out in one flat pool of base codes.

    The segments go into the pool in a seeded random order, separated by gaps of
    0..max_gap uniform random bases, after `base_len` leading random bases.
    Returns (pool codes uint8 [L], offsets int64 [n]): pair p's reference is
    pool[offsets[p] : offsets[p] + lengths[p]].
    """
    rng = np.random.default_rng(seed)
    n = pairs.n
    order = rng.permutation(n)
    gaps = rng.integers(0, max_gap + 1, n)
    lens = pairs.lengths.astype(np.int64)
    step = gaps + lens[order]
    starts_in_order = base_len + np.cumsum(step) - lens[order]
    offsets = np.empty(n, dtype=np.int64)
    offsets[order] = starts_in_order
    total = int(base_len + step.sum() + max_gap)
    out = pool(total, seed=seed + 1)
    stride = pairs.T.shape[1]
    cols = np.arange(stride)
    chunk = 1 << 16
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        mask = cols[None, :] < pairs.lengths[lo:hi, None]
        pos = offsets[lo:hi, None] + cols[None, :]
        out[pos[mask]] = pairs.T[lo:hi][mask]
    return out, offsets
