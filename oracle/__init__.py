"""CPU oracle for the Shouji pre-alignment filter -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the bench's CPU-baseline leg may import this
package; the product path (the HIP library and its binding) never does.  The
oracle works on base codes (uint8 0..3, one per base) and shares no code with
the GPU path.  See shouji_oracle.c for the steps and the readings it adopts,
levenshtein.c for the ground-truth edit distance.

Pinned by tests/test_oracle_pins.py (worked examples of Fig. 1 and Fig. 6,
proven invariants, an independent matrix-indexed implementation on tiny
inputs, and edit-distance closed forms).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

READING_B = 0   # adopted reading (global key: zeros, then leading zero, then scan order)
READING_A = 1   # sensitivity study only: main diagonal replaces on strictly more zeros

# counting modes of the last step (Sec. 2.2.3; Suppl. Sec. 8, Fig. 6(c))
GLOBAL = 0          # every one of S[0..m_T)
LOCAL = 1           # without the runs of ones before the first and after the last zero
GLOCAL_START = 2    # without the run of ones before the first zero
GLOCAL_END = 3      # without the run of ones after the last zero


CC = "gcc"
CFLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build():
    """Compile the oracle's C sources into _build/liboracle.so (gcc -O2, OpenMP)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call([CC] + CFLAGS +
                          [os.path.join(_HERE, "shouji_oracle.c"),
                           os.path.join(_HERE, "levenshtein.c"),
                           os.path.join(_HERE, "magnet_oracle.c"), "-o", tmp])
    os.replace(tmp, _SO)


def compiler():
    """The compiler and flags the oracle library is built with, e.g. for a
    benchmark record: 'gcc (Ubuntu 11.4.0-1ubuntu1~22.04) 11.4.0 -O2 -fopenmp ...'."""
    try:
        ver = subprocess.run([CC, "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        ver = CC
    return "%s %s" % (ver, " ".join(CFLAGS))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.oracle_shouji_pair.restype = ctypes.c_int
        lib.oracle_shouji_pair.argtypes = [vp, vp, i32, i32, i32, vp]
        lib.oracle_shouji_batch.restype = ctypes.c_int
        lib.oracle_shouji_batch.argtypes = [vp, vp, i64, vp, i64, i32, vp, i32, i32, vp, vp]
        lib.oracle_shouji_pair2.restype = ctypes.c_int
        lib.oracle_shouji_pair2.argtypes = [vp, i32, vp, i32, i32, i32, i32, vp]
        lib.oracle_shouji_batch2.restype = ctypes.c_int
        lib.oracle_shouji_batch2.argtypes = [vp, vp, i64, vp, vp, i64, i32, vp, i32, i32, vp, vp]
        lib.oracle_shouji_pair_w.restype = ctypes.c_int
        lib.oracle_shouji_pair_w.argtypes = [vp, vp, i32, i32, i32, vp]
        lib.oracle_shouji_batch_w.restype = ctypes.c_int
        lib.oracle_shouji_batch_w.argtypes = [vp, vp, i64, vp, i64, i32, i32, i32, vp, vp]
        lib.oracle_magnet_pair.restype = ctypes.c_int
        lib.oracle_magnet_pair.argtypes = [vp, vp, i32, i32, vp]
        lib.oracle_magnet_batch.restype = ctypes.c_int
        lib.oracle_magnet_batch.argtypes = [vp, vp, i64, vp, i64, i32, i32, vp, vp]
        lib.oracle_shouji_map_row.restype = ctypes.c_int
        lib.oracle_shouji_map_row.argtypes = [vp, vp, i32, i32, vp]
        lib.oracle_default_threads.restype = ctypes.c_int
        lib.oracle_edit_distance.restype = i32
        lib.oracle_edit_distance.argtypes = [vp, i32, vp, i32]
        lib.oracle_edit_distance_banded.restype = i32
        lib.oracle_edit_distance_banded.argtypes = [vp, i32, vp, i32, i32]
        lib.oracle_edit_distance_batch.restype = ctypes.c_int
        lib.oracle_edit_distance_batch.argtypes = [vp, vp, i64, vp, i64, vp, i32, vp]
        _lib = lib
    return _lib


_CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def codes(s):
    """ACGT string -> uint8 codes."""
    return np.frombuffer(bytes(_CODE[c] for c in s), dtype=np.uint8).copy()


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def shouji_pair(P, T, E, reading=READING_B):
    """Filter one pair (strings or code arrays).  Returns (popcount, S as '0'/'1' string)."""
    P = codes(P) if isinstance(P, str) else _c(P, np.uint8)
    T = codes(T) if isinstance(T, str) else _c(T, np.uint8)
    if len(P) != len(T):
        raise ValueError("global filtering needs equal lengths")
    m = len(T)
    S = np.zeros(max(m, 1), dtype=np.uint8)
    ones = _load().oracle_shouji_pair(P.ctypes.data, T.ctypes.data, m, int(E), reading, S.ctypes.data)
    if ones < 0:
        raise ValueError("bad arguments")
    return ones, "".join(str(int(b)) for b in S[:m])


def shouji_pair_w(P, T, E, W):
    """Filter one equal-length pair with W-column windows.  Returns (popcount, S string)."""
    P = codes(P) if isinstance(P, str) else _c(P, np.uint8)
    T = codes(T) if isinstance(T, str) else _c(T, np.uint8)
    if len(P) != len(T):
        raise ValueError("global filtering needs equal lengths")
    m = len(T)
    S = np.zeros(max(m, 1), dtype=np.uint8)
    ones = _load().oracle_shouji_pair_w(P.ctypes.data, T.ctypes.data, m, int(E), int(W), S.ctypes.data)
    if ones < 0:
        raise ValueError("bad arguments")
    return ones, "".join(str(int(b)) for b in S[:m])


def shouji_batch_w(P, T, lengths, E, W, nthreads=0):
    """Batch with W-column windows.  Returns (accept, popcount)."""
    P = _c(P, np.uint8)
    T = _c(T, np.uint8)
    L = _c(lengths, np.int32)
    n, stride = P.shape
    acc = np.empty(n, dtype=np.uint8)
    pc = np.empty(n, dtype=np.int16)
    rc = _load().oracle_shouji_batch_w(P.ctypes.data, T.ctypes.data, stride, L.ctypes.data, n, int(E), int(W),
                                       nthreads, acc.ctypes.data, pc.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return acc, pc


def magnet_pair(P, T, E):
    """MAGNET (Suppl. Sec. 7, Algorithms 3-4) on one equal-length pair.
    Returns (ones of the MAGNET bit-vector, the vector as a string)."""
    P = codes(P) if isinstance(P, str) else _c(P, np.uint8)
    T = codes(T) if isinstance(T, str) else _c(T, np.uint8)
    if len(P) != len(T):
        raise ValueError("MAGNET needs equal lengths")
    m = len(T)
    V = np.zeros(max(m, 1), dtype=np.uint8)
    ones = _load().oracle_magnet_pair(P.ctypes.data, T.ctypes.data, m, int(E), V.ctypes.data)
    if ones < 0:
        raise ValueError("bad arguments")
    return ones, "".join(str(int(b)) for b in V[:m])


def magnet_batch(P, T, lengths, E, nthreads=0):
    """MAGNET over a batch (rows of P and T, lengths[p] bases each).  Returns
    (accept, popcount) with the filter's sentinels for invalid lengths."""
    P = _c(P, np.uint8)
    T = _c(T, np.uint8)
    L = _c(lengths, np.int32)
    n, stride = P.shape
    acc = np.empty(n, dtype=np.uint8)
    pc = np.empty(n, dtype=np.int16)
    rc = _load().oracle_magnet_batch(P.ctypes.data, T.ctypes.data, stride, L.ctypes.data, n, int(E), nthreads,
                                     acc.ctypes.data, pc.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return acc, pc


def shouji_pair2(P, T, E, mode=GLOBAL, reading=READING_B):
    """Filter one pair of possibly different lengths (read P, reference T) with a
    counting mode.  Returns (count, S over the reference's positions as a string)."""
    P = codes(P) if isinstance(P, str) else _c(P, np.uint8)
    T = codes(T) if isinstance(T, str) else _c(T, np.uint8)
    mT = len(T)
    S = np.zeros(max(mT, 1), dtype=np.uint8)
    ones = _load().oracle_shouji_pair2(P.ctypes.data, len(P), T.ctypes.data, mT, int(E), int(mode),
                                       reading, S.ctypes.data)
    if ones < 0:
        raise ValueError("bad arguments")
    return ones, "".join(str(int(b)) for b in S[:mT])


def shouji_batch2(P, T, read_lengths, ref_lengths, E=None, E_per_pair=None, mode=GLOBAL, nthreads=0):
    """Batch of pairs with two lengths and a counting mode.  Returns (accept, count)."""
    P = _c(P, np.uint8)
    T = _c(T, np.uint8)
    if P.shape != T.shape:
        raise ValueError("P and T must share one [n, stride] shape")
    LP = _c(read_lengths, np.int32)
    LT = _c(ref_lengths, np.int32)
    n, stride = P.shape
    acc = np.empty(n, dtype=np.uint8)
    pc = np.empty(n, dtype=np.int16)
    Ep = None if E_per_pair is None else _c(E_per_pair, np.int32)
    rc = _load().oracle_shouji_batch2(P.ctypes.data, T.ctypes.data, stride, LP.ctypes.data, LT.ctypes.data,
                                      n, -1 if E is None else int(E),
                                      None if Ep is None else Ep.ctypes.data, int(mode), nthreads,
                                      acc.ctypes.data, pc.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return acc, pc


def map_row(P, T, d):
    """Diagonal d of the neighbourhood map as a '0'/'1' string over text columns 0..m-1."""
    P = codes(P) if isinstance(P, str) else _c(P, np.uint8)
    T = codes(T) if isinstance(T, str) else _c(T, np.uint8)
    m = len(T)
    out = np.zeros(max(m, 1), dtype=np.uint8)
    _load().oracle_shouji_map_row(P.ctypes.data, T.ctypes.data, m, int(d), out.ctypes.data)
    return "".join(str(int(b)) for b in out[:m])


def shouji_batch(P, T, lengths, E=None, E_per_pair=None, reading=READING_B, nthreads=0):
    """Filter n pairs given as code matrices [n, stride].  Returns (accept uint8, popcount int16)."""
    P = _c(P, np.uint8)
    T = _c(T, np.uint8)
    L = _c(lengths, np.int32)
    n, stride = P.shape
    acc = np.empty(n, dtype=np.uint8)
    pc = np.empty(n, dtype=np.int16)
    Ep = None if E_per_pair is None else _c(E_per_pair, np.int32)
    rc = _load().oracle_shouji_batch(P.ctypes.data, T.ctypes.data, stride, L.ctypes.data, n,
                                     -1 if E is None else int(E),
                                     None if Ep is None else Ep.ctypes.data,
                                     reading, nthreads, acc.ctypes.data, pc.ctypes.data)
    if rc != 0:
        raise ValueError("bad arguments")
    return acc, pc


def default_threads():
    return int(_load().oracle_default_threads())


def edit_distance(a, b):
    a = codes(a) if isinstance(a, str) else _c(a, np.uint8)
    b = codes(b) if isinstance(b, str) else _c(b, np.uint8)
    return int(_load().oracle_edit_distance(a.ctypes.data, len(a), b.ctypes.data, len(b)))


def edit_distance_banded(a, b, k):
    a = codes(a) if isinstance(a, str) else _c(a, np.uint8)
    b = codes(b) if isinstance(b, str) else _c(b, np.uint8)
    return int(_load().oracle_edit_distance_banded(a.ctypes.data, len(a), b.ctypes.data, len(b), int(k)))


def edit_distance_batch(P, T, lengths, k=None, k_per_pair=None):
    """Banded threshold labels: distance if <= k else -1, per pair."""
    P = _c(P, np.uint8)
    T = _c(T, np.uint8)
    L = _c(lengths, np.int32)
    n, stride = P.shape
    out = np.empty(n, dtype=np.int32)
    kp = None if k_per_pair is None else _c(k_per_pair, np.int32)
    _load().oracle_edit_distance_batch(P.ctypes.data, T.ctypes.data, stride, L.ctypes.data, n,
                                       None if kp is None else kp.ctypes.data,
                                       -1 if k is None else int(k), out.ctypes.data)
    return out
