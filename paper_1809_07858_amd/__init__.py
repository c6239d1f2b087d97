"""MI355X Shouji pre-alignment filter: thin Python binding over libshouji.so.

Every step of the filter runs in the HIP kernels behind the C ABI declared in
include/shouji.h; this module only marshals arguments (device pointers of
torch tensors, the current HIP stream).  It fails loudly when the library is
not built -- there is no CPU fallback.

Device layout (see include/shouji.h): sequences 2-bit packed, 16 bases per
32-bit word, word-major (word w of pair p at [w, p] of an [nwords, ld] array).
`pack_words` builds that layout on the host from base codes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshouji.so")
BASES_PER_WORD = 16
MAX_LEN = 1024
MAX_E = 31
_lib = None


class ShoujiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("shouji error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libshouji.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libshouji.so is not built: run __graft_entry__.build() "
                              "or python -m paper_1809_07858_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.shouji_filter.restype = ctypes.c_int
        L.shouji_filter.argtypes = [vp, vp, vp, i32, vp, vp, i64, i32, i64, vp]
        L.shouji_batched_workspace_bytes.restype = ctypes.c_int64
        L.shouji_batched_workspace_bytes.argtypes = [i64, i32]
        L.shouji_filter_batched.restype = ctypes.c_int
        L.shouji_filter_batched.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i64, vp, i64, vp, vp]
        L.shouji_tune_batched.restype = ctypes.c_int
        L.shouji_tune_batched.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i64, vp, i64, vp, vp, vp]
        L.shouji_last_error.restype = ctypes.c_char_p
        L.shouji_version.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise ShoujiError(rc, lib().shouji_last_error().decode())


def nwords(max_len):
    return (int(max_len) + BASES_PER_WORD - 1) // BASES_PER_WORD


def pack_words(codes, max_len=None, ld=None, chunk=1 << 18):
    """Base codes [n, stride] (uint8 0..3) -> packed words [nwords, ld] (int32 bit patterns).

    Word w of pair p holds bases 16w..16w+15 of row p, base j in bits 2(j%16)..2(j%16)+1.
    """
    codes = np.asarray(codes)
    n, stride = codes.shape
    max_len = stride if max_len is None else int(max_len)
    nw = nwords(max_len)
    ld = n if ld is None else int(ld)
    out = np.zeros((nw, ld), dtype=np.uint32)
    w = min(stride, nw * BASES_PER_WORD)
    shifts = (2 * np.arange(BASES_PER_WORD, dtype=np.uint32))
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        buf = np.zeros((hi - lo, nw * BASES_PER_WORD), dtype=np.uint32)
        buf[:, :w] = codes[lo:hi, :w] & 3
        words = np.bitwise_or.reduce(buf.reshape(hi - lo, nw, BASES_PER_WORD) << shifts, axis=2)
        out[:, lo:hi] = words.T
    return out.view(np.int32)


def pack_words_device(codes, max_len=None, ld=None, chunk=1 << 20):
    """Same layout as pack_words, computed on the GPU from a uint8 code tensor [n, stride]
    (host or device).  Returns an int32 CUDA tensor [nwords, ld]."""
    import torch
    n, stride = codes.shape
    max_len = stride if max_len is None else int(max_len)
    nw = nwords(max_len)
    ld = n if ld is None else int(ld)
    dev = torch.device("cuda", torch.cuda.current_device())
    out = torch.zeros((nw, ld), dtype=torch.int32, device=dev)
    w = min(stride, nw * BASES_PER_WORD)
    shifts = (2 * torch.arange(BASES_PER_WORD, dtype=torch.int64, device=dev))
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = torch.as_tensor(codes[lo:hi, :w]).to(dev, non_blocking=False).to(torch.int64) & 3
        buf = torch.zeros((hi - lo, nw * BASES_PER_WORD), dtype=torch.int64, device=dev)
        buf[:, :w] = c
        words = (buf.view(hi - lo, nw, BASES_PER_WORD) << shifts).sum(dim=2)
        words = torch.where(words >= 2 ** 31, words - 2 ** 32, words)
        out[:, lo:hi] = words.to(torch.int32).t()
    return out


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def shouji_filter(reads, refs, lengths, E, out_accept=None, out_popcount=None, n_pairs=None,
                  max_len=None, ld=None, stream=None, want_popcount=True):
    """Run the plain filter on device tensors.

    reads, refs : int32 CUDA tensors [nwords, ld] in the packed word-major layout
    lengths     : int32 CUDA tensor [n] or None (every pair has max_len bases)
    Returns (accept uint8 [n], popcount int16 [n] or None).
    """
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    ld = reads.shape[1] if ld is None else int(ld)
    if n_pairs is None:
        n_pairs = lengths.shape[0] if lengths is not None else ld
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    if lengths is not None and (not lengths.is_cuda or lengths.dtype != torch.int32
                                or lengths.numel() < n_pairs):
        raise ValueError("lengths must be an int32 CUDA tensor with n_pairs entries")
    dev = reads.device
    if out_accept is None:
        out_accept = torch.empty(n_pairs, dtype=torch.uint8, device=dev)
    if out_popcount is None and want_popcount:
        out_popcount = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    rc = lib().shouji_filter(ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
                             None if lengths is None else ctypes.c_void_p(lengths.data_ptr()),
                             int(E), ctypes.c_void_p(out_accept.data_ptr()),
                             None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
                             int(n_pairs), int(max_len), ld, _stream_handle(stream))
    _check(rc)
    return out_accept, out_popcount


class BatchedConfig(ctypes.Structure):
    """Tuning knobs of the batched form (0 = default / autotuned)."""
    _fields_ = [("bin_width", ctypes.c_int32), ("waves_per_group", ctypes.c_int32)]


def batched_workspace_bytes(n_pairs, max_len):
    v = lib().shouji_batched_workspace_bytes(int(n_pairs), int(max_len))
    if v < 0:
        _check(int(v))
    return int(v)


def _batched_args(reads, refs, lengths, E_per_pair, out_accept, out_popcount, n_pairs, max_len,
                  workspace, want_popcount):
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    if E_per_pair is None or not E_per_pair.is_cuda or E_per_pair.dtype != torch.int32:
        raise ValueError("E_per_pair must be an int32 CUDA tensor")
    ld = reads.shape[1]
    if n_pairs is None:
        n_pairs = E_per_pair.shape[0]
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    if lengths is not None and (not lengths.is_cuda or lengths.dtype != torch.int32
                                or lengths.numel() < n_pairs):
        raise ValueError("lengths must be an int32 CUDA tensor with n_pairs entries")
    dev = reads.device
    if out_accept is None:
        out_accept = torch.empty(n_pairs, dtype=torch.uint8, device=dev)
    if out_popcount is None and want_popcount:
        out_popcount = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    need = batched_workspace_bytes(n_pairs, max_len)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace too small: %d bytes needed" % need)
    args = [ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
            None if lengths is None else ctypes.c_void_p(lengths.data_ptr()),
            ctypes.c_void_p(E_per_pair.data_ptr()), ctypes.c_void_p(out_accept.data_ptr()),
            None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
            int(n_pairs), int(max_len), int(ld), ctypes.c_void_p(workspace.data_ptr()),
            int(workspace.numel() * workspace.element_size())]
    return args, out_accept, out_popcount, workspace


def shouji_filter_batched(reads, refs, lengths, E_per_pair, out_accept=None, out_popcount=None,
                          n_pairs=None, max_len=None, workspace=None, config=None, stream=None,
                          want_popcount=True):
    """Batched form: per-pair thresholds, mixed lengths.  config: (bin_width, waves_per_group) or None."""
    args, out_accept, out_popcount, workspace = _batched_args(
        reads, refs, lengths, E_per_pair, out_accept, out_popcount, n_pairs, max_len, workspace,
        want_popcount)
    cfg = None
    if config is not None:
        cfg = ctypes.byref(BatchedConfig(int(config[0]), int(config[1])))
    _check(lib().shouji_filter_batched(*args, cfg, _stream_handle(stream)))
    return out_accept, out_popcount


def tune_batched(reads, refs, lengths, E_per_pair, n_pairs=None, max_len=None, workspace=None,
                 stream=None):
    """Run the library's autotuner on these inputs; returns ((bin_width, waves_per_group), ms)."""
    args, _, _, _ = _batched_args(reads, refs, lengths, E_per_pair, None, None, n_pairs, max_len,
                                  workspace, True)
    best = BatchedConfig(0, 0)
    ms = ctypes.c_float(0.0)
    _check(lib().shouji_tune_batched(*args, _stream_handle(stream), ctypes.byref(best),
                                     ctypes.byref(ms)))
    return (best.bin_width, best.waves_per_group), float(ms.value)
