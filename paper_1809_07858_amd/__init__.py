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


class ServerConfig(ctypes.Structure):
    _fields_ = [("pool", ctypes.c_void_p), ("pool_bases", ctypes.c_int64), ("max_len", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("max_batch_pairs", ctypes.c_int64),
                ("memory_budget", ctypes.c_int64), ("host_threads", ctypes.c_int32),
                ("fill_wait_us", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_void_p), ("words_per_read", ctypes.c_int32),
                ("ref_offsets", ctypes.c_void_p), ("lengths", ctypes.c_void_p), ("E", ctypes.c_void_p),
                ("out_accept", ctypes.c_void_p), ("out_popcount", ctypes.c_void_p),
                ("n_pairs", ctypes.c_int64), ("flags", ctypes.c_uint32), ("read_words", ctypes.c_int64)]


REQUEST_PINNED = 1
REQUEST_PACKED = 2


class ServerStats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("batches", ctypes.c_int64), ("pairs_done", ctypes.c_int64),
                ("requests_done", ctypes.c_int64), ("requests_deferred", ctypes.c_int64),
                ("queued_pairs", ctypes.c_int64)]


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
        L.shouji_filter_local.restype = ctypes.c_int
        L.shouji_filter_local.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, i64, i32, i64, vp]
        L.shouji_filter_window.restype = ctypes.c_int
        L.shouji_filter_window.argtypes = [vp, vp, vp, i32, i32, vp, vp, i64, i32, i64, vp]
        L.shouji_filter_magnet.restype = ctypes.c_int
        L.shouji_filter_magnet.argtypes = [vp, vp, vp, i32, vp, vp, i64, i32, i64, vp]
        L.shouji_verify_workspace_bytes.restype = ctypes.c_int64
        L.shouji_verify_workspace_bytes.argtypes = [i64]
        L.shouji_verify.restype = ctypes.c_int
        L.shouji_verify.argtypes = [vp, vp, vp, i32, vp, vp, i64, i32, i64, vp, i64, vp]
        L.shouji_batched_workspace_bytes.restype = ctypes.c_int64
        L.shouji_batched_workspace_bytes.argtypes = [i64, i32]
        L.shouji_filter_batched.restype = ctypes.c_int
        L.shouji_filter_batched.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i64, vp, i64, vp, vp]
        L.shouji_filter_batched_noalloc.restype = ctypes.c_int
        L.shouji_filter_batched_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i64, vp, vp]
        L.shouji_tune_batched.restype = ctypes.c_int
        L.shouji_tune_batched.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, i64, vp, i64, vp, vp, vp]
        L.shouji_server_slot_bytes.restype = ctypes.c_int64
        L.shouji_server_slot_bytes.argtypes = [i64, i32]
        L.shouji_server_create.restype = ctypes.c_int
        L.shouji_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.shouji_server_submit.restype = ctypes.c_int
        L.shouji_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.shouji_server_poll.restype = ctypes.c_int
        L.shouji_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32)]
        L.shouji_server_wait.restype = ctypes.c_int
        L.shouji_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.shouji_server_get_stats.restype = ctypes.c_int
        L.shouji_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.shouji_server_destroy.restype = ctypes.c_int
        L.shouji_server_destroy.argtypes = [vp]
        L.shouji_relayout_pair_major.restype = ctypes.c_int
        L.shouji_relayout_pair_major.argtypes = [vp, i64, i64, i32, vp, i64, vp]
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


def pack_pair_major(codes, max_len=None, words_per_seq=None):
    """Base codes [n, stride] (uint8 0..3) -> [n, words_per_seq] uint64: each pair's
    sequence 32 bases per 64-bit word, base j in bits 2(j%32)..2(j%32)+1 of word j/32
    (words_per_seq defaults to ceil(max_len/32)).  The input of relayout_pair_major."""
    codes = np.asarray(codes)
    n, stride = codes.shape
    max_len = stride if max_len is None else int(max_len)
    need = (max_len + 31) // 32
    wps = need if words_per_seq is None else int(words_per_seq)
    if wps < need:
        raise ValueError("words_per_seq %d < %d for max_len %d" % (wps, need, max_len))
    buf = np.zeros((n, wps * 32), dtype=np.uint64)
    w = min(stride, max_len)
    buf[:, :w] = codes[:, :w] & 3
    shifts = 2 * np.arange(32, dtype=np.uint64)
    return np.bitwise_or.reduce(buf.reshape(n, wps, 32) << shifts, axis=2)


def relayout_pair_major(src, max_len, n_pairs=None, ld=None, out=None, stream=None):
    """Device relayout of pair-major 64-bit words (an int64 CUDA tensor [n, words_per_seq],
    as from pack_pair_major) into the filters' word-major layout: an int32 CUDA tensor
    [ceil(max_len/16), ld] (the same words pack_words gives for the same bases)."""
    import torch
    if src.dim() != 2 or not src.is_cuda or src.dtype != torch.int64 or not src.is_contiguous():
        raise ValueError("src must be a contiguous int64 CUDA tensor [n_pairs, words_per_seq]")
    n = src.shape[0] if n_pairs is None else int(n_pairs)
    if n > src.shape[0]:
        raise ValueError("n_pairs exceeds the rows of src")
    ld = n if ld is None else int(ld)
    if out is None:
        out = torch.zeros((nwords(max_len), ld), dtype=torch.int32, device=src.device)
    if out.dim() != 2 or out.dtype != torch.int32 or not out.is_contiguous() or out.shape[0] < nwords(max_len) \
            or out.shape[1] != ld:
        raise ValueError("out must be a contiguous int32 tensor [ceil(max_len/16), ld]")
    _check(lib().shouji_relayout_pair_major(ctypes.c_void_p(src.data_ptr()), int(src.shape[1]), n, int(max_len),
                                            ctypes.c_void_p(out.data_ptr()), ld, _stream_handle(stream)))
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


COUNT_GLOBAL, COUNT_LOCAL, COUNT_GLOCAL_START, COUNT_GLOCAL_END = 0, 1, 2, 3


def shouji_filter_local(reads, refs, read_lengths, ref_lengths, E, mode=COUNT_LOCAL, out_accept=None,
                        out_popcount=None, n_pairs=None, max_len=None, stream=None, want_popcount=True):
    """Two-length form: reads and references of different lengths (int32 CUDA tensors of
    lengths), counting mode COUNT_GLOBAL / COUNT_LOCAL / COUNT_GLOCAL_START / COUNT_GLOCAL_END."""
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    ld = reads.shape[1]
    if n_pairs is None:
        n_pairs = ld
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    for t in (read_lengths, ref_lengths):
        if not t.is_cuda or t.dtype != torch.int32 or t.numel() < n_pairs:
            raise ValueError("lengths must be int32 CUDA tensors with n_pairs entries")
    dev = reads.device
    if out_accept is None:
        out_accept = torch.empty(n_pairs, dtype=torch.uint8, device=dev)
    if out_popcount is None and want_popcount:
        out_popcount = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    _check(lib().shouji_filter_local(
        ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
        ctypes.c_void_p(read_lengths.data_ptr()), ctypes.c_void_p(ref_lengths.data_ptr()), int(E), int(mode),
        ctypes.c_void_p(out_accept.data_ptr()),
        None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
        int(n_pairs), int(max_len), int(ld), _stream_handle(stream)))
    return out_accept, out_popcount


def shouji_filter_window(reads, refs, lengths, E, W, out_accept=None, out_popcount=None, n_pairs=None,
                         max_len=None, stream=None, want_popcount=True):
    """Window-width variant: the filter with W-column windows (1..16)."""
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    ld = reads.shape[1]
    if n_pairs is None:
        n_pairs = ld
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    if lengths is not None and (not lengths.is_cuda or lengths.dtype != torch.int32 or lengths.numel() < n_pairs):
        raise ValueError("lengths must be an int32 CUDA tensor with n_pairs entries")
    dev = reads.device
    if out_accept is None:
        out_accept = torch.empty(n_pairs, dtype=torch.uint8, device=dev)
    if out_popcount is None and want_popcount:
        out_popcount = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    _check(lib().shouji_filter_window(
        ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
        None if lengths is None else ctypes.c_void_p(lengths.data_ptr()), int(E), int(W),
        ctypes.c_void_p(out_accept.data_ptr()),
        None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
        int(n_pairs), int(max_len), int(ld), _stream_handle(stream)))
    return out_accept, out_popcount


def shouji_filter_magnet(reads, refs, lengths, E, out_accept=None, out_popcount=None, n_pairs=None,
                         max_len=None, stream=None, want_popcount=True):
    """MAGNET filter (divide-and-conquer runs of matches) on equal-length pairs."""
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    ld = reads.shape[1]
    if n_pairs is None:
        n_pairs = ld
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    if lengths is not None and (not lengths.is_cuda or lengths.dtype != torch.int32 or lengths.numel() < n_pairs):
        raise ValueError("lengths must be an int32 CUDA tensor with n_pairs entries")
    dev = reads.device
    if out_accept is None:
        out_accept = torch.empty(n_pairs, dtype=torch.uint8, device=dev)
    if out_popcount is None and want_popcount:
        out_popcount = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    _check(lib().shouji_filter_magnet(
        ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
        None if lengths is None else ctypes.c_void_p(lengths.data_ptr()), int(E),
        ctypes.c_void_p(out_accept.data_ptr()),
        None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
        int(n_pairs), int(max_len), int(ld), _stream_handle(stream)))
    return out_accept, out_popcount


def shouji_verify(reads, refs, lengths, E, filter_accept=None, out_distance=None, n_pairs=None,
                  max_len=None, workspace=None, stream=None):
    """Banded edit distance of the pairs a filter accepted (all pairs when filter_accept is
    None): int16 per pair, distance if <= E, -1 above, -2 not verified, -3 invalid length."""
    import torch
    if reads.dim() != 2 or refs.shape != reads.shape:
        raise ValueError("reads/refs must be [nwords, ld] tensors of the same shape")
    for t in (reads, refs):
        if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("reads/refs must be contiguous int32 CUDA tensors")
    ld = reads.shape[1]
    if n_pairs is None:
        n_pairs = ld
    if max_len is None:
        max_len = reads.shape[0] * BASES_PER_WORD
    if reads.shape[0] < nwords(max_len):
        raise ValueError("reads hold fewer words than max_len needs")
    if lengths is not None and (not lengths.is_cuda or lengths.dtype != torch.int32 or lengths.numel() < n_pairs):
        raise ValueError("lengths must be an int32 CUDA tensor with n_pairs entries")
    if filter_accept is not None and (not filter_accept.is_cuda or filter_accept.dtype != torch.uint8
                                      or filter_accept.numel() < n_pairs):
        raise ValueError("filter_accept must be a uint8 CUDA tensor with n_pairs entries")
    dev = reads.device
    if out_distance is None:
        out_distance = torch.empty(n_pairs, dtype=torch.int16, device=dev)
    need = lib().shouji_verify_workspace_bytes(int(n_pairs))
    if need < 0:
        _check(int(need))
    if workspace is None:
        workspace = torch.empty(int(need), dtype=torch.uint8, device=dev)
    _check(lib().shouji_verify(
        ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
        None if lengths is None else ctypes.c_void_p(lengths.data_ptr()), int(E),
        None if filter_accept is None else ctypes.c_void_p(filter_accept.data_ptr()),
        ctypes.c_void_p(out_distance.data_ptr()), int(n_pairs), int(max_len), int(ld),
        ctypes.c_void_p(workspace.data_ptr()), int(workspace.numel() * workspace.element_size()),
        _stream_handle(stream)))
    return out_distance


class BatchedConfig(ctypes.Structure):
    """Tuning knobs of the batched form (0 = default / autotuned)."""
    _fields_ = [("bin_width", ctypes.c_int32), ("waves_per_group", ctypes.c_int32)]


def batched_workspace_bytes(n_pairs, max_len):
    v = lib().shouji_batched_workspace_bytes(int(n_pairs), int(max_len))
    if v < 0:
        _check(int(v))
    return int(v)


def _batched_args(reads, refs, lengths, E_per_pair, out_accept, out_popcount, n_pairs, max_len,
                  workspace, want_popcount, with_workspace=True):
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
    args = [ctypes.c_void_p(reads.data_ptr()), ctypes.c_void_p(refs.data_ptr()),
            None if lengths is None else ctypes.c_void_p(lengths.data_ptr()),
            ctypes.c_void_p(E_per_pair.data_ptr()), ctypes.c_void_p(out_accept.data_ptr()),
            None if out_popcount is None else ctypes.c_void_p(out_popcount.data_ptr()),
            int(n_pairs), int(max_len), int(ld)]
    if not with_workspace:
        return args, out_accept, out_popcount, None
    need = batched_workspace_bytes(n_pairs, max_len)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace too small: %d bytes needed" % need)
    args += [ctypes.c_void_p(workspace.data_ptr()), int(workspace.numel() * workspace.element_size())]
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


NOALLOC_SCRATCH_BYTES = 128 << 20   # SHOUJI_NOALLOC_SCRATCH_BYTES


def shouji_filter_batched_noalloc(reads, refs, lengths, E_per_pair, out_accept=None, out_popcount=None,
                                  n_pairs=None, max_len=None, config=None, stream=None,
                                  want_popcount=True):
    """Batched form without a workspace: the library's own scratch array holds the
    binned copy (at most NOALLOC_SCRATCH_BYTES; see include/shouji.h).  With the
    outputs passed in, nothing is allocated on the way to the library."""
    args, out_accept, out_popcount, _ = _batched_args(
        reads, refs, lengths, E_per_pair, out_accept, out_popcount, n_pairs, max_len, None,
        want_popcount, with_workspace=False)
    cfg = None
    if config is not None:
        cfg = ctypes.byref(BatchedConfig(int(config[0]), int(config[1])))
    _check(lib().shouji_filter_batched_noalloc(*args, cfg, _stream_handle(stream)))
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


def pack_pairs(codes, max_len=None):
    """Base codes [n, stride] (uint8 0..3) -> pair-major packed words [n, nwords] (uint32),
    the read layout of a server request."""
    return np.ascontiguousarray(pack_words(codes, max_len).view(np.uint32).T)


def packed_read_words(lengths, max_len):
    """Words each read takes in the packed request layout: ceil(m/16), none for a
    length outside [1, max_len] (int64 [n])."""
    lens = np.asarray(lengths, dtype=np.int64)
    return np.where((lens >= 1) & (lens <= int(max_len)), (lens + BASES_PER_WORD - 1) // BASES_PER_WORD, 0)


def _packed_words_total(lens, max_len):
    """Sum of packed_read_words over an int32 length array (fast when every length is
    in range, the usual case)."""
    if lens.size == 0:
        return 0
    if int(lens.min()) >= 1 and int(lens.max()) <= int(max_len):
        return int(np.add.reduce((lens + (BASES_PER_WORD - 1)) // BASES_PER_WORD, dtype=np.int64))
    return int(packed_read_words(lens, max_len).sum())


def pack_reads_packed(codes, lengths, max_len):
    """Base codes [n, stride] (uint8 0..3) and lengths -> (words, offsets): the reads
    back to back, read p in words[offsets[p]:offsets[p+1]] (ceil(m_p/16) words), the
    packed read layout of a server request (SHOUJI_REQUEST_PACKED).  A request made of
    pairs lo..hi-1 passes words[offsets[lo]:offsets[hi]]."""
    rows = pack_pairs(codes, max_len)
    k = packed_read_words(lengths, max_len)
    offsets = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    mask = np.arange(rows.shape[1])[None, :] < k[:, None]
    return np.ascontiguousarray(rows[mask]), offsets


def pack_pool(codes):
    """Flat base codes (uint8 0..3) -> packed pool words (uint32): base b in bits
    2(b%16).. of word b/16, the reference-pool layout of the server."""
    codes = np.asarray(codes, dtype=np.uint8).ravel()
    nw = nwords(codes.size)
    buf = np.zeros(nw * BASES_PER_WORD, dtype=np.uint32)
    buf[:codes.size] = codes & 3
    shifts = 2 * np.arange(BASES_PER_WORD, dtype=np.uint32)
    return np.bitwise_or.reduce(buf.reshape(nw, BASES_PER_WORD) << shifts, axis=1)


def server_slot_bytes(max_batch_pairs, max_len):
    """Device bytes of one server batch slot (to size memory_budget)."""
    v = lib().shouji_server_slot_bytes(int(max_batch_pairs), int(max_len))
    if v < 0:
        _check(int(v))
    return int(v)


class Ticket:
    """A submitted request: keeps its host buffers alive until Server.wait returns."""

    def __init__(self, tid, bufs, out_accept, out_popcount):
        self.id = tid
        self._bufs = bufs
        self.out_accept = out_accept
        self.out_popcount = out_popcount
        self.latency_ms = None


class Server:
    """Request server with continuous batching (shouji_server_* in include/shouji.h).

    pool: int32 CUDA tensor of packed reference words (pack_pool), resident for the
    server's lifetime.  Requests are host numpy arrays.
    """

    def __init__(self, pool, pool_bases, max_len, slots=3, max_batch_pairs=1 << 20,
                 memory_budget=0, host_threads=0, fill_wait_us=0):
        import torch
        if not pool.is_cuda or pool.dtype != torch.int32 or not pool.is_contiguous():
            raise ValueError("pool must be a contiguous int32 CUDA tensor")
        if pool.numel() < nwords(pool_bases):
            raise ValueError("pool holds fewer words than pool_bases needs")
        self.pool = pool
        self.max_len = int(max_len)
        self.nw = nwords(max_len)
        cfg = ServerConfig(pool.data_ptr(), int(pool_bases), int(max_len), int(slots),
                           int(max_batch_pairs), int(memory_budget), int(host_threads),
                           int(fill_wait_us))
        h = ctypes.c_void_p()
        _check(lib().shouji_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, reads, ref_offsets, lengths, E, want_popcount=True, pinned=False,
               out_accept=None, out_popcount=None, packed=False):
        """Queue a request.  reads: uint32 [n, words_per_read] (pack_pairs), or with
        packed=True the reads back to back as one uint32 array (pack_reads_packed);
        ref_offsets int64, lengths int32, E int32 (scalar or per pair).  pinned=True declares
        that every buffer, outputs included, is pinned host memory (e.g. numpy views of torch
        pin_memory tensors), so the server moves it by DMA without staging.  Returns a
        Ticket."""
        reads = np.ascontiguousarray(reads, dtype=np.uint32)
        lens = np.ascontiguousarray(lengths, dtype=np.int32)
        if packed:
            if reads.ndim != 1:
                raise ValueError("packed reads are one flat uint32 array")
            n = lens.shape[0]
            need = _packed_words_total(lens, self.max_len)
            if reads.size != need:
                raise ValueError("packed reads hold %d words, the lengths need %d" % (reads.size, need))
        else:
            if reads.ndim != 2:
                raise ValueError("reads must be [n_pairs, words_per_read]")
            n = reads.shape[0]
        offs = np.ascontiguousarray(ref_offsets, dtype=np.int64)
        Ep = np.ascontiguousarray(np.broadcast_to(np.asarray(E, dtype=np.int32), (n,)))
        if offs.shape != (n,) or lens.shape != (n,):
            raise ValueError("ref_offsets and lengths need one entry per pair")
        if pinned:
            given = (reads, ref_offsets, lengths, E)
            if (out_accept is None or (want_popcount and out_popcount is None)
                    or any(not isinstance(g, np.ndarray) or a.ctypes.data != g.ctypes.data
                           for g, a in zip(given, (reads, offs, lens, Ep)))):
                raise ValueError("a pinned request passes contiguous uint32/int64/int32/int32 "
                                 "arrays (per-pair E) and its own pinned outputs")
        acc = np.empty(n, dtype=np.uint8) if out_accept is None else out_accept
        pc = out_popcount if out_popcount is not None else (
            np.empty(n, dtype=np.int16) if want_popcount else None)
        if acc.shape != (n,) or acc.dtype != np.uint8 or (pc is not None and (
                pc.shape != (n,) or pc.dtype != np.int16)):
            raise ValueError("outputs must be uint8 / int16 arrays with one entry per pair")
        req = Request(reads.ctypes.data, 1 if packed else max(1, reads.shape[1]), offs.ctypes.data,
                      lens.ctypes.data, Ep.ctypes.data, acc.ctypes.data,
                      None if pc is None else pc.ctypes.data, n,
                      (REQUEST_PINNED if pinned else 0) | (REQUEST_PACKED if packed else 0),
                      reads.size if packed else 0)
        t = ctypes.c_uint64()
        _check(lib().shouji_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return Ticket(t.value, (reads, offs, lens, Ep), acc, pc)

    def poll(self, ticket):
        d = ctypes.c_int32()
        _check(lib().shouji_server_poll(self._h, ticket.id, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket):
        """Block until done; returns (out_accept, out_popcount, latency_ms)."""
        ms = ctypes.c_double()
        _check(lib().shouji_server_wait(self._h, ticket.id, ctypes.byref(ms)))
        ticket.latency_ms = ms.value
        ticket._bufs = None
        return ticket.out_accept, ticket.out_popcount, ms.value

    def stats(self):
        st = ServerStats()
        _check(lib().shouji_server_get_stats(self._h, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().shouji_server_destroy(self._h))
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
