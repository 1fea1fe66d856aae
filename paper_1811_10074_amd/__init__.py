"""sws: sliding window sums and minimizer seed tables on AMD MI355X (gfx950).

A thin binding over libsws.so (include/sws.h): every step runs in the HIP
kernels; this module only allocates torch tensors for device memory, passes
pointers and the current torch stream, and maps status codes to exceptions.

    sliding_sum(op, w, x, path="auto")   Sec. 2.2 Eq. 2 (op: add/min/max/affine)
    pack2bit(seq)                         2-bit codes + invalid bits
    kmers(seq, k, canonical, hashed)      one value per k-mer (UINT64_MAX if invalid)
    minimizers(seq, k, w, ...)            Sec. 2.4 / Fig. 2 seeds: (hash, pos)
    minimizers_2bit(packed, invalid, n, k, w, ...)
    minimizers_batch(seqs, offsets, k, w, ...)
    seed_table(hash, pos, bits, shift)    Sec. 2.4 / Fig. 1 pointer + position tables

Device tensors hold unsigned data in signed torch dtypes (int32 for uint32,
int64 for uint64); ``.view(numpy.uint32)`` etc. on the host restores the
unsigned reading.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import SwsError, check

__all__ = ["sliding_sum", "pack2bit", "kmers", "minimizers", "minimizers_2bit", "seed_table",
           "minimizers_batch", "MinimizerRunner", "window_bound", "SwsError"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _need_cuda(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _flags(canonical: bool, hashed: bool, split: bool = False) -> int:
    return ((0 if canonical else _lib.KMER_FORWARD) | (0 if hashed else _lib.HASH_IDENTITY)
            | (_lib.SPLIT_AT_INVALID if split else 0))


def window_bound(n: int, k: int, w: int) -> int:
    """Most minimizers a sequence of n bases can have."""
    return max(0, n - k - w + 2)


def sliding_sum(op: str, w: int, x, path: str = "auto", out=None):
    """y_i = x_i (+) ... (+) x_{i+w-1}.  x: int32/uint32 tensor [n], or [n, 2]
    (a, b) pairs for op='affine'.  Returns a tensor of n-w+1 elements."""
    torch = _torch()
    _need_cuda(x, "x")
    if op not in _lib.OPS:
        raise ValueError("unknown op %r" % op)
    if path not in _lib.PATHS:
        raise ValueError("unknown path %r" % path)
    if x.element_size() != 4:
        raise ValueError("x must hold 32-bit elements")
    pair = op == "affine"
    if pair and (x.dim() != 2 or x.shape[1] != 2):
        raise ValueError("affine input must have shape [n, 2]")
    n = x.shape[0]
    cnt = max(0, n - w + 1) if w >= 1 else 0
    shape = (cnt, 2) if pair else (cnt,)
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != x.dtype:
        raise ValueError("out must have shape %s and dtype %s" % (shape, x.dtype))
    lib = _lib.load()
    b = ctypes.c_uint64(0)
    check(lib.sws_sliding_sum_workspace(_lib.OPS[op], w, n, _lib.PATHS[path], ctypes.byref(b)),
          "sws_sliding_sum_workspace")
    ws = torch.empty(int(b.value), dtype=torch.uint8, device=x.device) if b.value else None
    st = lib.sws_sliding_sum_ws(_lib.OPS[op], w, _ptr(x), n, _ptr(out), _lib.PATHS[path],
                                _ptr(ws), int(b.value), _stream())
    check(st, "sws_sliding_sum_ws")
    return out


def set_sliding_waves(waves: int = 0) -> None:
    """Wavefronts a generic-path sliding_sum launch aims for (0: default);
    each streams ceil(slabs / waves) consecutive slabs.  Process-wide."""
    check(_lib.load().sws_set_sliding_waves(int(waves)), "sws_set_sliding_waves")


def pack2bit(seq, with_invalid: bool = True):
    """ASCII uint8 tensor -> (packed int32[ceil(n/16)], invalid int32[ceil(n/32)] or None)."""
    torch = _torch()
    _need_cuda(seq, "seq")
    n = seq.numel()
    packed = torch.empty((n + 15) // 16, dtype=torch.int32, device=seq.device)
    invalid = torch.empty((n + 31) // 32, dtype=torch.int32, device=seq.device) if with_invalid else None
    check(_lib.load().sws_pack2bit(_ptr(seq), n, _ptr(packed), _ptr(invalid), _stream()),
          "sws_pack2bit")
    return packed, invalid


def kmers(seq, k: int, canonical: bool = True, hashed: bool = True):
    torch = _torch()
    _need_cuda(seq, "seq")
    n = seq.numel()
    out = torch.empty(max(0, n - k + 1), dtype=torch.int64, device=seq.device)
    check(_lib.load().sws_kmers(_ptr(seq), n, k, _flags(canonical, hashed), _ptr(out), _stream()),
          "sws_kmers")
    return out


def minimizer_workspace_bytes(n: int, k: int, w: int) -> int:
    b = ctypes.c_uint64(0)
    check(_lib.load().sws_minimizers_workspace(n, k, w, ctypes.byref(b)), "sws_minimizers_workspace")
    return int(b.value)


class MinimizerRunner:
    """Preallocated outputs and workspace for repeated minimizer calls on
    sequences of up to ``max_n`` bases (no allocation per call)."""

    def __init__(self, max_n: int, k: int, w: int, device="cuda"):
        torch = _torch()
        self.k, self.w, self.max_n = k, w, max_n
        self.capacity = window_bound(max_n, k, w)
        self.hash = torch.empty(max(self.capacity, 1), dtype=torch.int64, device=device)
        self.pos = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        ws = minimizer_workspace_bytes(max_n, k, w)
        # zero-filled once, then kept by the library between calls
        # (SWS_WORKSPACE_KEPT), which saves clearing it on every call
        self.workspace = torch.zeros(max(ws, 8), dtype=torch.uint8, device=device)
        self.calls = 0
        for name in ("hash", "pos", "count", "workspace"):
            _need_cuda(getattr(self, name), name)

    def launch(self, seq=None, packed=None, invalid=None, n=None, canonical=True, hashed=True,
               split=False):
        """Enqueue one call on the current stream; results stay on the device
        (self.hash, self.pos, self.count).  split: invalid bases cut the
        sequence into segments (SWS_SPLIT_AT_INVALID)."""
        lib = _lib.load()
        fl = _flags(canonical, hashed, split)
        # the library asks for a call without the flag at least every 2^30 calls
        if self.calls % (1 << 29) != 0:
            fl |= _lib.WORKSPACE_KEPT
        self.calls += 1
        if seq is not None:
            _need_cuda(seq, "seq")
            n = seq.numel()
            if n > self.max_n:
                raise ValueError("sequence longer than the runner's max_n")
            st = lib.sws_minimizers(_ptr(seq), n, self.k, self.w, fl, _ptr(self.hash),
                                    _ptr(self.pos), self.capacity, _ptr(self.count),
                                    _ptr(self.workspace), self.workspace.numel(), _stream())
            check(st, "sws_minimizers")
        else:
            if n is None or n > self.max_n:
                raise ValueError("n missing or above max_n")
            _need_cuda(packed, "packed")
            if invalid is not None:
                _need_cuda(invalid, "invalid")
            st = lib.sws_minimizers_2bit(_ptr(packed), _ptr(invalid), n, self.k, self.w, fl,
                                         _ptr(self.hash), _ptr(self.pos), self.capacity,
                                         _ptr(self.count), _ptr(self.workspace),
                                         self.workspace.numel(), _stream())
            check(st, "sws_minimizers_2bit")

    def result(self):
        """Synchronizes, then returns (hash int64[c], pos int32[c]) views."""
        c = int(self.count.item())
        if c < 0:  # all ones: a tile gave up waiting for its predecessor
            raise SwsError(_lib.SWS_ERR_DEVICE, "minimizer kernel reported an internal error")
        return self.hash[:c], self.pos[:c]


def minimizers(seq, k: int, w: int, canonical: bool = True, hashed: bool = True,
               split: bool = False):
    """Deduplicated minimizers of one ASCII sequence: (hash int64[c], pos int32[c])."""
    _need_cuda(seq, "seq")
    r = MinimizerRunner(seq.numel(), k, w, device=seq.device)
    r.launch(seq=seq, canonical=canonical, hashed=hashed, split=split)
    h, p = r.result()
    return h.clone(), p.clone()


def minimizers_2bit(packed, invalid, n: int, k: int, w: int, canonical: bool = True,
                    hashed: bool = True, split: bool = False):
    _need_cuda(packed, "packed")
    r = MinimizerRunner(n, k, w, device=packed.device)
    r.launch(packed=packed, invalid=invalid, n=n, canonical=canonical, hashed=hashed, split=split)
    h, p = r.result()
    return h.clone(), p.clone()


def minimizers_batch(seqs, offsets, k: int, w: int, canonical: bool = True, hashed: bool = True,
                     split: bool = False):
    from .batch import minimizers_batch as _mb
    return _mb(seqs, offsets, k, w, canonical=canonical, hashed=hashed, split=split)


class SeedTableRunner:
    """Preallocated outputs and workspace for seed tables of up to ``max_count``
    entries keyed by ``bits`` bits (no allocation per call)."""

    def __init__(self, max_count: int, bits: int, with_hash: bool = True, device="cuda"):
        torch = _torch()
        self.max_count, self.bits = max_count, bits
        b = ctypes.c_uint64(0)
        check(_lib.load().sws_seed_table_workspace(max_count, bits, ctypes.byref(b)),
              "sws_seed_table_workspace")
        self.ptr = torch.empty((1 << bits) + 1, dtype=torch.int32, device=device)
        self.pos = torch.empty(max(max_count, 1), dtype=torch.int32, device=device)
        self.hash = (torch.empty(max(max_count, 1), dtype=torch.int64, device=device)
                     if with_hash else None)
        self.workspace = torch.empty(max(int(b.value), 16), dtype=torch.uint8, device=device)
        for name in ("ptr", "pos", "workspace"):
            _need_cuda(getattr(self, name), name)

    def launch(self, hash_, pos, shift: int):
        """Enqueue on the current stream; results in self.ptr/pos/hash."""
        _need_cuda(hash_, "hash")
        _need_cuda(pos, "pos")
        count = pos.numel()
        if hash_.numel() != count or count > self.max_count:
            raise ValueError("hash and pos must have the same length, at most max_count")
        st = _lib.load().sws_seed_table(_ptr(hash_), _ptr(pos), count, self.bits, shift,
                                        _ptr(self.ptr), _ptr(self.pos), _ptr(self.hash),
                                        _ptr(self.workspace), self.workspace.numel(), _stream())
        check(st, "sws_seed_table")
        self.count = count


def seed_table(hash_, pos, bits: int, shift=None, with_hash: bool = True):
    """Seed pointer table int32[2^bits + 1] (ptr[j] = entries with key < j) and
    the positions (and hashes) grouped by key = (hash >> shift) mod 2^bits,
    each group in input order.  shift defaults to 64 - bits (the top bits)."""
    _need_cuda(hash_, "hash")
    _need_cuda(pos, "pos")
    shift = 64 - bits if shift is None else shift
    r = SeedTableRunner(pos.numel(), bits, with_hash, device=pos.device)
    r.launch(hash_, pos, shift)
    n = pos.numel()
    return r.ptr, r.pos[:n], (r.hash[:n] if with_hash else None)
