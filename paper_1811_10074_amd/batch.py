"""Batched minimizers over many reads of uneven length.

* ``minimizers_batch(seqs, offsets, k, w)``: one library call (one kernel
  launch over the concatenated reads) -> per-read results.
* ``BatchRunner``: preallocated device buffers for one batch; ``launch()``
  enqueues, ``result()`` synchronizes and returns views.
* ``BucketedBatch``: splits a batch into read-length buckets, runs each with
  the block size the tuner chose for its bucket (passed per call, no process
  state), and can capture the whole sequence of launches into one HIP graph
  (``capture()`` / ``replay()``).

The arithmetic is entirely in libsws (include/sws.h); this module only packs
CSR offsets, sizes buffers and issues the calls.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import SwsError, check

# Read-length buckets (mean length of the reads in a launch), as in the library.
BUCKET_LIMITS = (1000, 16000)


def bucket_of_length(length: int) -> int:
    return 0 if length < BUCKET_LIMITS[0] else (1 if length < BUCKET_LIMITS[1] else 2)


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _need_cuda(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor, got device %s" % (name, t.device))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def window_bound(offsets: np.ndarray, k: int, w: int) -> int:
    """Most minimizers the reads can have: sum over reads of max(0, L-k-w+2)."""
    lens = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(np.maximum(lens - k - w + 2, 0).sum())


def batch_workspace_bytes(total: int, nreads: int, k: int, w: int) -> int:
    b = ctypes.c_uint64(0)
    check(_lib.load().sws_minimizers_batch_workspace(total, nreads, k, w, ctypes.byref(b)),
          "sws_minimizers_batch_workspace")
    return int(b.value)


class BatchRunner:
    """Device buffers for one batch of reads (CSR: seqs + offsets)."""

    def __init__(self, seqs, offsets_np: np.ndarray, k: int, w: int, canonical=True, hashed=True,
                 device="cuda", split=False, threads: int = 0):
        torch = _torch()
        off = np.ascontiguousarray(offsets_np, dtype=np.uint64)
        self.k, self.w = k, w
        self.threads = int(threads)  # workgroup size of the launch; 0: the library default
        self.flags = ((0 if canonical else _lib.KMER_FORWARD) | (0 if hashed else _lib.HASH_IDENTITY)
                      | (_lib.SPLIT_AT_INVALID if split else 0))
        self.nreads = int(off.size - 1)
        self.total = int(off[-1])
        self.offsets_np = off
        if isinstance(seqs, np.ndarray):
            seqs = torch.from_numpy(np.ascontiguousarray(seqs, dtype=np.uint8)).to(device)
        if seqs.numel() != self.total:
            raise ValueError("seqs has %d bases, offsets say %d" % (seqs.numel(), self.total))
        _need_cuda(seqs, "seqs")
        self.seqs = seqs
        self.offsets = torch.from_numpy(off.view(np.int64)).to(device)
        self.capacity = window_bound(off, k, w)
        cap = max(self.capacity, 1)
        self.hash = torch.empty(cap, dtype=torch.int64, device=device)
        self.pos = torch.empty(cap, dtype=torch.int32, device=device)
        self.read = torch.empty(cap, dtype=torch.int32, device=device)
        self.read_out = torch.zeros(self.nreads + 1, dtype=torch.int64, device=device)
        ws = batch_workspace_bytes(self.total, self.nreads, k, w)
        # zero-filled once, then kept by the library between calls
        # (SWS_WORKSPACE_KEPT), which saves clearing it on every call
        self.workspace = torch.zeros(max(ws, 8), dtype=torch.uint8, device=device)
        self.calls = 0
        for name in ("offsets", "hash", "pos", "read", "read_out", "workspace"):
            _need_cuda(getattr(self, name), name)

    def launch(self, threads=None):
        """Enqueue on the current stream; threads overrides the runner's
        workgroup size for this call."""
        t = self.threads if threads is None else int(threads)
        fl = self.flags
        # the library asks for a call without the flag at least every 2^30 calls
        if self.calls % (1 << 29) != 0:
            fl |= _lib.WORKSPACE_KEPT
        self.calls += 1
        st = _lib.load().sws_minimizers_batch_ex(
            _ptr(self.seqs), _ptr(self.offsets), self.nreads, self.total, self.k, self.w,
            fl, _ptr(self.hash), _ptr(self.pos), _ptr(self.read), self.capacity,
            _ptr(self.read_out), _ptr(self.workspace), self.workspace.numel(), t, _stream())
        check(st, "sws_minimizers_batch_ex")

    def result(self):
        """Synchronizes; returns (hash, pos, read, read_offsets) device views."""
        ro = self.read_out
        total = int(ro[-1].item())
        if total < 0:
            raise SwsError(_lib.SWS_ERR_DEVICE, "batch minimizer kernel reported an internal error")
        if total > self.capacity:
            raise SwsError(_lib.SWS_ERR_CAPACITY, "outputs truncated")
        return self.hash[:total], self.pos[:total], self.read[:total], ro


def minimizers_batch(seqs, offsets, k: int, w: int, canonical: bool = True, hashed: bool = True,
                     split: bool = False):
    """Per-read minimizers of reads seqs[offsets[r]:offsets[r+1]] in one launch.

    seqs: uint8 device tensor (or numpy array); offsets: host array of
    nreads + 1 non-decreasing values from 0.  Returns (hash int64, pos int32,
    read int32, read_offsets int64[nreads+1]) on the device, read-major."""
    torch = _torch()
    off = np.asarray(offsets.cpu() if torch.is_tensor(offsets) else offsets, dtype=np.uint64)
    # numpy arrays also carry a .device ("cpu"): only a torch tensor names the device to use
    r = BatchRunner(seqs, off, k, w, canonical, hashed,
                    device=seqs.device if torch.is_tensor(seqs) else "cuda", split=split)
    r.launch()
    h, p, rd, ro = r.result()
    return h.clone(), p.clone(), rd.clone(), ro.clone()


class BucketedBatch:
    """A batch split into read-length buckets, one library call per bucket with
    the block size tuned for that bucket; optionally captured in a HIP graph.

    reads keep their relative order inside a bucket; ``bucket_of[r]`` and
    ``index_in_bucket[r]`` map an input read to its bucket's results."""

    def __init__(self, seqs_np: np.ndarray, offsets_np: np.ndarray, k: int, w: int,
                 canonical=True, hashed=True, tune_table=None, device="cuda"):
        torch = _torch()
        off = np.asarray(offsets_np, dtype=np.int64)
        lens = np.diff(off)
        self.k, self.w = k, w
        self.nreads = lens.size
        self.bucket_of = np.digitize(lens, BUCKET_LIMITS).astype(np.int8)
        self.index_in_bucket = np.zeros(lens.size, dtype=np.int64)
        self.tune_table = dict(tune_table or {})
        self.runners = {}
        for b in range(3):
            sel = np.nonzero(self.bucket_of == b)[0]
            if sel.size == 0:
                continue
            self.index_in_bucket[sel] = np.arange(sel.size)
            blens = lens[sel]
            boff = np.zeros(sel.size + 1, dtype=np.uint64)
            np.cumsum(blens, out=boff[1:])
            # gather the bucket's reads (host side, once, outside any timing)
            bseq = seqs_np[np.repeat(self.bucket_of == b, lens)]
            self.runners[b] = BatchRunner(torch.from_numpy(bseq).to(device), boff, k, w,
                                          canonical, hashed, device=device,
                                          threads=int(self.tune_table.get(b, 0)))
        self.graph = None

    def launch(self):
        for r in self.runners.values():
            r.launch()

    def capture(self):
        """Record every bucket's launches into one HIP graph (block sizes are
        fixed at capture time).  The captured calls keep their workspaces
        (SWS_WORKSPACE_KEPT, after the warm-up call), so the graph holds no
        clearing kernel; capture again before 2^30 replays."""
        torch = _torch()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.launch()  # warm up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self):
        return {b: r.result() for b, r in self.runners.items()}

    def read_result(self, r: int, results=None):
        """(hash, pos) of input read r, as host numpy arrays."""
        results = results or self.results()
        b = int(self.bucket_of[r])
        i = int(self.index_in_bucket[r])
        h, p, rd, ro = results[b]
        a, e = int(ro[i].item()), int(ro[i + 1].item())
        return (h[a:e].cpu().numpy().view(np.uint64), p[a:e].cpu().numpy().view(np.uint32))
