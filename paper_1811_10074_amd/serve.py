"""Continuous-batching server for minimizer sketching requests.

A request is a set of reads (CSR: bases + offsets).  The scheduler thread

1. admits queued requests, oldest first, while the device arena has room for
   the batch they form (inputs, outputs at their exact bound, workspace);
   a request larger than the whole arena is rejected;
2. packs the admitted requests into one CSR batch, copies it to its arena slot
   and launches one batched minimizer call on one of several streams;
3. polls the in-flight batches; a finished batch is copied back, split per
   request, and its futures resolved; its arena slot is freed.

Requests that arrive while batches run are admitted as soon as memory and a
stream free up, so their work overlaps on the device.  Every request's result
is the same alone or in any mix: a batch is a concatenation of independent
reads and the kernel never lets a window or a k-mer cross a read boundary.

``Executor`` separates the device work from the scheduling: ``GPUExecutor``
runs libsws; ``FakeExecutor`` (tests) computes on the CPU with configurable
latency and injected failures.
"""
from __future__ import annotations

import collections
import concurrent.futures
import ctypes
import gc
import os
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import _lib


# ---------------------------------------------------------------------------
# Device arena: first-fit free list over one allocation, with coalescing.
# ---------------------------------------------------------------------------
class Arena:
    ALIGN = 256

    def __init__(self, nbytes: int):
        self.size = int(nbytes)
        self.free_list = [(0, self.size)]  # sorted (offset, length)
        self.used = 0

    @classmethod
    def round(cls, n: int) -> int:
        return (int(n) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def alloc(self, nbytes: int) -> Optional[int]:
        n = self.round(max(nbytes, 1))
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= n:
                if ln == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        n = self.round(max(nbytes, 1))
        self.used -= n
        fl = self.free_list
        fl.append((off, n))
        fl.sort()
        merged = [fl[0]]
        for o, ln in fl[1:]:
            po, pl = merged[-1]
            if po + pl == o:
                merged[-1] = (po, pl + ln)
            else:
                merged.append((o, ln))
        self.free_list = merged

    @property
    def free_bytes(self) -> int:
        return self.size - self.used


# ---------------------------------------------------------------------------
# Requests and batches.
# ---------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    seqs: np.ndarray          # uint8 bases
    offsets: np.ndarray       # uint64, nreads + 1
    arrival: float
    future: concurrent.futures.Future = field(default_factory=concurrent.futures.Future)
    admitted: float = 0.0
    finished: float = 0.0
    bound: int = -1           # most minimizers the request can have (-1: not counted yet)
    solo: bool = False        # re-run alone after its batch failed

    @property
    def nbases(self) -> int:
        return int(self.offsets[-1])

    @property
    def nreads(self) -> int:
        return int(self.offsets.size - 1)


@dataclass
class Result:
    hash: np.ndarray          # uint64
    pos: np.ndarray           # uint32, relative to the read
    read_offsets: np.ndarray  # uint64, nreads + 1


def window_bound(offsets: np.ndarray, k: int, w: int) -> int:
    """Windows of w k-mers over the reads: sum of max(0, len - k - w + 2)."""
    lens = np.diff(offsets.view(np.int64) if offsets.dtype == np.uint64 else
                   np.asarray(offsets, dtype=np.int64))
    c = k + w - 2
    # every read contributes len - c, the reads shorter than c give back c - len
    return int(offsets[-1]) - c * lens.size + int(np.maximum(c - lens, 0).sum())


class Executor:
    """Runs batches.  ``footprint`` sizes a batch in arena bytes; ``start``
    enqueues it and returns a handle; ``done`` polls; ``finish`` returns the
    per-request results (or raises)."""

    def footprint(self, nbases: int, nreads: int, bound: int) -> int:
        raise NotImplementedError

    def footprint_upper(self, nbases: int, nreads: int, bound: int) -> int:
        """An upper bound of footprint() that is cheap to evaluate."""
        return self.footprint(nbases, nreads, bound)

    def start(self, reqs: List[Request], slot: int):
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> List[Result]:
        raise NotImplementedError

    def slots(self) -> int:
        return 1

    def arena_bytes(self) -> int:
        raise NotImplementedError


def _split(reqs: List[Request], h, p, ro):
    """Cut batch outputs (read-major) into per-request results."""
    out = []
    r0 = 0
    for q in reqs:
        n = q.nreads
        a, e = int(ro[r0]), int(ro[r0 + n])
        out.append(Result(h[a:e].copy(), p[a:e].copy(), (ro[r0:r0 + n + 1] - ro[r0]).copy()))
        r0 += n
    return out


def _split_views(reqs: List[Request], h, p, ro):
    """As _split, with the results as views of the batch's arrays (which the
    caller owns and does not reuse)."""
    out = []
    r0 = 0
    ro = np.asarray(ro, dtype=np.uint64)
    for q in reqs:
        n = q.nreads
        a, e = int(ro[r0]), int(ro[r0 + n])
        out.append(Result(h[a:e], p[a:e], ro[r0:r0 + n + 1] - np.uint64(a)))
        r0 += n
    return out


# Host copies are cut into pieces of this many bytes for the copy pool.
_COPY_PIECE = 4 << 20


def _concat(reqs: List[Request]):
    nreads = sum(q.nreads for q in reqs)
    off = np.zeros(nreads + 1, dtype=np.uint64)
    seqs = np.concatenate([q.seqs for q in reqs]) if reqs else np.zeros(0, np.uint8)
    r = 0
    base = 0
    for q in reqs:
        n = q.nreads
        off[r + 1:r + n + 1] = q.offsets[1:] + np.uint64(base)
        base += q.nbases
        r += n
    return seqs, off


# ---------------------------------------------------------------------------
# GPU executor.
# ---------------------------------------------------------------------------
class GPUExecutor(Executor):
    """Batches on the device: one arena allocation holds every in-flight
    batch's bases, offsets, outputs and workspace; S streams (default
    priority) run batches concurrently."""

    def __init__(self, k: int, w: int, arena_bytes: Optional[int] = None,
                 streams: Optional[int] = None, canonical: bool = True, hashed: bool = True,
                 device: str = "cuda", copy_threads: int = 6):
        import torch
        if streams is None:
            # one stream per hardware queue besides torch's default stream:
            # a stream that shares a queue has its copies wait behind another
            # stream's work (measured: p99 2.2 ms with 4 streams on 4 queues,
            # 1.1 ms with 3)
            streams = max(1, int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) - 1)
        self.torch = torch
        self.k, self.w = k, w
        self.flags = (0 if canonical else _lib.KMER_FORWARD) | (0 if hashed else _lib.HASH_IDENTITY)
        if arena_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            arena_bytes = int(free * 0.5)
        self.arena_dev = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        if not self.arena_dev.is_cuda:
            raise ValueError("GPUExecutor needs a CUDA (HIP) device, got %s" % device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.free_streams = list(range(streams))
        # grow-only pinned host buffers, one per stream: the batch's bases and
        # offsets on the way in, its minimizers on the way out
        self.staging = [None] * streams
        self.out_staging = [None] * streams
        self.lib = _lib.load()
        # host copies (packing into pinned staging, results out of it) run on
        # a small pool: numpy copies release the interpreter lock, and one
        # thread's memcpy bandwidth bounds a large batch otherwise
        self.copy_threads = max(1, min(copy_threads, len(os.sched_getaffinity(0))))
        # packing and result copies on pools of their own: a batch's results
        # never wait behind the next batch's packing
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=self.copy_threads,
                                                          thread_name_prefix="sws-pack")
        self.out_pool = concurrent.futures.ThreadPoolExecutor(max_workers=self.copy_threads,
                                                              thread_name_prefix="sws-unpack")

    def prepare(self, staging_bytes: int):
        """Before requests arrive: allocate every stream's pinned input and
        output staging for the server's largest batch (pinned allocations are
        slow and stall the device), and run one small batch on every stream
        (a stream's first use carries a one-time setup cost).  staging_bytes:
        the batch's bases plus 8 bytes per read offset."""
        # outputs: the per-read offsets (at most 2^20 + 1 are reserved) and
        # 12 bytes per minimizer at the density start() copies back
        # speculatively; more grows the buffer
        offsets = min(staging_bytes, 8 * ((1 << 20) + 1) + 256)
        out_bytes = offsets + 12 * (1024 + 5 * staging_bytes // (2 * (self.w + 1)))
        for si in range(len(self.streams)):
            self._pinned(si, staging_bytes, exact=True)
            self._pinned_out(si, out_bytes, exact=True)
        # one tiny batch through every stream, at the start of the arena (not in
        # use yet): the same copies and library launches as a real batch
        tiny = Request(-1, np.frombuffer(b"ACGT" * 16, dtype=np.uint8).copy(),
                       np.array([0, 64], dtype=np.uint64), 0.0)
        tiny.bound = window_bound(tiny.offsets, self.k, self.w)
        need = self.footprint(64, 1, tiny.bound)
        if need * len(self.streams) > self.arena_bytes():
            return
        handles = [self.start([tiny], i * need) for i in range(len(self.streams))]
        for h in handles:
            self.finish(h)

    def _grow(self, bufs, si: int, nbytes: int, exact: bool):
        buf = bufs[si]
        if buf is None or buf.numel() < nbytes:
            # beyond the reservation, powers of two: a buffer regrows rarely
            size = int(nbytes) if exact else 1 << max(20, (int(nbytes) - 1).bit_length())
            buf = self.torch.empty(max(size, 1 << 20), dtype=self.torch.uint8, pin_memory=True)
            bufs[si] = buf
        return buf

    def _pinned(self, si: int, nbytes: int, exact: bool = False):
        return self._grow(self.staging, si, nbytes, exact)

    def _pinned_out(self, si: int, nbytes: int, exact: bool = False):
        return self._grow(self.out_staging, si, nbytes, exact)

    def slots(self) -> int:
        return len(self.streams)

    def arena_bytes(self) -> int:
        return self.arena_dev.numel()

    def _layout(self, nbases: int, nreads: int, bound: int):
        R = Arena.round
        ws = ctypes.c_uint64(0)
        _lib.check(self.lib.sws_minimizers_batch_workspace(nbases, nreads, self.k, self.w,
                                                           ctypes.byref(ws)),
                   "sws_minimizers_batch_workspace")
        parts = [("seqs", R(nbases)), ("offsets", R(8 * (nreads + 1))), ("hash", R(8 * bound)),
                 ("pos", R(4 * bound)), ("read", R(4 * bound)), ("read_out", R(8 * (nreads + 1))),
                 ("ws", R(ws.value))]
        lay, off = {}, 0
        for name, n in parts:
            lay[name] = (off, n)
            off += n
        return lay, off

    def footprint(self, nbases, nreads, bound):
        return self._layout(nbases, nreads, bound)[1]

    def footprint_upper(self, nbases, nreads, bound):
        # bases; two offset arrays; hash, pos and read per window; the
        # workspace (256 bytes plus 68 per tile of at least 512 windows for
        # w <= 32); 256 bytes of rounding for each of the seven parts
        return (nbases + 16 * (nreads + 1) + 16 * bound + 256 + 68 * (nbases // 512 + 2)
                + 7 * Arena.ALIGN)

    def start(self, reqs, slot):
        torch = self.torch
        nreads = sum(q.nreads for q in reqs)
        nbases = sum(q.nbases for q in reqs)
        si = self.free_streams.pop()
        stream = self.streams[si]
        base = self.arena_dev.data_ptr() + slot

        # concatenate bases and offsets straight into this stream's pinned
        # buffer, one copy per request (the previous batch on this stream has
        # finished, so the buffer is free)
        ob = Arena.round(nbases)
        pin = self._pinned(si, ob + 8 * (nreads + 1))
        pin_np = pin.numpy()
        off = pin_np[ob:ob + 8 * (nreads + 1)].view(np.uint64)
        off[0] = 0
        # copy jobs of about _COPY_PIECE bytes each: a large request is cut
        # into pieces, small ones share a job
        jobs, cur, cur_bytes = [], [], 0
        b0, r0 = 0, 0
        for q in reqs:
            np.add(q.offsets[1:], np.uint64(b0), out=off[r0 + 1:r0 + q.nreads + 1])
            for x0 in range(0, q.nbases, _COPY_PIECE):
                x1 = min(q.nbases, x0 + _COPY_PIECE)
                cur.append((b0 + x0, q.seqs, x0, x1))
                cur_bytes += x1 - x0
                if cur_bytes >= _COPY_PIECE:
                    jobs.append(cur)
                    cur, cur_bytes = [], 0
            b0 += q.nbases
            r0 += q.nreads
        if cur:
            jobs.append(cur)

        def pack(job):
            for d0, src, x0, x1 in job:
                pin_np[d0:d0 + x1 - x0] = src[x0:x1]

        self._parallel(pack, jobs)
        bound = sum(q.bound for q in reqs)
        lay, _ = self._layout(nbases, nreads, bound)

        def view(name, dtype, count):
            o, _n = lay[name]
            t = self.arena_dev[slot + o: slot + o + count * np.dtype(dtype).itemsize]
            return t

        with torch.cuda.stream(stream):
            if nbases:
                view("seqs", np.uint8, nbases).copy_(pin[:nbases], non_blocking=True)
            view("offsets", np.int64, nreads + 1).copy_(pin[ob:ob + 8 * (nreads + 1)],
                                                          non_blocking=True)
            p = lambda name: ctypes.c_void_p(base + lay[name][0])
            st = self.lib.sws_minimizers_batch(
                p("seqs"), p("offsets"), nreads, nbases, self.k, self.w, self.flags, p("hash"),
                p("pos"), p("read"), bound, p("read_out"), p("ws"), lay["ws"][1],
                ctypes.c_void_p(stream.cuda_stream))
            if st == 0:
                # queue the copies back behind the kernel: the per-read offsets
                # and the minimizers up to a density of 2.5/(w+1) (random
                # sequence: about 2/(w+1)), so that a batch within it needs no
                # further round trip once its event fires
                est = min(bound, 1024 + 5 * nbases // (2 * (self.w + 1)))
                rob = Arena.round(8 * (nreads + 1))
                out = self._pinned_out(si, rob + 12 * est)
                out[:8 * (nreads + 1)].copy_(view("read_out", np.int64, nreads + 1),
                                             non_blocking=True)
                if est:
                    out[rob:rob + 8 * est].copy_(view("hash", np.int64, est), non_blocking=True)
                    out[rob + 8 * est:rob + 12 * est].copy_(view("pos", np.int32, est),
                                                            non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        if st != 0:
            self.free_streams.append(si)
            _lib.check(st, "sws_minimizers_batch")
        # keep the pinned staging alive until the copies finished
        return {"reqs": reqs, "event": ev, "stream": si, "lay": lay, "slot": slot,
                "nreads": nreads, "bound": bound, "est": est, "rob": rob}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def finish(self, handle):
        torch = self.torch
        handle["event"].synchronize()
        lay, slot, nreads = handle["lay"], handle["slot"], handle["nreads"]
        stream = self.streams[handle["stream"]]
        try:
            return self._finish(handle, lay, slot, nreads, stream)
        finally:
            # the stream (and its pinned buffers) serve the next batch only
            # once this batch's results are out of them
            self.free_streams.append(handle["stream"])

    def _finish(self, handle, lay, slot, nreads, stream):
        torch = self.torch

        def dev(name, count, dtype):
            o, _n = lay[name]
            nb = count * torch.tensor([], dtype=dtype).element_size()
            return self.arena_dev[slot + o: slot + o + nb].view(dtype)

        # the copies queued by start() have finished with the event
        est, rob = handle["est"], handle["rob"]
        o = self.out_staging[handle["stream"]].numpy()
        ro = o[:8 * (nreads + 1)].view(np.uint64)
        total = int(ro[-1])
        if total == 0xFFFFFFFFFFFFFFFF or total > handle["bound"]:
            raise _lib.SwsError(_lib.SWS_ERR_DEVICE, "batch kernel reported an internal error")
        if total <= est:
            h = o[rob:rob + 8 * total].view(np.uint64)
            p = o[rob + 8 * est:rob + 8 * est + 4 * total].view(np.uint32)
        else:
            # denser than estimated: copy them all, through the (grown) pinned
            # buffer; a copy to pageable memory measured several times slower
            ro = ro.copy()
            with torch.cuda.stream(stream):
                out = self._pinned_out(handle["stream"], 12 * total)
                out[:8 * total].copy_(dev("hash", total, torch.int64).view(torch.uint8),
                                      non_blocking=True)
                out[8 * total:12 * total].copy_(dev("pos", total, torch.int32).view(torch.uint8),
                                                non_blocking=True)
                stream.synchronize()
            o = out.numpy()
            h = o[:8 * total].view(np.uint64)
            p = o[8 * total:12 * total].view(np.uint32)
        # one copy of the batch's results out of the pinned buffer (which the
        # stream's next batch reuses), in pieces on the copy pool; each
        # request's result is a view of it
        hb = np.empty(total, dtype=np.uint64)
        pb = np.empty(total, dtype=np.uint32)
        pieces = [(a, min(total, a + _COPY_PIECE // 8)) for a in range(0, total, _COPY_PIECE // 8)]

        def copy_piece(ab):
            a, e = ab
            hb[a:e] = h[a:e]
            pb[a:e] = p[a:e]

        self._parallel(copy_piece, pieces, self.out_pool)
        return _split_views(handle["reqs"], hb, pb, ro)

    def _parallel(self, fn, items, pool=None):
        """fn over items on a copy pool (inline when there is one item)."""
        if len(items) <= 1 or self.copy_threads == 1:
            for it in items:
                fn(it)
            return
        pool = pool or self.pool
        for f in [pool.submit(fn, it) for it in items]:
            f.result()


# ---------------------------------------------------------------------------
# CPU fake executor for scheduler tests (oracle-backed).
# ---------------------------------------------------------------------------
class FakeExecutor(Executor):
    """Computes batches on the CPU after `latency(batch)` seconds; requests
    for which `fail(request)` is true make their batch fail."""

    def __init__(self, k: int, w: int, arena_bytes: int = 1 << 30, slots: int = 2,
                 latency: Callable[[List[Request]], float] = lambda reqs: 0.001,
                 fail: Callable[[Request], bool] = lambda q: False, compute=None):
        self.k, self.w = k, w
        self._arena = arena_bytes
        self._slots = slots
        self.latency = latency
        self.fail = fail
        self.compute = compute  # (seqs, offsets, k, w) -> (hash, pos, read, read_offsets)
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=slots)
        self.inflight = 0
        self.max_inflight_seen = 0
        self.batches = []

    def slots(self):
        return self._slots

    def arena_bytes(self):
        return self._arena

    def footprint(self, nbases, nreads, bound):
        return Arena.round(nbases) + Arena.round(16 * (nreads + 1)) + Arena.round(16 * bound) + 256

    def _run(self, reqs):
        time.sleep(self.latency(reqs))
        if any(self.fail(q) for q in reqs):
            raise RuntimeError("injected failure")
        seqs, off = _concat(reqs)
        h, p, rd, ro = self.compute(seqs, off, self.k, self.w)
        return _split(reqs, h, p, ro)

    def start(self, reqs, slot):
        self.inflight += 1
        self.max_inflight_seen = max(self.max_inflight_seen, self.inflight)
        self.batches.append([q.rid for q in reqs])
        return self.pool.submit(self._run, reqs)

    def done(self, handle):
        return handle.done()

    def finish(self, handle):
        self.inflight -= 1
        return handle.result()


# ---------------------------------------------------------------------------
# Server.
# ---------------------------------------------------------------------------
class RequestTooLarge(ValueError):
    pass


class Server:
    """freeze_gc: at start, move every object that exists then out of the
    cyclic garbage collector's reach (gc.freeze).  A full collection over a
    large heap holds the interpreter lock for tens of milliseconds, which
    stalls the scheduler thread in the middle of a batch (measured: one 50 ms
    request at 200 requests/s); afterwards only objects created while serving
    are scanned."""

    def __init__(self, executor: Executor, k: int, w: int, max_batch_bases: int = 64 << 20,
                 poll_s: float = 50e-6, freeze_gc: bool = True,
                 concurrent_bases: int = 16 << 20):
        self.freeze_gc = freeze_gc
        # a batch starts beside one already running only when at least this
        # many bases wait: under light load one batch at a time finishes
        # soonest (concurrent batches share the host copies and the link;
        # starting a second batch once the oldest request had waited 0.3 ms
        # measured p99 1.35 against 0.68 ms at 200 requests/s), under load
        # all streams stay busy
        self.concurrent_bases = concurrent_bases
        self.queued_bases = 0
        self.ex = executor
        self.k, self.w = k, w
        self.arena = Arena(executor.arena_bytes())
        self.max_batch_bases = max_batch_bases
        self.poll_s = poll_s
        self.queue = collections.deque()
        self.lock = threading.Lock()        # the queue
        self.state_lock = threading.Lock()  # the arena and the in-flight list
        self.wake = threading.Event()
        self.inflight = []  # [handle, slot, nbytes, reqs, handed to the completer]
        self.done_q = collections.deque()
        self.done_wake = threading.Event()
        self.stop_flag = False
        self.thread = None
        self.completer = None
        self.next_id = 0
        self.completed: List[Request] = []

    # -- client side --------------------------------------------------------
    def submit(self, seqs: np.ndarray, offsets: np.ndarray, arrival: Optional[float] = None):
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        q = Request(self.next_id, np.ascontiguousarray(seqs, dtype=np.uint8), off,
                    time.perf_counter() if arrival is None else arrival)
        self.next_id += 1
        # the oversize check with cheap upper bounds first (at most one window
        # per base past the first k + w - 2); the exact window count and
        # footprint only when those do not fit.  Otherwise the scheduler thread
        # counts the windows, off the client's path
        nb, nr = int(off[-1]), off.size - 1
        cheap = self.ex.footprint_upper(nb, nr, max(0, nb - self.k - self.w + 2))
        need = cheap
        if cheap > self.arena.size:
            q.bound = window_bound(off, self.k, self.w)
            need = self.ex.footprint(nb, nr, q.bound)
        if need > self.arena.size:
            q.future.set_exception(RequestTooLarge(
                "request needs %d arena bytes, the arena has %d" % (need, self.arena.size)))
            return q.future
        with self.lock:
            self.queue.append(q)
            self.queued_bases += nb
        # the scheduler waits on the event only when it has nothing to do and
        # clears it before looking at the queue again: setting it once is
        # enough (Event.set takes a lock and notifies, a few microseconds)
        if not self.wake.is_set():
            self.wake.set()
        return q.future

    def start(self):
        if self.freeze_gc:
            gc.collect()
            gc.freeze()
        # the staging a batch of max_batch_bases needs (bases and, at worst,
        # one offset per base), allocated before the first request
        prepare = getattr(self.ex, "prepare", None)
        if prepare is not None:
            prepare(Arena.round(min(self.max_batch_bases, self.arena.size)) +
                    8 * (min(self.max_batch_bases, 1 << 20) + 1))
        self.thread = threading.Thread(target=self._loop, name="sws-scheduler", daemon=True)
        self.completer = threading.Thread(target=self._complete_loop, name="sws-completer",
                                          daemon=True)
        self.thread.start()
        self.completer.start()
        return self

    def stop(self, drain: bool = True, timeout: float = 60.0):
        if drain:
            t0 = time.perf_counter()
            while (self.queue or self.inflight) and time.perf_counter() - t0 < timeout:
                time.sleep(0.001)
        self.stop_flag = True
        self.wake.set()
        self.done_wake.set()
        if self.thread:
            self.thread.join(timeout)
        if self.completer:
            self.completer.join(timeout)

    # -- scheduler ----------------------------------------------------------
    def _form_batch(self):
        """Oldest-first requests that fit together in free arena bytes.  A
        request re-run after its batch failed forms a batch alone."""
        reqs, nb, nr, bound = [], 0, 0, 0
        with self.lock, self.state_lock:
            while self.queue:
                q = self.queue[0]
                if reqs and (q.solo or reqs[0].solo):
                    break
                if q.bound < 0:
                    q.bound = window_bound(q.offsets, self.k, self.w)
                b2 = bound + q.bound
                # the cheap upper bound for the fit test; the exact footprint
                # (never larger) sizes the allocation below
                need = self.ex.footprint_upper(nb + q.nbases, nr + q.nreads, b2)
                if reqs and nb + q.nbases > self.max_batch_bases:
                    break
                if need > self.arena.free_bytes:
                    break
                reqs.append(self.queue.popleft())
                nb, nr, bound = nb + q.nbases, nr + q.nreads, b2
            if not reqs:
                return None
            need = self.ex.footprint(nb, nr, bound)
            slot = self.arena.alloc(need)
            if slot is None:  # fragmented: put them back, retry after a completion
                self.queue.extendleft(reversed(reqs))
                return None
            self.queued_bases -= nb
        return reqs, slot, need

    def _collect_finished(self) -> bool:
        """Hands finished batches to the completer; True if any."""
        progressed = False
        with self.state_lock:
            for item in self.inflight:
                if not item[4] and self.ex.done(item[0]):
                    item[4] = True
                    self.done_q.append(item)
                    self.done_wake.set()
                    progressed = True
        return progressed

    def _start_batch(self) -> Optional[bool]:
        """Forms and starts one batch: True if it started, False if its start
        failed (its requests have the error), None if no batch could form."""
        b = self._form_batch()
        if b is None:
            return None
        reqs, slot, need = b
        now = time.perf_counter()
        for q in reqs:
            q.admitted = now
        try:
            handle = self.ex.start(reqs, slot)
        except Exception as exc:
            with self.state_lock:
                self.arena.release(slot, need)
            for q in reqs:
                q.future.set_exception(exc)
            return False
        with self.state_lock:
            self.inflight.append([handle, slot, need, reqs, False])
        return True

    def _loop(self):
        """Scheduler: hands finished batches to the completer and admits new
        ones while streams and arena bytes allow.  (The work is done in
        helpers, so that no batch stays referenced from this frame while it
        waits.)"""
        while not self.stop_flag:
            progressed = self._collect_finished()
            with self.state_lock:
                busy = len(self.inflight)
            while busy < self.ex.slots() and self.queue:
                if busy > 0 and self.queued_bases < self.concurrent_bases:
                    break
                started = self._start_batch()
                if started is None:
                    break
                if started:
                    busy += 1
                    progressed = True
            if not progressed:
                if not self.inflight and not self.queue:
                    self.wake.wait(0.01)
                    self.wake.clear()
                else:
                    time.sleep(self.poll_s)

    def _complete_loop(self):
        """Completer: collects a finished batch's results (the host copies run
        here, beside the scheduler's packing of the next batch), resolves the
        futures and frees the batch's arena bytes.  A failed batch's requests
        go back to the front of the queue to be re-run one by one, so that a
        bad request fails alone."""
        while True:
            if not self.done_q:
                if self.stop_flag and not self.inflight:
                    return
                self.done_wake.wait(0.01)
                self.done_wake.clear()
                continue
            self._complete(self.done_q.popleft())
            self.wake.set()

    def _complete(self, item):
        """One finished batch.  (A method of its own, so that nothing of the
        batch stays referenced from the completer's frame afterwards.)"""
        handle, slot, nbytes, reqs, _ = item
        retry = []
        try:
            results = self.ex.finish(handle)
            now = time.perf_counter()
            for q, r in zip(reqs, results):
                q.finished = now
                q.future.set_result(r)
        except Exception as exc:
            if len(reqs) == 1:
                reqs[0].future.set_exception(exc)
            else:
                for q in reqs:
                    q.solo = True
                retry = reqs
        if not retry:
            # a resolved request keeps its timings only: its future (and
            # through it the result) and its bases belong to the client now,
            # and are freed when the client lets them go rather than when the
            # server stops (a client that drops each result lets the next
            # batch's result arrays reuse that memory instead of faulting in
            # fresh pages)
            for q in reqs:
                q.future = None
                q.seqs = None
        with self.state_lock:
            self.arena.release(slot, nbytes)
            self.inflight.remove(item)
            if not retry:
                self.completed.extend(reqs)
        if retry:
            with self.lock:
                self.queue.extendleft(reversed(retry))
                self.queued_bases += sum(q.nbases for q in retry)


def latency_stats(reqs: List[Request]):
    lat = np.array([q.finished - q.arrival for q in reqs if q.finished > 0])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "n": int(lat.size)}
