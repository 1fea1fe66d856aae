"""CPU oracle for sliding window sums and minimizer seed tables.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the library and its product path never
do.  It shares no code with the HIP implementation.

``oracle.c`` holds the arithmetic (plain C loops, each routine citing the
passage of Snytsar & Turakhia, arXiv:1811.10074, that it writes out).  This
module only marshals numpy arrays into it.  ``brute.py`` is a second, tiny,
pure-Python formulation used to check ``oracle.c`` on small inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OPS = {"add": 0, "min": 1, "max": 2, "affine": 3}
FORWARD = 1   # forward k-mer instead of canonical
IDENTITY = 2  # k-mer value instead of its hash
SPLIT = 4     # invalid bases split the sequence into segments

_lock = threading.Lock()
_lib = None


def build(out: str = LIB_PATH, src: str = _SRC, extra_flags=()) -> str:
    """Compile oracle.c with gcc into a shared library (always recompiles)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *extra_flags, "-o", tmp, src]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(lib):
    u64, u32p, u64p, u8p = (ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint8))
    ll = ctypes.c_longlong
    lib.oracle_sliding_sum.argtypes = [ctypes.c_int, u64, u32p, u64, u32p]
    lib.oracle_sliding_sum.restype = ll
    lib.oracle_sliding_extremum_deque.argtypes = [ctypes.c_int, u64, u32p, u64, u32p]
    lib.oracle_sliding_extremum_deque.restype = ll
    lib.oracle_affine_windows_by_prefix.argtypes = [u64, u32p, u64, u32p]
    lib.oracle_affine_windows_by_prefix.restype = ll
    lib.oracle_mix64.argtypes = [u64]
    lib.oracle_mix64.restype = u64
    lib.oracle_mix64_inv.argtypes = [u64]
    lib.oracle_mix64_inv.restype = u64
    lib.oracle_mix64_array.argtypes = [u64p, u64, ctypes.c_int, u64p]
    lib.oracle_mix64_array.restype = None
    lib.oracle_base_code.argtypes = [ctypes.c_uint8]
    lib.oracle_base_code.restype = ctypes.c_int
    lib.oracle_kmers.argtypes = [u8p, u64, ctypes.c_uint32, ctypes.c_uint32, u64p]
    lib.oracle_kmers.restype = ll
    lib.oracle_seed_table.argtypes = [u64p, u32p, u64, ctypes.c_uint32, ctypes.c_uint32, u64p,
                                      u32p, u64p]
    lib.oracle_seed_table.restype = ctypes.c_int
    for name in ("oracle_minimizers_naive", "oracle_minimizers_deque"):
        f = getattr(lib, name)
        f.argtypes = [u8p, u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                      u64p, u32p, u64]
        f.restype = ll
    lib.oracle_minimizers_batch.argtypes = [u8p, u64p, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_uint32, u64p, u32p,
                                            u32p, u64, u64p]
    lib.oracle_minimizers_batch.restype = ll
    return lib


def load(path: str | None = None):
    """Load liboracle.so (building it first only when it does not exist).

    With ``path`` given, load that library (e.g. a deliberately mutated build)
    without caching it."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_bytes(seq) -> np.ndarray:
    if isinstance(seq, (bytes, bytearray)):
        return np.frombuffer(bytes(seq), dtype=np.uint8)
    if isinstance(seq, str):
        return np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    return np.ascontiguousarray(seq, dtype=np.uint8)


def sliding_sum(op: str, w: int, x: np.ndarray, lib=None) -> np.ndarray:
    """Eq. 2 as a left fold.  x: uint32[n] (uint32[n, 2] of (a, b) for affine)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    pair = op == "affine"
    n = x.shape[0]
    if pair and (x.ndim != 2 or x.shape[1] != 2):
        raise ValueError("affine input must be uint32[n, 2]")
    cnt = max(0, n - w + 1) if w >= 1 else 0
    y = np.zeros((cnt, 2) if pair else (cnt,), dtype=np.uint32)
    r = lib.oracle_sliding_sum(OPS[op], w, _ptr(x, ctypes.c_uint32), n,
                               _ptr(y, ctypes.c_uint32))
    if r < 0:
        raise ValueError("oracle_sliding_sum rejected op=%s w=%d" % (op, w))
    assert r == cnt
    return y


def sliding_extremum_deque(op: str, w: int, x: np.ndarray, lib=None) -> np.ndarray:
    """min or max over every window of w by the monotone deque, O(N)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    n = x.shape[0]
    cnt = max(0, n - w + 1) if w >= 1 else 0
    y = np.zeros(cnt, dtype=np.uint32)
    r = lib.oracle_sliding_extremum_deque(OPS[op], w, _ptr(x, ctypes.c_uint32), n,
                                          _ptr(y, ctypes.c_uint32))
    if r < 0:
        raise ValueError("oracle_sliding_extremum_deque rejected op=%s w=%d" % (op, w))
    assert r == cnt
    return y


def affine_windows_by_prefix(w: int, x: np.ndarray, lib=None) -> np.ndarray:
    """Affine windows of x (uint32[n, 2], every multiplier odd) as
    P_i^{-1} o P_{i+w} from prefix compositions, O(N)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.uint32)
    if x.ndim != 2 or x.shape[1] != 2:
        raise ValueError("affine input must be uint32[n, 2]")
    n = x.shape[0]
    cnt = max(0, n - w + 1) if w >= 1 else 0
    y = np.zeros((cnt, 2), dtype=np.uint32)
    r = lib.oracle_affine_windows_by_prefix(w, _ptr(x, ctypes.c_uint32), n, _ptr(y, ctypes.c_uint32))
    if r == -2:
        raise ValueError("affine_windows_by_prefix needs odd multipliers")
    if r < 0:
        raise ValueError("affine_windows_by_prefix rejected w=%d" % w)
    assert r == cnt
    return y


def mix64(x, inverse: bool = False, lib=None):
    lib = lib or load()
    if np.isscalar(x):
        return int((lib.oracle_mix64_inv if inverse else lib.oracle_mix64)(int(x)))
    x = np.ascontiguousarray(x, dtype=np.uint64)
    y = np.empty_like(x)
    lib.oracle_mix64_array(_ptr(x, ctypes.c_uint64), x.size, int(inverse),
                           _ptr(y, ctypes.c_uint64))
    return y


def flags_of(canonical: bool = True, hashed: bool = True, split: bool = False) -> int:
    return (0 if canonical else FORWARD) | (0 if hashed else IDENTITY) | (SPLIT if split else 0)


def kmers(seq, k: int, canonical: bool = True, hashed: bool = True, lib=None) -> np.ndarray:
    lib = lib or load()
    s = _as_bytes(seq)
    n = s.size
    out = np.zeros(max(0, n - k + 1), dtype=np.uint64)
    r = lib.oracle_kmers(_ptr(s, ctypes.c_uint8), n, k, flags_of(canonical, hashed),
                         _ptr(out, ctypes.c_uint64))
    if r < 0:
        raise ValueError("oracle_kmers rejected k=%d" % k)
    return out


def window_bound(n: int, k: int, w: int) -> int:
    """Number of windows of w k-mers in a sequence of n bases."""
    return max(0, n - k - w + 2)


def minimizers(seq, k: int, w: int, canonical: bool = True, hashed: bool = True,
               method: str = "deque", lib=None, split: bool = False):
    """Deduplicated (hash uint64, pos uint32) minimizers of one sequence
    (split: invalid bases cut it into segments, see oracle.c)."""
    lib = lib or load()
    s = _as_bytes(seq)
    n = s.size
    cap = window_bound(n, k, w)
    h = np.zeros(max(cap, 1), dtype=np.uint64)
    p = np.zeros(max(cap, 1), dtype=np.uint32)
    f = lib.oracle_minimizers_naive if method == "naive" else lib.oracle_minimizers_deque
    r = f(_ptr(s, ctypes.c_uint8), n, k, w, flags_of(canonical, hashed, split),
          _ptr(h, ctypes.c_uint64), _ptr(p, ctypes.c_uint32), cap)
    if r < 0:
        raise ValueError("oracle minimizers rejected k=%d w=%d" % (k, w))
    assert r <= cap
    return h[:r].copy(), p[:r].copy()


def minimizers_batch(seqs: np.ndarray, offsets: np.ndarray, k: int, w: int,
                     canonical: bool = True, hashed: bool = True, lib=None, split: bool = False):
    """Per-read minimizers of reads seqs[offsets[r]:offsets[r+1]].

    Returns (hash, pos, read, read_offsets) with read-major order, pos relative
    to the read start, read_offsets of length nreads + 1."""
    lib = lib or load()
    s = _as_bytes(seqs)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nreads = off.size - 1
    lens = np.diff(off.astype(np.int64))
    cap = int(np.maximum(lens - k - w + 2, 0).sum())
    h = np.zeros(max(cap, 1), dtype=np.uint64)
    p = np.zeros(max(cap, 1), dtype=np.uint32)
    rd = np.zeros(max(cap, 1), dtype=np.uint32)
    ro = np.zeros(nreads + 1, dtype=np.uint64)
    r = lib.oracle_minimizers_batch(_ptr(s, ctypes.c_uint8), _ptr(off, ctypes.c_uint64),
                                    nreads, k, w, flags_of(canonical, hashed, split),
                                    _ptr(h, ctypes.c_uint64), _ptr(p, ctypes.c_uint32),
                                    _ptr(rd, ctypes.c_uint32), cap,
                                    _ptr(ro, ctypes.c_uint64))
    if r < 0:
        raise ValueError("oracle batch minimizers rejected k=%d w=%d" % (k, w))
    return h[:r].copy(), p[:r].copy(), rd[:r].copy(), ro


def seed_table(hash_, pos, bits: int, shift: int, lib=None):
    """Seed pointer table (uint64[2^bits + 1]) and the positions and hashes
    grouped by key = (hash >> shift) mod 2^bits, each group in input order."""
    lib = lib or load()
    h = np.ascontiguousarray(hash_, dtype=np.uint64)
    p = np.ascontiguousarray(pos, dtype=np.uint32)
    if h.size != p.size:
        raise ValueError("hash and pos differ in length")
    ptr = np.zeros((1 << bits) + 1, dtype=np.uint64)
    po = np.zeros(max(p.size, 1), dtype=np.uint32)
    ho = np.zeros(max(h.size, 1), dtype=np.uint64)
    r = lib.oracle_seed_table(_ptr(h, ctypes.c_uint64), _ptr(p, ctypes.c_uint32), h.size, bits,
                              shift, _ptr(ptr, ctypes.c_uint64), _ptr(po, ctypes.c_uint32),
                              _ptr(ho, ctypes.c_uint64))
    if r != 0:
        raise ValueError("oracle seed table rejected bits=%d shift=%d" % (bits, shift))
    return ptr, po[:p.size].copy(), ho[:h.size].copy()


def host_threads() -> int:
    """Threads this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def minimizers_batch_parallel(seqs, offsets, k: int, w: int, canonical: bool = True,
                              hashed: bool = True, threads: int | None = None,
                              split: bool = False):
    """minimizers_batch over groups of consecutive reads on several threads.

    Reads are independent sequences, so each group runs the same C routine on
    its own reads (the call releases the interpreter lock); the groups'
    results are concatenated with their read ids and offsets shifted."""
    from concurrent.futures import ThreadPoolExecutor
    lib = load()
    s = _as_bytes(seqs)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    nreads = off.size - 1
    threads = threads or host_threads()
    ngroups = max(1, min(nreads, 4 * threads))
    # group boundaries at about equal numbers of bases
    targets = np.linspace(0, float(off[-1]), ngroups + 1)
    cuts = np.unique(np.concatenate([[0], np.searchsorted(off[1:].astype(np.float64), targets[1:-1],
                                                          side="left") + 1, [nreads]]))
    cuts = [int(c) for c in cuts if 0 <= c <= nreads]

    def run(g):
        r0, r1 = cuts[g], cuts[g + 1]
        b0 = int(off[r0])
        sub = s[b0:int(off[r1])]
        h, p, rd, ro = minimizers_batch(sub, off[r0:r1 + 1] - np.uint64(b0), k, w, canonical,
                                        hashed, lib=lib, split=split)
        return h, p, rd + np.uint32(r0), ro

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(run, range(len(cuts) - 1)))
    ro_all = np.zeros(nreads + 1, dtype=np.uint64)
    base = 0
    for g, (_, _, _, ro) in enumerate(parts):
        r0, r1 = cuts[g], cuts[g + 1]
        ro_all[r0:r1 + 1] = ro + np.uint64(base)
        base += int(ro[-1])
    if not parts:
        return (np.zeros(0, np.uint64), np.zeros(0, np.uint32), np.zeros(0, np.uint32), ro_all)
    return (np.concatenate([q[0] for q in parts]), np.concatenate([q[1] for q in parts]),
            np.concatenate([q[2] for q in parts]), ro_all)


def minimizers_chunked(seq, k: int, w: int, canonical: bool = True, hashed: bool = True,
                       threads: int | None = None, chunks: int | None = None,
                       split: bool = False):
    """Single-sequence minimizers computed in chunks of windows on several
    threads; equals minimizers().

    Chunk c owns windows [a_c, a_{c+1}).  It runs the deque routine on the
    bases of windows a_c - 1 .. a_{c+1} - 1 (k + w - 1 bases of overlap with
    the chunk before), so that the store-once rule at a_c sees window
    a_c - 1's minimizer; the entry window a_c - 1 itself stores (it stores one
    iff it has a minimizer) belongs to the chunk before and is dropped."""
    from concurrent.futures import ThreadPoolExecutor
    lib = load()
    s = _as_bytes(seq)
    n = s.size
    nwin = window_bound(n, k, w)
    threads = threads or host_threads()
    chunks = chunks or 4 * threads
    chunks = max(1, min(chunks, nwin))
    starts = [nwin * c // chunks for c in range(chunks + 1)]
    span = k + w - 1  # bases of one window

    def run(c):
        a, b = starts[c], starts[c + 1]
        if a == b:
            return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
        lead = 1 if c > 0 else 0
        lo = a - lead
        h, p = minimizers(s[lo:b - 1 + span], k, w, canonical, hashed, lib=lib, split=split)
        drop = 0
        if lead:
            h1, _ = minimizers(s[lo:lo + span], k, w, canonical, hashed, lib=lib, split=split)
            drop = h1.size
        return h[drop:], (p[drop:] + np.uint32(lo)).astype(np.uint32)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(run, range(chunks)))
    if not parts:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    return np.concatenate([q[0] for q in parts]), np.concatenate([q[1] for q in parts])
