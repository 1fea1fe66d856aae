"""Autotuner for the batched minimizer kernel's workgroup size per read-length
bucket.

For each bucket present in a sample batch it times every candidate block size
(64, 128, 256, 512 threads: 1, 2, 4 or 8 wavefront tiles per workgroup) with HIP
events.  A candidate replaces the library default (256) only when it is faster
by more than ``MARGIN``; otherwise the bucket is reported as flat and keeps the
default, so timing noise never decides.  The block size travels with each call
(``sws_minimizers_batch_ex``): tuning changes no process-wide state.  The table
is persisted as JSON keyed by GPU architecture, library ABI version, k and w.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib
from .batch import BUCKET_LIMITS, BatchRunner

CANDIDATES = (64, 128, 256, 512)
DEFAULT_THREADS = 256
MARGIN = 0.03  # a candidate must beat the default by more than 3%
DEFAULT_PATH = os.environ.get("SWS_TUNE_FILE",
                              os.path.join(os.path.expanduser("~"), ".cache", "sws", "tune.json"))


def _key(k: int, w: int) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return "%s/abi%d/k%d/w%d" % (arch, _lib.load().sws_abi_version(), k, w)


def time_runner(runner: BatchRunner, threads: int, reps: int = 5, warmup: int = 2) -> float:
    """Median ms of one launch with the given workgroup size."""
    import torch
    for _ in range(warmup):
        runner.launch(threads)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        runner.launch(threads)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def choose(timings: dict, margin: float = MARGIN):
    """(threads, flat) from {threads: ms}: the fastest candidate if it beats the
    default by more than margin, else the default; flat when every candidate
    is within margin of the fastest."""
    best_t = min(timings, key=timings.get)
    best = timings[best_t]
    flat = all(v <= best * (1.0 + margin) for v in timings.values())
    base = timings.get(DEFAULT_THREADS)
    if base is not None and best >= base * (1.0 - margin):
        return DEFAULT_THREADS, flat
    return best_t, flat


def tune(seqs_np: np.ndarray, offsets_np: np.ndarray, k: int, w: int, reps: int = 5):
    """Returns (table {bucket: threads}, report) for the buckets present in the
    sample.  report[bucket] = {"ms": {threads: median ms}, "flat": bool}."""
    import torch
    off = np.asarray(offsets_np, dtype=np.int64)
    lens = np.diff(off)
    buckets = np.digitize(lens, BUCKET_LIMITS)
    table, report = {}, {}
    for b in sorted(set(buckets.tolist())):
        sel = np.nonzero(buckets == b)[0]
        blens = lens[sel]
        boff = np.zeros(sel.size + 1, dtype=np.uint64)
        np.cumsum(blens, out=boff[1:])
        bseq = seqs_np[np.repeat(buckets == b, lens)]
        runner = BatchRunner(torch.from_numpy(bseq).cuda(), boff, k, w)
        ms = {t: time_runner(runner, t, reps=reps) for t in CANDIDATES}
        t, flat = choose(ms)
        table[int(b)] = t
        report[int(b)] = {"ms": ms, "flat": flat}
        del runner
    return table, report


def save(table, k: int, w: int, path: str = DEFAULT_PATH) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except ValueError:
            data = {}
    data[_key(k, w)] = {str(b): t for b, t in table.items()}
    tmp = path + ".tmp"
    json.dump(data, open(tmp, "w"), indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(k: int, w: int, path: str = DEFAULT_PATH):
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    t = data.get(_key(k, w))
    return {int(b): int(v) for b, v in t.items()} if t else None
