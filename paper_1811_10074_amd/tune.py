"""Autotuner for the minimizer kernels' workgroup size per read-length bucket.

For each bucket present in a sample batch it times every candidate block size
(64, 128, 256, 512 threads: 1, 2, 4 or 8 wavefront tiles per workgroup) with HIP
events and keeps the fastest.  The table is persisted as JSON keyed by GPU
architecture, library ABI version, k and w, and applied with
``sws_set_minimizer_block``.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib
from .batch import BatchRunner, bucket_of_length, set_block

CANDIDATES = (64, 128, 256, 512)
DEFAULT_PATH = os.environ.get("SWS_TUNE_FILE",
                              os.path.join(os.path.expanduser("~"), ".cache", "sws", "tune.json"))


def _key(k: int, w: int) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return "%s/abi%d/k%d/w%d" % (arch, _lib.load().sws_abi_version(), k, w)


def time_runner(runner: BatchRunner, reps: int = 5, warmup: int = 2) -> float:
    import torch
    for _ in range(warmup):
        runner.launch()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        runner.launch()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(seqs_np: np.ndarray, offsets_np: np.ndarray, k: int, w: int, reps: int = 5):
    """Returns {bucket: threads} for the buckets present in the sample."""
    import torch
    off = np.asarray(offsets_np, dtype=np.int64)
    lens = np.diff(off)
    buckets = np.digitize(lens, (1000, 16000))
    table, timings = {}, {}
    for b in sorted(set(buckets.tolist())):
        sel = np.nonzero(buckets == b)[0]
        blens = lens[sel]
        boff = np.zeros(sel.size + 1, dtype=np.uint64)
        np.cumsum(blens, out=boff[1:])
        bseq = seqs_np[np.repeat(buckets == b, lens)]
        runner = BatchRunner(torch.from_numpy(bseq).cuda(), boff, k, w)
        best = None
        for t in CANDIDATES:
            set_block(int(b), t)
            ms = time_runner(runner, reps=reps)
            timings["%d/%d" % (b, t)] = ms
            if best is None or ms < best[1]:
                best = (t, ms)
        table[int(b)] = best[0]
        set_block(int(b), best[0])
    return table, timings


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


def apply(table) -> None:
    for b, t in (table or {}).items():
        set_block(int(b), int(t))
