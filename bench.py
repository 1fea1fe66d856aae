#!/usr/bin/env python3
"""Benchmark of the minimizer seed-table pass and the sliding window sums.

One step = one fused minimizer pass (2-bit coding, canonical 15-mers, mix64,
sliding minimum over w = 10, dedup, ordered emission) over a 64-Mbase i.i.d.
uniform A/C/G/T sequence (seed 1) already resident in HBM.  Prints one JSON
line.  Extras in the same line: the same pass from the pre-packed 2-bit layout,
the sliding-sum sweep (N = 2^28, w in {4, 16, 64, 256, 1024}, every operator
and path), the N = 2^20 plain sliding min/+ latency, the batched-reads
workload against one launch per read, and the serving loop.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

The CPU baseline is the oracle (test infrastructure) timed on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Integer VALU issue slots of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Issue slots per base of the minimizer pass as formulated (k <= 16, canonical,
# hashed): k-mer and reverse complement 7, mix64 37 (7 quarter-rate 32-bit
# multiplies = 28 slots, plus shifts, xors and carries), three leftmost-minimum
# combines 15, dedup and emission 3.
ALU_OPS_PER_BASE = 62
METRIC = "Gbases/s minimizers (k=15,w=10) + % HBM peak; batched vs per-read launch; p99 ms"


def profiled_traffic(profile_name):
    """HBM bytes per launch recorded in a committed rocprofv3 summary under
    profiles/, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k_, v_ = line.strip().split(":", 1)
            fields[k_.strip()] = v_.strip()
    # source: the kernel's file and the headers it includes, comma-separated;
    # source_sha256 covers their bytes concatenated in that order
    srcs = [os.path.join(ROOT, f.strip()) for f in fields.get("source", "").split(",") if f.strip()]
    if not srcs or not all(os.path.isfile(f) for f in srcs) \
            or "traffic_bytes_per_launch" not in fields:
        return None
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(f, "rb").read())
    if h.hexdigest() != fields.get("source_sha256"):
        return None
    return float(fields["traffic_bytes_per_launch"])


def profile_summary(profile_name):
    """The key: value lines and the per-kernel average durations (ns) of a
    committed rocprofv3 summary under profiles/, or None when the kernel's
    source changed since it was taken (or the summary records no source)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    fields, kernels, in_table = {}, {}, False
    for line in open(path):
        if line.startswith("Kernel statistics"):
            in_table = True
            continue
        if in_table:
            parts = line.split()
            if not parts:
                in_table = False
            elif parts[0] != "kernel" and len(parts) >= 5 and parts[-4].isdigit():
                kernels[" ".join(parts[:-4])] = float(parts[-3])
            continue
        if ":" in line:
            k_, v_ = line.strip().split(":", 1)
            fields[k_.strip()] = v_.strip()
    srcs = [os.path.join(ROOT, f.strip()) for f in fields.get("source", "").split(",") if f.strip()]
    if not srcs or not all(os.path.isfile(f) for f in srcs):
        return None
    h = hashlib.sha256()
    for f in srcs:
        h.update(open(f, "rb").read())
    if h.hexdigest() != fields.get("source_sha256"):
        return None
    return {"fields": fields, "kernels": kernels}


def profiled_kernel_us(profile_name, kernel_substr):
    prof = profile_summary(profile_name)
    if prof is None:
        return None
    for name, ns in prof["kernels"].items():
        if kernel_substr in name:
            return ns / 1e3
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_launches(torch, fn, steps, warmup):
    """Mean ms per call of `steps` calls queued back to back with events only
    around the run (an event pair around every call leaves ~10 us between
    kernels), then the median and the per-call times from a second run of
    `steps` calls with events around each."""
    mean = time_back_to_back(torch, fn, steps, warmup)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    each = sorted(a.elapsed_time(b) for a, b in evs)
    return mean, each[len(each) // 2], each


def time_back_to_back(torch, fn, steps, warmup):
    """Mean ms per call of `steps` calls queued back to back, with events only
    around the whole run (for kernels short enough that per-call events would
    show)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def cpu_info():
    """The host CPU as /proc/cpuinfo states it (model name, family/model/
    stepping, vector extensions) and the threads this process may use."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if info:
                    break
                continue
            key, val = (x.strip() for x in line.split(":", 1))
            if key in ("model name", "cpu family", "model", "stepping", "flags") and key not in info:
                info[key] = val
    except OSError:
        pass
    flags = set(info.pop("flags", "").split())
    info["vector_extensions"] = [f for f in ("avx", "avx2", "avx512f", "avx512bw", "avx512vl")
                                 if f in flags]
    info.setdefault("model name", platform.processor())
    info["threads_available"] = len(os.sched_getaffinity(0))
    return info


def _timed(fn, target_s, max_reps):
    """Repeats fn until about target_s seconds have passed; returns (reps, s)."""
    t0 = time.perf_counter()
    reps = 0
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= max_reps:
            return reps, el


def _sliding_chunked(oracle, op, w, x, threads):
    """The oracle's fold (Eq. 2, O(wN)) over contiguous output ranges on
    several threads; each range reads w - 1 inputs past its end."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    cnt = x.shape[0] - w + 1
    cuts = [cnt * i // (4 * threads) for i in range(4 * threads + 1)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda c: oracle.sliding_sum(op, w, x[cuts[c]:cuts[c + 1] + w - 1]),
                            range(4 * threads)))
    return np.concatenate(parts)


def cpu_baseline(seq_np, k, w, target_s=8.0):
    """The oracle (test infrastructure) on this host's cores, as a baseline
    only: deque minimizers over chunks of the same sequence on every thread
    this process may use (chunks of windows overlapping by k + w - 1 bases),
    single-threaded for reference, and the naive O(wN) sliding sums of the
    N = 2^20 and N = 2^28 workloads at w = 16 (the latter on a 2^26 prefix)."""
    import numpy as np
    import oracle
    from paper_1811_10074_amd import inputs

    threads = min(16, len(os.sched_getaffinity(0)))
    out = {"kind": "oracle", "unit": "Gbases/s", "cores": threads, "cpu": cpu_info()}
    # multi-threaded: the whole 64-Mbase sequence, chunked
    reps, el = _timed(lambda: oracle.minimizers_chunked(seq_np, k, w, threads=threads), target_s, 20)
    out["value"] = reps * seq_np.size / el / 1e9
    out["sample"] = ("deque minimizers (k=%d, w=%d) over the whole %d-base sequence in %d chunks "
                     "on %d threads, %d repetitions, %.1f s" % (k, w, seq_np.size, 4 * threads,
                                                               threads, reps, el))
    # one thread, a 2^24-base prefix
    pre = seq_np[: 1 << 24]
    reps1, el1 = _timed(lambda: oracle.minimizers(pre, k, w), target_s / 2, 8)
    out["single_thread"] = {"Gbases/s": reps1 * pre.size / el1 / 1e9,
                            "sample": "first 2^24 bases, %d repetitions, %.1f s" % (reps1, el1)}
    # naive sliding sums (Eq. 2 as one fold per output), Gelem/s of input
    sl = {}
    x1 = inputs.uniform_u32(1 << 20, seed=0)
    x3 = inputs.uniform_u32(1 << 26, seed=2)
    for name, x in (("n2^20_w16", x1), ("n2^28_w16_prefix2^26", x3)):
        for op in ("min", "add"):
            r, e = _timed(lambda: _sliding_chunked(oracle, op, 16, x, threads), target_s / 8, 50)
            sl["%s_%s" % (name, op)] = round(r * x.size / e / 1e9, 3)
    out["sliding_naive_Gelem_s"] = sl
    return out


def bench_sliding(torch, steps, warmup, quick):
    import numpy as np
    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import inputs

    out = {}
    x1 = torch.from_numpy(inputs.uniform_u32(1 << 20, seed=0).view(np.int32)).cuda()
    y1 = torch.empty((1 << 20) - 15, dtype=torch.int32, device="cuda")
    for op in ("min", "add"):
        ms, med, _ = time_launches(torch, lambda: sws.sliding_sum(op, 16, x1, out=y1), 50, 10)
        out["n2^20_w16_%s_us" % op] = round(med * 1000, 2)
        # the device side alone: 100 calls captured in one HIP graph, so that
        # the host's per-call cost (ctypes, argument checks) stays out
        g = torch.cuda.CUDAGraph()
        sws.sliding_sum(op, 16, x1, out=y1)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            for _ in range(100):
                sws.sliding_sum(op, 16, x1, out=y1)
        g.replay()
        torch.cuda.synchronize()
        gms = time_back_to_back(torch, g.replay, 10, 2)
        out["n2^20_w16_%s_device_us" % op] = round(gms * 1e3 / 100, 2)
        del g
    n = 1 << 28
    x = torch.from_numpy(inputs.uniform_u32(n, seed=2).view(np.int32)).cuda()
    xa = None if quick else torch.from_numpy(inputs.affine_pairs(n, seed=2).view(np.int32)).cuda()
    sweep = {}
    for op in ("add", "min", "max", "affine"):
        if op == "affine" and xa is None:
            continue
        src = xa if op == "affine" else x
        esz = 8 if op == "affine" else 4
        paths = {"min": ("generic", "log"), "max": ("generic", "log"), "add": ("generic", "prefix"),
                 "affine": ("generic",)}[op]
        for path in paths:
            for w in ((16, 1024) if quick else (4, 16, 64, 256, 1024)):
                cnt = n - w + 1
                y = torch.empty((cnt, 2) if op == "affine" else (cnt,), dtype=torch.int32, device="cuda")
                ms, med, _ = time_launches(torch, lambda: sws.sliding_sum(op, w, src, path=path, out=y),
                                           max(steps, 10), warmup)
                gbs = (n + cnt) * esz / (med / 1e3) / 1e9
                sweep["%s_%s_w%d" % (op, path, w)] = {"us": round(med * 1000, 1), "GB/s": round(gbs, 1),
                                                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)}
                del y
    out["n2^28_sweep"] = sweep
    # the plain kernel's roofline: + mod 2^32, w = 16, n = 2^28 (HBM-bound)
    ref = sweep.get("add_generic_w16")
    if ref:
        out["roofline_add_w16"] = {"bound": "hbm", "achieved": ref["GB/s"], "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(ref["GB/s"] / HBM_PEAK_GBS, 3),
                                   "traffic": profiled_traffic(
                                       "sliding_generic_kernel_add_w16_n2p28.txt")}
    return out


def bench_seed_table(torch, runner, count, steps, warmup):
    """Seed pointer + position tables (Sec. 2.4, Fig. 1) over the step's
    minimizers, keyed by the top 24 bits of the hash; algorithmic bytes =
    12 B read + 12 B written per entry + the 4-byte pointer table."""
    import paper_1811_10074_amd as sws
    bits = 24
    h, p = runner.hash[:count], runner.pos[:count]
    st = sws.SeedTableRunner(count, bits)
    ms, med, _ = time_launches(torch, lambda: st.launch(h, p, 64 - bits), steps, warmup)
    algo = 24 * count + 4 * ((1 << bits) + 1)
    return {"entries": count, "bits": bits, "ms": round(ms, 4), "median_ms": round(med, 4),
            "Mentries/s": round(count / (ms / 1e3) / 1e6, 1),
            "algorithmic_bytes": algo, "GB/s": round(algo / (ms / 1e3) / 1e9, 1),
            "hbm_frac": round(algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 3)}


def bench_batch(torch, quick):
    """Uneven reads in one launch (bucketed, tuned, graph) against one launch
    per read."""
    import ctypes
    import numpy as np
    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import _lib, batch, inputs, tune

    scale = 10 if quick else 1
    k, w = 15, 10
    log("generating the uneven-read batch")
    seqs, off = inputs.read_batch(n_short=2_000_000 // scale, n_long=100_000 // scale, seed=3)
    nreads, total = off.size - 1, int(off[-1])
    out = {"workload": "%d reads of 150 b + %d lognormal long reads (median 8 kb, sigma 0.8, "
                       "1-100 kb), 1%% N, k=15, w=10" % (2_000_000 // scale, 100_000 // scale),
           "reads": int(nreads), "bases": total}
    # one launch over all reads, default block size
    runner = batch.BatchRunner(torch.from_numpy(seqs).cuda(), off, k, w)
    ms, med, _ = time_launches(torch, runner.launch, 5, 2)
    out["one_launch"] = {"ms": round(ms, 3), "Gbases/s": round(total / (ms / 1e3) / 1e9, 2),
                         "minimizers": int(runner.read_out[-1].item())}
    del runner
    torch.cuda.empty_cache()
    # tuned block size per length bucket: eager per-bucket launches, then the
    # same launches captured in one HIP graph
    sub = slice(0, max(off.size // 20, 2))
    soff = off[sub] - off[0]
    table, report = tune.tune(seqs[: int(soff[-1])], soff, k, w, reps=3)
    bb = batch.BucketedBatch(seqs, off, k, w, tune_table=table)
    ms_e, _, _ = time_launches(torch, bb.launch, 5, 2)
    bb.capture()
    ms_g, med_g, _ = time_launches(torch, bb.replay, 5, 2)
    out["bucketed_eager"] = {"ms": round(ms_e, 3), "Gbases/s": round(total / (ms_e / 1e3) / 1e9, 2)}
    out["bucketed_graph"] = {"ms": round(ms_g, 3), "Gbases/s": round(total / (ms_g / 1e3) / 1e9, 2),
                             "graph_gain_vs_eager": round(ms_e / ms_g, 3),
                             "tune_table": {str(b): t for b, t in table.items()},
                             "tune_ms": {"%d/%d" % (b, t): round(v, 3)
                                         for b, r in report.items() for t, v in r["ms"].items()},
                             "tune_flat": {str(b): r["flat"] for b, r in report.items()}}
    del bb
    torch.cuda.empty_cache()
    # baseline: one library call per read (no batching), on the first reads
    nsample = 2000 if quick else 20000
    dev = torch.from_numpy(seqs[: int(off[nsample])]).cuda()
    maxlen = int(np.diff(off[: nsample + 1].astype(np.int64)).max())
    r = sws.MinimizerRunner(maxlen, k, w)
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base_ptr = dev.data_ptr()
    args = [(ctypes.c_void_p(base_ptr + int(off[i])), int(off[i + 1] - off[i])) for i in range(nsample)]
    hp, pp, cp, wp = (ctypes.c_void_p(t.data_ptr()) for t in (r.hash, r.pos, r.count, r.workspace))
    wsz = r.workspace.numel()

    def per_read():
        for ptr, n in args:
            lib.sws_minimizers(ptr, n, k, w, 0, hp, pp, r.capacity, cp, wp, wsz, stream)

    ms_p, _, _ = time_launches(torch, per_read, 1, 1)
    sbases = int(off[nsample])
    per_read_rate = sbases / (ms_p / 1e3) / 1e9
    out["per_read_launch"] = {"sample_reads": nsample, "sample_bases": sbases, "ms": round(ms_p, 3),
                              "us_per_read": round(ms_p * 1e3 / nsample, 2),
                              "Gbases/s": round(per_read_rate, 4)}
    best = max(out["one_launch"]["Gbases/s"], out["bucketed_graph"]["Gbases/s"])
    out["speedup_vs_per_read"] = round(best / per_read_rate, 1)
    return out


def bench_serve(torch, quick):
    """Poisson requests (k=19, w=19) through the continuous-batching server,
    open loop at the arrival times and closed loop, against one unbatched
    launch per request."""
    import numpy as np
    from paper_1811_10074_amd import inputs
    from paper_1811_10074_amd.serve import GPUExecutor, Server, latency_stats

    k, w = 19, 19
    dur = 3.0 if quick else 60.0
    log("generating %.0f s of Poisson requests" % dur)
    reqs = inputs.poisson_requests(rate=200.0, duration_s=dur, seed=4)
    bases = sum(int(o[-1]) for _, _, o in reqs)
    out = {"workload": "Poisson arrivals at 200 req/s for %.0f s, 1-4096 reads per request "
                       "(log-uniform), read lengths from the uneven-read mix, 1%% N, k=19, w=19"
                       % dur, "requests": len(reqs), "bases": bases}

    big = sorted(range(len(reqs)), key=lambda i: -int(reqs[i][2][-1]))[:4]

    def run(max_batch, streams, open_loop):
        ex = GPUExecutor(k, w, arena_bytes=16 << 30, streams=streams)  # None: the default
        srv = Server(ex, k, w, max_batch_bases=max_batch).start()
        # warm up kernels, buffers and the host allocator: the first request and
        # the four largest (the first multi-megabase copies of a process run
        # about twice as long as later ones)
        for i in [0] + big:
            srv.submit(reqs[i][1], reqs[i][2]).result(timeout=60)
        if not open_loop:
            # the closed loop's first pass over fresh host memory (result
            # arrays of gigabytes) runs about 5% slower than later ones:
            # one untimed pass over the first 2000 requests first
            for f in [srv.submit(sq, of) for _, sq, of in reqs[:2000]]:
                f.result(timeout=600)
        srv.completed.clear()
        # the client consumes each result as it arrives (counts it and lets it
        # go) instead of holding every result of the run
        left = [len(reqs)]
        errors = []
        finished = threading.Event()
        count_lock = threading.Lock()

        def consumed(f):
            if f.exception() is not None:
                errors.append(f.exception())
            with count_lock:
                left[0] -= 1
                if left[0] == 0:
                    finished.set()

        t0 = time.perf_counter()
        for t, sq, of in reqs:
            if open_loop:
                d = t0 + t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
            srv.submit(sq, of).add_done_callback(consumed)
        if not finished.wait(600):
            raise RuntimeError("serving run did not finish within 600 s")
        if errors:
            raise errors[0]
        wall = time.perf_counter() - t0
        srv.stop()
        st = latency_stats(srv.completed)
        st["Gbases/s"] = round(bases / wall / 1e9, 3)
        st["wall_s"] = round(wall, 3)
        del ex, srv
        torch.cuda.empty_cache()
        return {kk: (round(v, 3) if isinstance(v, float) else v) for kk, v in st.items()}

    out["closed_loop_warmup"] = "2000 requests, untimed, on the same server"
    out["batched_open_loop"] = run(64 << 20, None, True)
    out["batched_closed_loop"] = run(64 << 20, None, False)
    out["unbatched_closed_loop"] = run(1, 1, False)
    out["unbatched_open_loop"] = run(1, 1, True)
    return out


# the sliding-sum workloads --profile runs: (op, w, n, path)
SLIDING_PROFILES = {
    "sliding": ("add", 16, 1 << 28, "generic"),
    "affine1024": ("affine", 1024, 1 << 28, "auto"),
    "config1": ("min", 16, 1 << 20, "auto"),
    "add1024": ("add", 1024, 1 << 28, "auto"),
    "minlog64": ("min", 64, 1 << 28, "log"),
    "scalar16": ("add", 16, 1 << 28, "scalar"),
}


def profile_run(torch, args):
    """A plain device copy of exactly 1 GiB (its FETCH_SIZE / WRITE_SIZE
    calibrate the counters), then the kernel under study."""
    import numpy as np
    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import inputs

    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    if args.profile == "minimizer":
        n = 1 << 26
        seq = torch.from_numpy(inputs.dna(n, seed=1)).cuda()
        r = sws.MinimizerRunner(n, 15, 10)
        ms, med, _ = time_launches(torch, lambda: r.launch(seq=seq), args.steps, args.warmup)
        print(json.dumps({"kernel": "minimizer", "ms_per_step": ms, "count": int(r.count.item())}))
    elif args.profile in SLIDING_PROFILES:
        op, w, n, path = SLIDING_PROFILES[args.profile]
        x = inputs.affine_pairs(n, seed=2) if op == "affine" else \
            inputs.uniform_u32(n, seed=0 if n == 1 << 20 else 2)
        x = torch.from_numpy(x.view(np.int32)).cuda()
        y = torch.empty((n - w + 1, 2) if op == "affine" else (n - w + 1,), dtype=torch.int32,
                        device="cuda")
        ms, med, _ = time_launches(torch, lambda: sws.sliding_sum(op, w, x, path=path, out=y),
                                   args.steps, args.warmup)
        print(json.dumps({"kernel": "sliding %s w=%d n=%d path=%s" % (op, w, n, path),
                          "ms_per_step": ms}))
    elif args.profile == "seedtable":
        n = 1 << 26
        seq = torch.from_numpy(inputs.dna(n, seed=1)).cuda()
        r = sws.MinimizerRunner(n, 15, 10)
        r.launch(seq=seq)
        h, p = r.result()
        st = sws.SeedTableRunner(h.numel(), 24)
        ms, med, _ = time_launches(torch, lambda: st.launch(h, p, 40), args.steps, args.warmup)
        print(json.dumps({"kernel": "seed table 24 bits", "entries": h.numel(), "ms_per_step": ms}))
    elif args.profile == "batch":
        from paper_1811_10074_amd import batch
        seqs, off = inputs.read_batch(n_short=2_000_000, n_long=100_000, seed=3)
        runner = batch.BatchRunner(torch.from_numpy(seqs).cuda(), off, 15, 10)
        ms, med, _ = time_launches(torch, runner.launch, args.steps, args.warmup)
        print(json.dumps({"kernel": "batched minimizers, config 4, one launch", "ms_per_step": ms,
                          "bases": int(off[-1])}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="smaller extras")
    ap.add_argument("--primary-only", action="store_true",
                    help="only the timed minimizer steps (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", choices=["minimizer", "seedtable", "batch"] + list(SLIDING_PROFILES),
                    help="run only a 1-GiB plain copy (counter calibration) and the named kernel "
                         "--steps times, for rocprofv3")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile:
        return profile_run(torch, args)
    k, w, n = 15, 10, 1 << 26
    log("generating %d bases (seed 1)" % n)
    seq_np = inputs.dna(n, seed=1)
    seq = torch.from_numpy(seq_np).cuda()
    runner = sws.MinimizerRunner(n, k, w)
    step = lambda: runner.launch(seq=seq)
    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    ms, med, each = time_launches(torch, step, args.steps, args.warmup)
    count = int(runner.count.item())
    value = n / (ms / 1e3) / 1e9

    # the 2-bit input layout of the same sequence
    packed, _ = sws.pack2bit(seq, with_invalid=False)
    ms2 = time_back_to_back(torch, lambda: runner.launch(packed=packed, invalid=None, n=n),
                            args.steps, args.warmup)
    count2 = int(runner.count.item())

    if args.primary_only:
        print(json.dumps({"metric": METRIC, "value": value, "ms_per_step": ms, "count": count}))
        return

    # the same step with the 256 MB Infinity Cache flushed first: a 512 MiB
    # fill before every call, the call alone between the events
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    cold = []
    for i in range(args.warmup + args.steps):
        flush.fill_(i & 0xFF)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        if i >= args.warmup:
            cold.append((a, b))
    torch.cuda.synchronize()
    ms_cold = sum(a.elapsed_time(b) for a, b in cold) / len(cold)
    del flush

    algo_bytes = n + 12 * count  # ASCII in, (u64 hash, u32 pos) out
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "minimizer table: 64 Mbases i.i.d. uniform ACGT (seed 1) resident "
                               "as ASCII, canonical 15-mers, mix64, sliding min over w=10, dedup",
                   "n_bases": n, "k": k, "w": w, "parallelism": "single GPU"},
        "roofline": {
            "bound": "alu",
            "achieved": round(ALU_OPS_PER_BASE * n / (ms / 1e3) / 1e12, 2),
            "peak": round(ALU_PEAK_TOPS, 2),
            "unit": "Tops/s",
            "frac": round(ALU_OPS_PER_BASE * n / (ms / 1e3) / 1e12 / ALU_PEAK_TOPS, 3),
            "traffic": profiled_traffic("minimizer_wave_kernel_64Mbases_k15_w10.txt"),
            "ops_per_base_modelled": ALU_OPS_PER_BASE,
        },
        "hbm": {"algorithmic_bytes": algo_bytes,
                "GB/s": round(algo_bytes / (ms / 1e3) / 1e9, 1),
                "frac_of_peak": round(algo_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "note": "back-to-back steps: the 64 MB input and 146 MB output stay in the "
                        "256 MB Infinity Cache; dram_cold is the same step after a flush"},
        "dram_cold": {"ms_per_step": round(ms_cold, 5),
                      "Gbases/s": round(n / (ms_cold / 1e3) / 1e9, 2),
                      "GB/s": round(algo_bytes / (ms_cold / 1e3) / 1e9, 1),
                      "frac_of_peak": round(algo_bytes / (ms_cold / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                      "flush": "512 MiB fill before each step, outside the timed interval"},
        "minimizers_per_step": count,
        "median_ms": round(med, 5),
        "input_2bit": {"Gbases/s": round(n / (ms2 / 1e3) / 1e9, 2), "ms_per_step": round(ms2, 5),
                       "same_count": count2 == count},
    }
    # the committed rocprofv3 summaries of the same kernel (when its source
    # is unchanged since): its average duration, and the lane operations its
    # VALU instructions issue per base against the modelled count
    kus = profiled_kernel_us("minimizer_wave_kernel_64Mbases_k15_w10.txt", "minimizer_wave_kernel")
    if kus:
        line["roofline"]["profiled_kernel_us"] = round(kus, 2)
        line["roofline"]["frac_at_profiled_kernel_time"] = round(
            ALU_OPS_PER_BASE * n / (kus / 1e6) / 1e12 / ALU_PEAK_TOPS, 3)
    sq = profile_summary("minimizer_wave_kernel_64Mbases_k15_w10_sq_counters.txt")
    if sq and "valu_lane_ops_per_base" in sq["fields"]:
        # counted by SQ_INSTS_VALU: VALU lane operations per base, and issue
        # slots per base with the quarter-rate multiplies at four each
        line["roofline"]["ops_per_base_issued"] = float(sq["fields"]["valu_lane_ops_per_base"])
        if "issue_slot_lane_ops_per_base" in sq["fields"]:
            line["roofline"]["issue_slots_per_base"] = float(
                sq["fields"]["issue_slot_lane_ops_per_base"])
    # the standalone steps a3 and a4 on the same sequence
    msp = time_back_to_back(torch, lambda: sws.pack2bit(seq), args.steps, args.warmup)
    msk = time_back_to_back(torch, lambda: sws.kmers(seq, k), args.steps, args.warmup)
    pack_bytes = n + n // 4 + n // 8  # ASCII in; codes and invalid bits out
    kmer_bytes = n + 8 * (n - k + 1)  # ASCII in; one u64 per k-mer out
    line["pack2bit"] = {"us": round(msp * 1e3, 1), "GB/s": round(pack_bytes / msp / 1e6, 1),
                        "hbm_frac": round(pack_bytes / msp / 1e6 / HBM_PEAK_GBS, 3)}
    line["kmers_k15"] = {"us": round(msk * 1e3, 1), "GB/s": round(kmer_bytes / msk / 1e6, 1),
                         "hbm_frac": round(kmer_bytes / msk / 1e6 / HBM_PEAK_GBS, 3)}
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        line["cpu_baseline"] = cpu_baseline(seq_np, k, w)
        # parity of the timed output on the same prefix
        import oracle
        eh, ep = oracle.minimizers(seq_np[: 1 << 20], k, w)
        runner.launch(seq=seq)
        torch.cuda.synchronize()
        line["parity_prefix_2^20"] = bool(
            np.array_equal(runner.pos[: len(ep)].cpu().numpy().view(np.uint32), ep)
            and np.array_equal(runner.hash[: len(ep)].cpu().numpy().view(np.uint64), eh))
    log("seed table over the timed minimizers")
    line["seed_table"] = bench_seed_table(torch, runner, count, args.steps, args.warmup)
    del runner, seq, packed
    torch.cuda.empty_cache()
    log("sliding-sum extras")
    line["sliding"] = bench_sliding(torch, args.steps, args.warmup, args.quick)
    torch.cuda.empty_cache()
    log("batched reads")
    line["batched"] = bench_batch(torch, args.quick)
    torch.cuda.empty_cache()
    log("serving")
    line["serving"] = bench_serve(torch, args.quick)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
