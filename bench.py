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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_launches(torch, fn, steps, warmup):
    """Mean and median ms per call over `steps` timed calls on the current
    stream, bracketed by synchronizations."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    end.record()
    torch.cuda.synchronize()
    total = start.elapsed_time(end)
    each = sorted(a.elapsed_time(b) for a, b in evs)
    return total / steps, each[len(each) // 2], each


def cpu_baseline(seq_np, k, w, target_s=10.0):
    """The oracle's deque minimizer on a prefix of the same sequence, repeated
    until about target_s seconds of CPU work."""
    import numpy as np
    import oracle

    sample = seq_np[: 1 << 24]
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.minimizers(sample, k, w)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 8:
            break
    rate = reps * sample.size / el / 1e9
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = platform.processor()
    return {"value": rate, "unit": "Gbases/s", "cores": 1, "kind": "oracle",
            "sample": "deque minimizers (k=15, w=10) over the first 2^24 bases of the same "
                      "sequence, %d repetitions, %.1f s, single thread" % (reps, el),
            "cpu": model, "host_threads_available": len(os.sched_getaffinity(0))}


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
    n = 1 << 28
    x = torch.from_numpy(inputs.uniform_u32(n, seed=2).view(np.int32)).cuda()
    xa = None if quick else torch.from_numpy(inputs.affine_pairs(n, seed=2).view(np.int32)).cuda()
    sweep = {}
    for op in ("add", "min", "max", "affine"):
        if op == "affine" and xa is None:
            continue
        src = xa if op == "affine" else x
        esz = 8 if op == "affine" else 4
        for path in (("generic", "log") if op in ("min", "max") else ("generic",)):
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
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="smaller extras")
    ap.add_argument("--primary-only", action="store_true",
                    help="only the timed minimizer steps (for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the design for "
              "sharding is in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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
    ms2, med2, _ = time_launches(torch, lambda: runner.launch(packed=packed, invalid=None, n=n),
                                 args.steps, args.warmup)
    count2 = int(runner.count.item())

    if args.primary_only:
        print(json.dumps({"metric": METRIC, "value": value, "ms_per_step": ms, "count": count}))
        return

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
            "traffic": None,
        },
        "hbm": {"algorithmic_bytes": algo_bytes,
                "GB/s": round(algo_bytes / (ms / 1e3) / 1e9, 1),
                "frac_of_peak": round(algo_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "minimizers_per_step": count,
        "median_ms": round(med, 5),
        "input_2bit": {"Gbases/s": round(n / (ms2 / 1e3) / 1e9, 2), "ms_per_step": round(ms2, 5),
                       "same_count": count2 == count},
    }
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
    del runner, seq, packed
    torch.cuda.empty_cache()
    log("sliding-sum extras")
    line["sliding"] = bench_sliding(torch, args.steps, args.warmup, args.quick)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
