"""The serving loop on the GPU: every request's minimizers equal the oracle's,
alone and in a Poisson mix, also when a small arena forces admission to wait."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import torch_cuda
from paper_1811_10074_amd import inputs

pytestmark = pytest.mark.gpu
K, W = 19, 19


def reqs_small(count, seed):
    return [(s, o) for _, s, o in inputs.poisson_requests(rate=1000.0, duration_s=10.0,
                                                          max_reads=64, seed=seed,
                                                          max_requests=count)]


def check(res, seqs, off):
    h, p, r, ro = oracle.minimizers_batch(seqs, off, K, W)
    assert np.array_equal(res.read_offsets, ro)
    assert np.array_equal(res.pos, p) and np.array_equal(res.hash, h)


def test_alone_equals_mix():
    torch_cuda()
    from paper_1811_10074_amd.serve import GPUExecutor, Server
    reqs = reqs_small(24, seed=4)
    ex = GPUExecutor(K, W, arena_bytes=1 << 30, streams=4)
    srv = Server(ex, K, W).start()
    alone = [srv.submit(s, o).result(timeout=60) for s, o in reqs]
    futs = [srv.submit(s, o) for s, o in reqs]
    mixed = [f.result(timeout=60) for f in futs]
    srv.stop()
    for (s, o), a, m in zip(reqs, alone, mixed):
        check(a, s, o)
        check(m, s, o)
    assert srv.arena.free_bytes == srv.arena.size


def test_admission_under_memory_pressure():
    torch_cuda()
    from paper_1811_10074_amd.serve import GPUExecutor, Server
    reqs = reqs_small(16, seed=5)
    biggest = max(int(o[-1]) for _, o in reqs)
    ex = GPUExecutor(K, W, arena_bytes=max(40 * biggest, 1 << 22), streams=3)
    srv = Server(ex, K, W).start()
    futs = [srv.submit(s, o) for s, o in reqs]
    for (s, o), f in zip(reqs, futs):
        check(f.result(timeout=120), s, o)
    srv.stop()
    assert srv.arena.free_bytes == srv.arena.size


def test_poisson_replay_short():
    torch_cuda()
    from paper_1811_10074_amd.serve import GPUExecutor, Server, latency_stats
    reqs = inputs.poisson_requests(rate=200.0, duration_s=1.0, max_reads=256, seed=6)
    ex = GPUExecutor(K, W, arena_bytes=2 << 30, streams=4)
    srv = Server(ex, K, W).start()
    t0 = time.perf_counter()
    futs = []
    for t, s, o in reqs:
        delay = t0 + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(srv.submit(s, o))
    for (t, s, o), f in zip(reqs, futs):
        check(f.result(timeout=120), s, o)
    srv.stop()
    st = latency_stats(srv.completed)
    assert st["n"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_denser_than_the_copy_back_estimate():
    """A poly-A read stores a minimizer at every window (every k-mer ties,
    the leftmost wins), far above the density the executor copies back with
    the kernel; the rest comes by a second copy.  A random read in the same
    batch and alone stays exact."""
    torch_cuda()
    from paper_1811_10074_amd.serve import GPUExecutor, Server
    dense = np.frombuffer(b"A" * 20000, dtype=np.uint8).copy()
    rnd = inputs.dna(30000, seed=9, n_rate=0.01)
    seqs = np.concatenate([dense, rnd])
    off = np.array([0, dense.size, seqs.size], dtype=np.uint64)
    ex = GPUExecutor(K, W, arena_bytes=1 << 28, streams=2)
    srv = Server(ex, K, W).start()
    got = srv.submit(seqs, off).result(timeout=60)
    alone = srv.submit(rnd, np.array([0, rnd.size], dtype=np.uint64)).result(timeout=60)
    srv.stop()
    check(got, seqs, off)
    check(alone, rnd, np.array([0, rnd.size], dtype=np.uint64))
    assert got.read_offsets[1] == 20000 - K - W + 2  # every window of the poly-A read


def test_config5_sized_requests_alone_and_mixed():
    """Requests of the serving workload's full size range (1 to 4096 reads of
    the uneven-read mix, several Mbases at the top): the largest requests of
    ten seconds of Poisson arrivals plus a spread of others, each served alone
    and then all submitted at once; every result equals the oracle's."""
    torch_cuda()
    from paper_1811_10074_amd.serve import GPUExecutor, Server
    allreq = [(s, o) for _, s, o in inputs.poisson_requests(rate=200.0, duration_s=10.0,
                                                            max_reads=4096, seed=4)]
    by_size = sorted(range(len(allreq)), key=lambda i: int(allreq[i][1][-1]))
    pick = sorted(set(by_size[-6:]) | set(by_size[:: max(1, len(by_size) // 30)]))
    reqs = [allreq[i] for i in pick]
    assert max(int(o[-1]) for _, o in reqs) > 2_000_000
    assert max(o.size - 1 for _, o in reqs) > 1000
    ex = GPUExecutor(K, W, arena_bytes=4 << 30, streams=3)
    srv = Server(ex, K, W).start()
    alone = [srv.submit(s, o).result(timeout=120) for s, o in reqs]
    futs = [srv.submit(s, o) for s, o in reqs]
    mixed = [f.result(timeout=120) for f in futs]
    srv.stop()
    for (s, o), a, m in zip(reqs, alone, mixed):
        h, p, r, ro = oracle.minimizers_batch_parallel(s, o, K, W)
        for res in (a, m):
            assert np.array_equal(res.read_offsets, ro)
            assert np.array_equal(res.pos, p) and np.array_equal(res.hash, h)
    assert srv.arena.free_bytes == srv.arena.size
