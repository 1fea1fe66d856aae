"""The serving scheduler on the CPU with the oracle-backed fake executor:
admission by arena bytes, oldest-first order, overlap of in-flight batches,
per-request failure isolation, oversize rejection, and identical results
alone and in a mix."""
import gc
import time
import weakref

import numpy as np
import pytest

import oracle
from paper_1811_10074_amd import inputs
from paper_1811_10074_amd.serve import (Arena, FakeExecutor, RequestTooLarge, Server,
                                        latency_stats, window_bound)

K, W = 15, 10


def oracle_compute(seqs, off, k, w):
    return oracle.minimizers_batch(seqs, off, k, w)


def make_request(seed, nreads=None, short=150, uniform=False):
    rng = np.random.default_rng(seed)
    n = nreads or int(rng.integers(1, 20))
    lens = np.full(n, short) if uniform else np.where(rng.random(n) < 0.8, short,
                                                     rng.integers(200, 3000, n))
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    seqs = inputs.dna(int(off[-1]), seed=seed, n_rate=0.01)
    return seqs, off


def expected(seqs, off):
    h, p, r, ro = oracle.minimizers_batch(seqs, off, K, W)
    return h, p, ro


def same(res, exp):
    h, p, ro = exp
    return np.array_equal(res.hash, h) and np.array_equal(res.pos, p) and np.array_equal(res.read_offsets, ro)


def test_arena_first_fit_and_coalescing():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    a.release(x, 1000)
    assert a.free_list[0] == (0, 2048)
    assert a.alloc(2000) == 0
    a.release(0, 2000)
    a.release(z, 1000)
    assert a.free_list == [(0, 4096)] and a.free_bytes == 4096


def test_results_alone_equal_mix():
    reqs = [make_request(s) for s in range(40)]
    exp = [expected(*r) for r in reqs]
    # alone: one request at a time
    srv = Server(FakeExecutor(K, W, compute=oracle_compute), K, W).start()
    alone = [srv.submit(*r).result(timeout=30) for r in reqs]
    srv.stop()
    # mixed: all at once, batched together, several in flight
    ex = FakeExecutor(K, W, slots=3, compute=oracle_compute, latency=lambda rs: 0.005)
    srv = Server(ex, K, W, max_batch_bases=20_000, concurrent_bases=0).start()
    futs = [srv.submit(*r) for r in reqs]
    mixed = [f.result(timeout=30) for f in futs]
    srv.stop()
    for a, m, e in zip(alone, mixed, exp):
        assert same(a, e) and same(m, e)
    assert any(len(b) > 1 for b in ex.batches), "requests were never batched together"
    assert ex.max_inflight_seen >= 2, "batches never overlapped"


def test_admission_waits_for_memory():
    reqs = [make_request(100 + s, nreads=10, uniform=True) for s in range(12)]
    one = FakeExecutor(K, W).footprint(int(reqs[0][1][-1]), 10, window_bound(reqs[0][1], K, W))
    # room for about two requests at a time
    ex = FakeExecutor(K, W, arena_bytes=int(2.5 * one), slots=4, compute=oracle_compute,
                      latency=lambda rs: 0.01)
    srv = Server(ex, K, W).start()
    futs = [srv.submit(*r) for r in reqs]
    res = [f.result(timeout=30) for f in futs]
    srv.stop()
    assert all(same(r, expected(*q)) for r, q in zip(res, reqs))
    assert max(len(b) for b in ex.batches) <= 2
    assert srv.arena.free_bytes == srv.arena.size


def test_oldest_first():
    ex = FakeExecutor(K, W, slots=1, compute=oracle_compute, latency=lambda rs: 0.002)
    srv = Server(ex, K, W, max_batch_bases=1).start()  # one request per batch
    futs = [srv.submit(*make_request(200 + s)) for s in range(10)]
    [f.result(timeout=30) for f in futs]
    srv.stop()
    order = [b[0] for b in ex.batches]
    assert order == sorted(order)


def test_failure_isolated_per_request():
    reqs = [make_request(300 + s) for s in range(8)]
    bad = {3}
    ex = FakeExecutor(K, W, compute=oracle_compute, fail=lambda q: q.rid in bad,
                      latency=lambda rs: 0.002)
    srv = Server(ex, K, W).start()
    futs = [srv.submit(*r) for r in reqs]
    for i, f in enumerate(futs):
        if i in bad:
            with pytest.raises(RuntimeError):
                f.result(timeout=30)
        else:
            assert same(f.result(timeout=30), expected(*reqs[i]))
    srv.stop()


def test_oversize_rejected():
    ex = FakeExecutor(K, W, arena_bytes=10_000, compute=oracle_compute)
    srv = Server(ex, K, W).start()
    f = srv.submit(*make_request(400, nreads=30))
    with pytest.raises(RequestTooLarge):
        f.result(timeout=5)
    srv.stop()


def test_latency_stats():
    ex = FakeExecutor(K, W, compute=oracle_compute, latency=lambda rs: 0.003)
    srv = Server(ex, K, W).start()
    futs = [srv.submit(*make_request(500 + s)) for s in range(10)]
    [f.result(timeout=30) for f in futs]
    srv.stop()
    st = latency_stats(srv.completed)
    assert st["n"] == 10 and st["p99_ms"] >= st["p50_ms"] >= 3.0


def test_concurrency_follows_the_queue():
    """A second batch runs beside the first only when enough bases wait: with
    a threshold above the whole workload, batches never overlap; with one
    below it they do."""
    reqs = [make_request(600 + s) for s in range(30)]
    total = sum(int(o[-1]) for _, o in reqs)
    for thr, overlap in ((10 * total, False), (1, True)):
        ex = FakeExecutor(K, W, slots=3, compute=oracle_compute, latency=lambda rs: 0.004)
        srv = Server(ex, K, W, max_batch_bases=5_000, concurrent_bases=thr).start()
        futs = [srv.submit(*r) for r in reqs]
        res = [f.result(timeout=30) for f in futs]
        srv.stop()
        assert all(same(r, expected(*q)) for r, q in zip(res, reqs))
        assert (ex.max_inflight_seen >= 2) == overlap, (thr, ex.max_inflight_seen)


def test_results_not_retained():
    """Once the client lets a result go, nothing in the server keeps it (or
    the request's bases) alive: a long-running server does not accumulate
    what it has handed out, and freed result memory is reused."""
    srv = Server(FakeExecutor(K, W, compute=oracle_compute), K, W).start()
    seqs, off = make_request(700)
    f = srv.submit(seqs, off)
    res = f.result(timeout=30)
    ok = same(res, expected(seqs, off))  # (an assert's rewritten temporaries would hold res)
    assert ok
    ref_res, ref_seqs = weakref.ref(res), weakref.ref(seqs)
    del f, res, seqs
    time.sleep(0.05)  # the completer finishes its round
    gc.collect()
    assert ref_res() is None, "the server still holds a result the client dropped"
    assert ref_seqs() is None, "the server still holds a completed request's bases"
    # its timings stay for the latency statistics
    assert latency_stats(srv.completed)["n"] == 1
    srv.stop()
