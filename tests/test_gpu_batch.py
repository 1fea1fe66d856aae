"""Batched minimizers (many uneven reads, one launch) against the oracle run
read by read.  Bit-exact, including per-read output offsets."""
import numpy as np
import pytest

import oracle
from gpu_util import host_u32, host_u64, torch_cuda
from paper_1811_10074_amd import inputs

pytestmark = pytest.mark.gpu


def make_batch(lens, seed, n_rate=0.02, lower=0.02):
    lens = np.asarray(lens, dtype=np.int64)
    off = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    seqs = inputs.dna(int(off[-1]), seed=seed, n_rate=n_rate, lowercase_rate=lower)
    return seqs, off


def check_batch(torch, seqs, off, k, w, canonical=True, hashed=True, tag=""):
    from paper_1811_10074_amd import batch
    h, p, r, ro = batch.minimizers_batch(torch.from_numpy(seqs).cuda(), off, k, w, canonical, hashed)
    torch.cuda.synchronize()
    eh, ep, er, ero = oracle.minimizers_batch(seqs, off, k, w, canonical, hashed)
    assert np.array_equal(ro.cpu().numpy().view(np.uint64), ero), tag
    assert np.array_equal(host_u32(r), er), tag
    assert np.array_equal(host_u32(p), ep), tag
    assert np.array_equal(host_u64(h), eh), tag


@pytest.mark.parametrize("k,w", [(15, 10), (19, 19), (3, 3), (1, 1), (5, 2), (21, 28), (16, 32),
                                 (31, 18)])
def test_random_batches(k, w):
    torch = torch_cuda()
    rng = np.random.default_rng(k * 100 + w)
    for trial in range(3):
        lens = rng.integers(0, 400, 300)
        lens[rng.random(300) < 0.1] = 0
        seqs, off = make_batch(lens, seed=trial + 7 * k + w)
        check_batch(torch, seqs, off, k, w, tag="random %d" % trial)
    seqs, off = make_batch(rng.integers(0, 3000, 40), seed=99)
    for can in (True, False):
        for hsh in (True, False):
            check_batch(torch, seqs, off, k, w, can, hsh, tag="flags")


@pytest.mark.parametrize("w", list(range(1, 33)))
def test_every_window_up_to_32(w):
    """Every window length of the batched kernel, with k cycled so that short,
    long and FULL keys all meet the run pairings (k + w <= 49); reads with N
    and reads without."""
    torch = torch_cuda()
    ks = (15, 1, 31, 16, 17, 7, 22, 30, 11)
    k = min(ks[w % len(ks)], 49 - w)
    rng = np.random.default_rng(500 + w)
    lens = rng.integers(0, 600, 120)
    seqs, off = make_batch(lens, seed=w, n_rate=0.01)
    check_batch(torch, seqs, off, k, w, tag="every w, N")
    seqs, off = make_batch(rng.integers(200, 3000, 12), seed=w + 1, n_rate=0.0, lower=0.0)
    check_batch(torch, seqs, off, k, w, tag="every w, valid")


def test_edges():
    torch = torch_cuda()
    k, w = 15, 10
    cases = {
        "all empty": [0, 0, 0],
        "one empty": [0],
        "too short": [k + w - 2] * 50,
        "exact": [k + w - 1] * 50,
        "tiny many": list(np.random.default_rng(1).integers(0, 6, 5000)),
        "trailing empty": [500, 700, 0, 0],
        "leading empty": [0, 0, 800, 3],
        "one long": [200_000],
        "alternating": [1, 3000] * 40,
    }
    for name, lens in cases.items():
        seqs, off = make_batch(lens, seed=len(name))
        check_batch(torch, seqs, off, k, w, tag=name)
    # tiny reads with k = w = 1: every base is a window, up to a thousand reads per tile
    seqs, off = make_batch(np.random.default_rng(2).integers(0, 4, 20000), seed=3, n_rate=0.1)
    check_batch(torch, seqs, off, 1, 1, tag="k=w=1 tiny")


def test_matches_single_sequence():
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    seqs, off = make_batch([300_001], seed=11, n_rate=0.01)
    from paper_1811_10074_amd import batch
    h, p, r, ro = batch.minimizers_batch(torch.from_numpy(seqs).cuda(), off, 15, 10)
    hs, ps = sws.minimizers(torch.from_numpy(seqs).cuda(), 15, 10)
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(h), host_u64(hs)) and np.array_equal(host_u32(p), host_u32(ps))


def test_unsupported():
    torch = torch_cuda()
    from paper_1811_10074_amd import batch
    seqs, off = make_batch([100, 200], seed=1)
    with pytest.raises(ValueError):
        batch.minimizers_batch(torch.from_numpy(seqs).cuda(), off, 31, 19)
    with pytest.raises(ValueError):
        batch.minimizers_batch(torch.from_numpy(seqs).cuda(), off, 15, 33)


def test_config4_subsample_bucketed_graph():
    """A subsample of the uneven-read workload (150-b reads plus lognormal
    long reads, 1% N), split into length buckets with tuned block sizes and
    captured in one HIP graph: every replay equals the oracle, read by read."""
    torch = torch_cuda()
    from paper_1811_10074_amd import batch, tune
    seqs, off = inputs.read_batch(n_short=20_000, n_long=300, seed=3)
    table, report = tune.tune(seqs, off, 15, 10, reps=2)
    assert set(table) <= {0, 1, 2} and all(t in tune.CANDIDATES for t in table.values())
    assert set(report) == set(table)
    bb = batch.BucketedBatch(seqs, off, 15, 10, tune_table=table)
    bb.capture()
    eh, ep, er, ero = oracle.minimizers_batch(seqs, off, 15, 10)
    rng = np.random.default_rng(0)
    sample = rng.choice(off.size - 1, 300, replace=False)
    for rep in range(3):
        # eager work between replays
        junk = torch.arange(1 << 20, device="cuda").sum()
        bb.replay()
        torch.cuda.synchronize()
        res = bb.results()
        total = sum(int(v[3][-1].item()) for v in res.values())
        assert total == int(ero[-1]), rep
        for r in sample.tolist():
            h, p = bb.read_result(r, res)
            a, e = int(ero[r]), int(ero[r + 1])
            assert np.array_equal(p, ep[a:e]) and np.array_equal(h, eh[a:e]), (rep, r)
        del junk


def test_batch_split_at_invalid():
    """The batched kernel with SWS_SPLIT_AT_INVALID matches the oracle read by
    read (reads with N runs, uneven lengths)."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    rng = np.random.default_rng(42)
    lens = np.concatenate([rng.integers(1, 400, 300), rng.integers(1000, 20000, 12)])
    rng.shuffle(lens)
    off = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    seqs = inputs.dna(int(off[-1]), seed=43, n_rate=0.01)
    for k, w in ((15, 10), (19, 19), (7, 32)):
        h, p, r, ro = sws.minimizers_batch(seqs, off, k, w, split=True)
        torch.cuda.synchronize()
        eh, ep, er, ero = oracle.minimizers_batch(seqs, off, k, w, split=True)
        assert np.array_equal(ro.cpu().numpy().view(np.uint64), ero), (k, w)
        assert np.array_equal(p.cpu().numpy().view(np.uint32), ep), (k, w)
        assert np.array_equal(h.cpu().numpy().view(np.uint64), eh), (k, w)
        assert np.array_equal(r.cpu().numpy().view(np.uint32), er), (k, w)


def test_truncated_capacity():
    """A capacity below the total: the first `capacity` entries are the
    oracle's, nothing is written at or past it, and the offsets still hold
    the full totals."""
    torch = torch_cuda()
    from paper_1811_10074_amd import batch
    k, w = 15, 10
    seqs, off = make_batch(np.random.default_rng(5).integers(0, 5000, 60), seed=41)
    eh, ep, er, ero = oracle.minimizers_batch(seqs, off, k, w)
    r = batch.BatchRunner(torch.from_numpy(seqs).cuda(), off, k, w)
    assert r.capacity > eh.size > 1000
    for cap in (eh.size // 3, 1):
        r.capacity = cap
        r.hash.fill_(-5)
        r.pos.fill_(-5)
        r.read.fill_(-5)
        r.launch()
        torch.cuda.synchronize()
        assert np.array_equal(r.read_out.cpu().numpy().view(np.uint64), ero), cap
        assert np.array_equal(host_u64(r.hash[:cap]), eh[:cap]), cap
        assert np.array_equal(host_u32(r.pos[:cap]), ep[:cap]), cap
        assert np.array_equal(host_u32(r.read[:cap]), er[:cap]), cap
        assert bool((r.hash[cap:] == -5).all()) and bool((r.pos[cap:] == -5).all()), cap
        assert bool((r.read[cap:] == -5).all()), cap


@pytest.mark.parametrize("threads", [0, 64, 128, 256, 512])
def test_block_sizes(threads):
    """Every workgroup size the batched call accepts (the tuner's candidates)
    gives the oracle's output: short and long reads, empty reads, N bases."""
    torch = torch_cuda()
    from paper_1811_10074_amd import batch
    rng = np.random.default_rng(threads + 1)
    lens = np.concatenate([rng.integers(0, 400, 600), rng.integers(1000, 30000, 12), [0, 0, 5]])
    rng.shuffle(lens)
    seqs, off = make_batch(lens, seed=threads + 3)
    for k, w in ((15, 10), (21, 28), (31, 18)):
        r = batch.BatchRunner(torch.from_numpy(seqs).cuda(), off, k, w, threads=threads)
        r.launch()
        h, p, rd, ro = r.result()
        eh, ep, er, ero = oracle.minimizers_batch(seqs, off, k, w)
        assert np.array_equal(ro.cpu().numpy().view(np.uint64), ero), (threads, k, w)
        assert np.array_equal(host_u32(rd), er) and np.array_equal(host_u32(p), ep), (threads, k, w)
        assert np.array_equal(host_u64(h), eh), (threads, k, w)


def _bucket_expected(bb, b, ero, arrays):
    """The oracle's outputs of bucket b's reads, in the bucket's order."""
    sel = np.nonzero(bb.bucket_of == b)[0]
    starts = ero[sel].astype(np.int64)
    counts = (ero[sel + 1] - ero[sel]).astype(np.int64)
    before = np.cumsum(counts) - counts
    idx = np.arange(int(counts.sum()), dtype=np.int64) - np.repeat(before, counts) + \
        np.repeat(starts, counts)
    bro = np.zeros(sel.size + 1, dtype=np.uint64)
    np.cumsum(counts, out=bro[1:])
    return [a[idx] for a in arrays], bro, np.repeat(np.arange(sel.size, dtype=np.uint32), counts)


def test_config4_full_batch():
    """The whole uneven-read workload (2,000,000 reads of 150 b plus 100,000
    lognormal long reads, 1% N, 1.4 Gbases, k = 15, w = 10) in both launch
    configurations the benchmark times -- one launch over every read, and the
    tuned length buckets captured in one HIP graph -- every minimizer, read id
    and per-read offset compared with the oracle run read by read."""
    torch = torch_cuda()
    from paper_1811_10074_amd import batch, tune
    k, w = 15, 10
    seqs, off = inputs.read_batch(n_short=2_000_000, n_long=100_000, seed=3)
    print("config 4 full batch: oracle", flush=True)
    eh, ep, er, ero = oracle.minimizers_batch_parallel(seqs, off, k, w)
    print("config 4 full batch: one launch", flush=True)
    runner = batch.BatchRunner(torch.from_numpy(seqs).cuda(), off, k, w)
    runner.launch()
    h, p, rd, ro = runner.result()
    assert np.array_equal(ro.cpu().numpy().view(np.uint64), ero)
    assert np.array_equal(host_u32(rd), er)
    assert np.array_equal(host_u32(p), ep)
    assert np.array_equal(host_u64(h), eh)
    del runner, h, p, rd, ro
    torch.cuda.empty_cache()
    print("config 4 full batch: bucketed graph", flush=True)
    sub = slice(0, max(off.size // 20, 2))
    soff = off[sub] - off[0]
    table, _ = tune.tune(seqs[: int(soff[-1])], soff, k, w, reps=2)
    bb = batch.BucketedBatch(seqs, off, k, w, tune_table=table)
    bb.capture()
    for rep in range(2):
        bb.replay()
        torch.cuda.synchronize()
        res = bb.results()
        for b, (h, p, rd, ro) in res.items():
            (xh, xp), xro, xrd = _bucket_expected(bb, b, ero, (eh, ep))
            assert np.array_equal(ro.cpu().numpy().view(np.uint64), xro), (rep, b)
            assert np.array_equal(host_u32(rd), xrd), (rep, b)
            assert np.array_equal(host_u32(p), xp), (rep, b)
            assert np.array_equal(host_u64(h), xh), (rep, b)
    del bb
    torch.cuda.empty_cache()


def test_kept_workspace_across_batches():
    """SWS_WORKSPACE_KEPT on the batched call: one zero-filled workspace shared
    by batches of falling and rising size (the look-back status words of
    earlier calls stay in it, told apart by their epoch), with a call without
    the flag in between and both look-back windows' workgroup sizes; every
    call against the oracle, read by read."""
    torch = torch_cuda()
    import ctypes
    from paper_1811_10074_amd import _lib
    from paper_1811_10074_amd.batch import batch_workspace_bytes
    lib = _lib.load()
    k, w = 15, 10
    rng = np.random.default_rng(77)
    plan = [(400, 0), (40, _lib.WORKSPACE_KEPT), (3, _lib.WORKSPACE_KEPT), (400, _lib.WORKSPACE_KEPT),
            (150, 0), (250, _lib.WORKSPACE_KEPT), (400, _lib.WORKSPACE_KEPT)]
    batches = [make_batch(rng.integers(0, 2500, nr), seed=900 + i, n_rate=0.01)
               for i, (nr, _) in enumerate(plan)]
    ws_bytes = max(batch_workspace_bytes(int(o[-1]), o.size - 1, k, w) for _, o in batches)
    ws = torch.zeros(ws_bytes, dtype=torch.uint8, device="cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    for i, ((seqs, off), (_, kept)) in enumerate(zip(batches, plan)):
        eh, ep, er, ero = oracle.minimizers_batch(seqs, off, k, w)
        cap = max(1, int(ero[-1]))
        d_seq = torch.from_numpy(seqs).cuda()
        d_off = torch.from_numpy(off.view(np.int64)).cuda()
        h = torch.empty(cap, dtype=torch.int64, device="cuda")
        p = torch.empty(cap, dtype=torch.int32, device="cuda")
        r = torch.empty(cap, dtype=torch.int32, device="cuda")
        ro = torch.empty(off.size, dtype=torch.int64, device="cuda")
        threads = 256 if i % 2 == 0 else 128
        st = lib.sws_minimizers_batch_ex(ptr(d_seq), ptr(d_off), off.size - 1, int(off[-1]), k, w,
                                         kept, ptr(h), ptr(p), ptr(r), cap, ptr(ro), ptr(ws),
                                         ws_bytes, threads, torch.cuda.current_stream().cuda_stream)
        assert st == _lib.SWS_OK, (i, st)
        torch.cuda.synchronize()
        got_ro = ro.cpu().numpy().view(np.uint64)
        assert np.array_equal(got_ro, ero), i
        n = int(ero[-1])
        assert np.array_equal(host_u64(h[:n]), eh) and np.array_equal(host_u32(p[:n]), ep), i
        assert np.array_equal(host_u32(r[:n]), er), i
