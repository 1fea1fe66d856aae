"""Parity of the HIP packing, k-mer and minimizer kernels with the CPU oracle
(Sec. 2.4, Fig. 2).  Everything is integer work: bit-exact."""
import numpy as np
import pytest

import oracle
import oracle_pins
from gpu_util import dev, host_u32, host_u64, torch_cuda
from paper_1811_10074_amd import inputs

pytestmark = pytest.mark.gpu

TILE = 256 * 16  # key positions per minimizer tile (256 threads)


def seq_dev(torch, s):
    if isinstance(s, str):
        s = np.frombuffer(s.encode(), dtype=np.uint8)
    return dev(np.ascontiguousarray(s, dtype=np.uint8), torch)


def gpu_minimizers(torch, s, k, w, canonical=True, hashed=True):
    import paper_1811_10074_amd as sws
    h, p = sws.minimizers(seq_dev(torch, s), k, w, canonical=canonical, hashed=hashed)
    torch.cuda.synchronize()
    return host_u64(h), host_u32(p)


def assert_same_minimizers(torch, s, k, w, canonical=True, hashed=True, tag=""):
    gh, gp = gpu_minimizers(torch, s, k, w, canonical, hashed)
    eh, ep = oracle.minimizers(s, k, w, canonical, hashed)
    if not (np.array_equal(gp, ep) and np.array_equal(gh, eh)):
        m = min(len(gp), len(ep))
        d = np.nonzero((gp[:m] != ep[:m]) | (gh[:m] != eh[:m]))[0]
        first = int(d[0]) if d.size else m
        raise AssertionError("%s k=%d w=%d can=%s hash=%s n=%d: gpu %d vs oracle %d, first diff at %d"
                             % (tag, k, w, canonical, hashed, len(s), len(gp), len(ep), first))


def test_pack2bit_layout():
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for n in (1, 15, 16, 17, 31, 32, 33, 1000, 65_537):
        s = inputs.dna(n, seed=n, n_rate=0.05, lowercase_rate=0.1)
        packed, invalid = sws.pack2bit(seq_dev(torch, s))
        torch.cuda.synchronize()
        pk, iv = host_u32(packed), host_u32(invalid)
        lib = oracle.load()
        codes = np.array([lib.oracle_base_code(int(b)) for b in s], dtype=np.int64)
        i = np.arange(n)
        got_code = (pk[i // 16] >> (30 - 2 * (i % 16)).astype(np.uint32)) & 3
        got_inv = (iv[i // 32] >> (i % 32).astype(np.uint32)) & 1
        assert np.array_equal(got_inv, (codes < 0).astype(np.uint32)), n
        assert np.array_equal(got_code, np.where(codes < 0, 0, codes).astype(np.uint32)), n
        # bits past n are zero
        tail = np.arange(n, len(pk) * 16)
        assert np.all(((pk[tail // 16] >> (30 - 2 * (tail % 16)).astype(np.uint32)) & 3) == 0)
        tail = np.arange(n, len(iv) * 32)
        assert np.all(((iv[tail // 32] >> (tail % 32).astype(np.uint32)) & 1) == 0)


@pytest.mark.parametrize("k", [1, 2, 3, 7, 15, 16, 17, 19, 21, 29, 30, 31])
def test_kmers(k):
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for n in (k, k + 1, 100, TILE + 17, 3 * TILE + 5):
        s = inputs.dna(n, seed=1000 + n + k, n_rate=0.02, lowercase_rate=0.05)
        for can in (True, False):
            for hsh in (True, False):
                if hsh and k >= 30:
                    continue
                got = host_u64(sws.kmers(seq_dev(torch, s), k, canonical=can, hashed=hsh))
                torch.cuda.synchronize()
                exp = oracle.kmers(s, k, canonical=can, hashed=hsh)
                assert np.array_equal(got, exp), (k, n, can, hsh)
    with pytest.raises(ValueError):
        sws.kmers(seq_dev(torch, "ACGT" * 20), 30, hashed=True)


@pytest.mark.parametrize("k", [15, 21])
def test_kmers_output_not_16_byte_aligned(k):
    """An output 8 bytes past a 16-byte boundary takes the one-value-per-store
    kernel; values are the same."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import _lib
    n = 3 * TILE + 5
    s = inputs.dna(n, seed=77 + k, n_rate=0.02)
    buf = torch.full((n - k + 3,), 7, dtype=torch.int64, device="cuda")
    out = buf[1:n - k + 2]
    assert out.data_ptr() % 16 == 8
    seq = seq_dev(torch, s)
    sws.check(_lib.load().sws_kmers(seq.data_ptr(), n, k, 0, out.data_ptr(), sws._stream()), "sws_kmers")
    torch.cuda.synchronize()
    got = host_u64(buf)
    assert np.array_equal(got[1:n - k + 2], oracle.kmers(s, k, canonical=True, hashed=True)), k
    assert got[0] == 7 and got[-1] == 7  # nothing written outside the output


def test_fig2_worked_example():
    torch = torch_cuda()
    g = oracle_pins.read_golden("fig2_worked_example.txt")
    k, w, s = int(g["k"][0]), int(g["w"][0]), g["sequence"][0]
    gh, gp = gpu_minimizers(torch, s, k, w, canonical=False, hashed=False)
    assert gp.tolist() == [int(v) for v in g["stored_positions"]]
    val = int("".join(str("ACGT".index(c)) for c in g["shared_minimizer"][0]), 4)
    assert (val, int(g["shared_minimizer"][1])) in list(zip(gh.tolist(), gp.tolist()))


@pytest.mark.parametrize("k,w", [(15, 10), (19, 19), (3, 3), (1, 1), (5, 1), (2, 7), (16, 16),
                                 (17, 5), (21, 11), (31, 10), (30, 3), (11, 64), (15, 100),
                                 (7, 255), (13, 1000), (15, 1024)])
def test_minimizers_random(k, w):
    torch = torch_cuda()
    for n in (k + w - 2, k + w - 1, k + w, 200, TILE - 7, 2 * TILE + 333, 5 * TILE + 1):
        for n_rate in (0.0, 0.03):
            s = inputs.dna(n, seed=7 * n + k + w, n_rate=n_rate, lowercase_rate=0.02)
            assert_same_minimizers(torch, s, k, w, tag="random")
    s = inputs.dna(3 * TILE + 77, seed=k * w, n_rate=0.01)
    for can in (True, False):
        for hsh in (True, False):
            assert_same_minimizers(torch, s, k, w, can, hsh, tag="flags")


# k values cycled over w so that every window length meets short, long (> 16)
# and FULL (hashed k >= 30) keys
_EVERY_K = (15, 1, 31, 16, 17, 7, 22, 30, 11)


@pytest.mark.parametrize("w", list(range(1, 33)))
def test_every_window_up_to_32(w):
    """Every window length of the wave-tile kernel (each has its own pairing
    of run prefixes and suffixes, or doubling steps): sequences over several
    wave tiles with a ragged end, all valid (waves skip the invalid bits), with
    scattered N, and with one N run between valid stretches (valid and invalid
    waves in one launch); ASCII and 2-bit input."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    k = _EVERY_K[w % len(_EVERY_K)]
    n = 5 * 1024 + 517
    for variant in range(3):
        s = inputs.dna(n, seed=1000 + 3 * w + variant, n_rate=0.01 if variant == 1 else 0.0)
        if variant == 2:
            s[2100:2100 + 37] = ord("N")
        assert_same_minimizers(torch, s, k, w, tag="every w, variant %d" % variant)
        sd = seq_dev(torch, s)
        packed, inv = sws.pack2bit(sd)
        h, p = sws.minimizers_2bit(packed, inv if variant else None, n, k, w)
        torch.cuda.synchronize()
        eh, ep = oracle.minimizers(s, k, w)
        assert np.array_equal(host_u32(p), ep) and np.array_equal(host_u64(h), eh), (k, w, variant)
    s = inputs.dna(3 * 1024 + 100, seed=w, n_rate=0.005)
    assert_same_minimizers(torch, s, k, w, canonical=False, hashed=False, tag="forward identity")


@pytest.mark.parametrize("w", [33, 64, 500, 992, 993, 1000, 1024])
def test_block_kernel_workspace_sizes(w):
    """Windows above 32 run on the 256-thread block kernel: the workspace the
    query returns holds every tile of the launch (regression: the query and the
    launch once assumed different tile widths), from one tile to many."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for n in (16_000, 20_481, 150_001):
        s = inputs.dna(n, seed=n + w, n_rate=0.01)
        need = sws.minimizer_workspace_bytes(n, 13, w)
        r = sws.MinimizerRunner(n, 13, w)
        assert r.workspace.numel() == max(need, 8)
        r.launch(seq=seq_dev(torch, s))
        h, p = r.result()
        eh, ep = oracle.minimizers(s, 13, w)
        assert np.array_equal(host_u32(p), ep) and np.array_equal(host_u64(h), eh), (n, w)


def test_minimizers_structured():
    """Repeats and ties (poly-A hashes to 0; tandem repeats tie the hash) and
    long N runs that empty whole windows and tiles."""
    torch = torch_cuda()
    parts = ["A" * 5000, "ACGT" * 1500, "N" * 9000, "AC" * 3000, "T" * 40, "N" * 3,
             "GATTACA" * 900]
    s = "".join(parts)
    for k, w in ((15, 10), (19, 19), (4, 50), (31, 10), (1, 3)):
        for can in (True, False):
            for hsh in (True, False):
                assert_same_minimizers(torch, s, k, w, can, hsh, tag="structured")
    assert_same_minimizers(torch, "N" * 20000, 15, 10, tag="all-N")


def test_minimizers_2bit_and_repeat():
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for n, n_rate in ((50_000, 0.0), (70_001, 0.01)):
        s = inputs.dna(n, seed=n, n_rate=n_rate)
        sd = seq_dev(torch, s)
        packed, invalid = sws.pack2bit(sd)
        for use_inv in (True, False):
            if not use_inv and n_rate > 0:
                continue
            h, p = sws.minimizers_2bit(packed, invalid if use_inv else None, n, 15, 10)
            torch.cuda.synchronize()
            eh, ep = oracle.minimizers(s, 15, 10)
            assert np.array_equal(host_u32(p), ep) and np.array_equal(host_u64(h), eh)
    # the same runner twice: identical, the second call clears its own workspace
    s = inputs.dna(100_000, seed=5, n_rate=0.01)
    r = sws.MinimizerRunner(200_000, 15, 10)
    outs = []
    for _ in range(2):
        r.launch(seq=seq_dev(torch, s))
        h, p = r.result()
        outs.append((host_u64(h).copy(), host_u32(p).copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_minimizers_edges():
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for s in ("", "ACGT", "ACGTACGTACGTACG", "N", "NNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNN"):
        t = seq_dev(torch, s) if s else torch.empty(0, dtype=torch.uint8, device="cuda")
        h, p = sws.minimizers(t, 15, 10)
        torch.cuda.synchronize()
        eh, ep = oracle.minimizers(s, 15, 10)
        assert np.array_equal(host_u32(p), ep) and np.array_equal(host_u64(h), eh), s


def test_config2_full():
    """64 Mbases i.i.d. uniform (seed 1), canonical 15-mers, mix64, w = 10:
    the whole output against the oracle, through both input layouts."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    n = 1 << 26
    s = inputs.dna(n, seed=1)
    eh, ep = oracle.minimizers(s, 15, 10)
    sd = seq_dev(torch, s)
    h, p = sws.minimizers(sd, 15, 10)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(p), ep)
    assert np.array_equal(host_u64(h), eh)
    packed, _ = sws.pack2bit(sd, with_invalid=False)
    h, p = sws.minimizers_2bit(packed, None, n, 15, 10)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(p), ep)
    assert np.array_equal(host_u64(h), eh)
    W = n - 15 - 10 + 2
    assert abs(len(ep) / (1 + (W - 1) * 2 / 11) - 1) < 0.005


def test_split_at_invalid():
    """Segment-split N semantics (SWS_SPLIT_AT_INVALID): every window holding
    an invalid k-mer stores nothing and dedup restarts after it; single
    sequences with N runs of every length, several k and w <= 32, ASCII and
    2-bit input."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    rng = np.random.default_rng(41)
    for n, rate in ((3000, 0.02), (50_000, 0.003), (200_001, 0.01)):
        s = inputs.dna(n, seed=int(rng.integers(1 << 30)), n_rate=rate)
        # runs of N as well as single ones
        for a in rng.integers(0, n - 40, 5):
            s[a:a + int(rng.integers(1, 40))] = ord("N")
        t = torch.from_numpy(s).cuda()
        for k, w in ((15, 10), (5, 1), (19, 19), (11, 32), (31, 2)):
            for canonical, hashed in ((True, True), (False, True), (True, False)):
                h, p = sws.minimizers(t, k, w, canonical=canonical, hashed=hashed, split=True)
                torch.cuda.synchronize()
                eh, ep = oracle.minimizers(s, k, w, canonical=canonical, hashed=hashed, split=True)
                assert np.array_equal(p.cpu().numpy().view(np.uint32), ep), (n, k, w)
                assert np.array_equal(h.cpu().numpy().view(np.uint64), eh), (n, k, w)
        packed, inv = sws.pack2bit(t)
        h, p = sws.minimizers_2bit(packed, inv, n, 15, 10, split=True)
        torch.cuda.synchronize()
        eh, ep = oracle.minimizers(s, 15, 10, split=True)
        assert np.array_equal(p.cpu().numpy().view(np.uint32), ep)
    with pytest.raises(Exception):
        sws.minimizers(t, 15, 33, split=True)  # w > 32 is unsupported with the flag


def _decode_2bit(words, s0, s1):
    """ASCII bases s0 .. s1 - 1 of a 2-bit word array (16 per word, first base
    in the top bits)."""
    idx = np.arange(s0, s1, dtype=np.int64)
    codes = (words[idx >> 4] >> (30 - 2 * (idx & 15)).astype(np.uint32)) & np.uint32(3)
    return np.frombuffer(b"ACGT", dtype=np.uint8)[codes]


def test_max_length_sampled():
    """The longest sequence the library takes (2^32 - 3 bases, i.i.d. uniform,
    as 2-bit words), in the bench's launch configuration.  Stretches around
    2^31 and at the end of the 32-bit position range are checked against the
    oracle run on the stretch alone: an entry is decided by the windows that
    contain it, so entries whose windows all lie inside the stretch must agree.
    Positions must increase over the whole output, and the count must match the
    density of random order (R16) within 0.2%."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    n = 0xFFFFFFFD
    k, w = 15, 10
    rng = np.random.default_rng(77)
    words = rng.integers(0, 1 << 32, (n + 15) // 16, dtype=np.uint32)
    packed = torch.from_numpy(words.view(np.int32)).cuda()
    r = sws.MinimizerRunner(n, k, w)
    r.launch(packed=packed, invalid=None, n=n)
    h, p = r.result()
    p64 = p.to(torch.int64) & 0xFFFFFFFF
    assert bool((p64[1:] > p64[:-1]).all())
    W = n - k - w + 2
    assert abs(p64.numel() / (1 + (W - 1) * 2 / (w + 1)) - 1) < 0.002
    for s0, s1 in ((2**31 - 100_000, 2**31 + 100_000), (n - 200_000, n), (0, 100_000)):
        eh, ep = oracle.minimizers(_decode_2bit(words, s0, s1), k, w)
        lo, hi = s0 + w - 1, s1 - k - w + 1
        ep = ep.astype(np.int64) + s0
        keep = (ep >= lo) & (ep <= hi)
        ab = torch.searchsorted(p64, torch.tensor([lo, hi + 1], device=p64.device)).cpu().numpy()
        gp = p64[ab[0]:ab[1]].cpu().numpy()
        gh = host_u64(h[ab[0]:ab[1]])
        assert np.array_equal(gp, ep[keep]), (s0, s1)
        assert np.array_equal(gh, eh[keep]), (s0, s1)
    del r, h, p, p64, packed
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k,w", [(15, 10), (13, 40)])
def test_kept_workspace_across_calls(k, w):
    """SWS_WORKSPACE_KEPT: one runner's workspace kept across calls of falling
    and rising length (the look-back status words of earlier calls stay in it,
    told apart by their epoch), through the wave (w <= 32) and block (w > 32)
    kernels, with calls without the flag in between; every call against the
    oracle."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd import _lib
    r = sws.MinimizerRunner(400_000, k, w)
    plan = [(400_000, 0.0), (120_000, 0.01), (3_000, 0.0), (30, 0.0), (400_000, 0.02),
            (250_001, 0.0), (400_000, 0.0)]
    for i, (n, n_rate) in enumerate(plan):
        s = inputs.dna(n, seed=500 + i, n_rate=n_rate)
        if i == 4:
            r.calls = 1 << 29  # this call goes without the flag (the periodic clearing)
        r.launch(seq=seq_dev(torch, s))
        h, p = r.result()
        eh, ep = oracle.minimizers(s, k, w)
        assert np.array_equal(host_u32(p), ep) and np.array_equal(host_u64(h), eh), (i, n)
    assert r.calls > 1 << 29
    assert _lib.WORKSPACE_KEPT == 8
