"""Parity of the HIP seed-table builder with the CPU oracle (Sec. 2.4, Fig. 1).

Bit-exact: the pointer table, the position table and the hash table are
compared whole."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host_u32, host_u64, torch_cuda
from paper_1811_10074_amd import inputs

pytestmark = pytest.mark.gpu

TILE = 4096  # entries per workgroup tile of the radix passes


def check(torch, h, p, bits, shift, with_hash=True):
    import paper_1811_10074_amd as sws
    ptr, po, ho = sws.seed_table(dev(h, torch), dev(p, torch), bits, shift, with_hash=with_hash)
    torch.cuda.synchronize()
    eptr, epo, eho = oracle.seed_table(h, p, bits, shift)
    got_ptr = host_u32(ptr).astype(np.uint64)
    assert np.array_equal(got_ptr, eptr), (bits, shift, h.size, np.nonzero(got_ptr != eptr)[0][:5])
    assert np.array_equal(host_u32(po), epo), (bits, shift, h.size)
    if with_hash:
        assert np.array_equal(host_u64(ho), eho), (bits, shift, h.size)


def random_entries(rng, count, heavy=0.0):
    h = rng.integers(0, 1 << 63, count, dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, count, dtype=np.uint64)
    if heavy and count:
        m = int(count * heavy)
        h[rng.choice(count, m, replace=False)] = h[0]
    p = np.sort(rng.choice(4 * count + 7, count, replace=False)).astype(np.uint32)
    return h, p


def test_fig1_example():
    """The Fig. 2 worked example's minimizers as a k = 3 lexicographic table."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    seq = "AGCTTAGA"
    h, p = sws.minimizers(dev(np.frombuffer(seq.encode(), np.uint8).copy(), torch), 3, 3,
                          canonical=False, hashed=False)
    torch.cuda.synchronize()
    hh, pp = host_u64(h), host_u32(p)
    assert pp.tolist() == [0, 2, 5]
    check(torch, hh, pp, 6, 0)


@pytest.mark.parametrize("bits", [1, 5, 8, 9, 12, 13, 16, 17, 20, 24, 25])
def test_sizes_and_widths(bits):
    """Counts from 0 across several tiles with ragged tails, 1 to 4 radix
    passes; the last pass writes the pointer table, each tile its share, so
    the tile counts cover one tile, fewer tiles than dies, and several tiles
    per die (36 tiles over 8 dies)."""
    torch = torch_cuda()
    rng = np.random.default_rng(100 + bits)
    for count in (0, 1, 63, 64, 65, TILE - 1, TILE, TILE + 1, 3 * TILE + 777, 36 * TILE - 5):
        h, p = random_entries(rng, count)
        check(torch, h, p, bits, 64 - bits)
    h, p = random_entries(rng, 5000)
    check(torch, h, p, bits, 0)
    check(torch, h, p, bits, (64 - bits) // 2, with_hash=False)


def test_heavy_and_degenerate_keys():
    """One key holding most entries, all keys equal, keys already sorted and
    reversed: group order must stay the input order."""
    torch = torch_cuda()
    rng = np.random.default_rng(7)
    h, p = random_entries(rng, 50_000, heavy=0.7)
    check(torch, h, p, 20, 44)
    # a key holding 10000 entries: its run spans several tiles
    h, p = random_entries(rng, 50_000, heavy=0.2)
    check(torch, h, p, 20, 44)
    h2 = np.full(20_000, 0xDEADBEEF00000000, dtype=np.uint64)
    p2 = np.arange(20_000, dtype=np.uint32) * 3
    check(torch, h2, p2, 16, 48)
    hs = np.sort(rng.integers(0, 1 << 62, 30_000, dtype=np.uint64))
    ps = np.arange(30_000, dtype=np.uint32)
    check(torch, hs, ps, 24, 40)
    check(torch, hs[::-1].copy(), ps, 24, 40)


def test_from_minimizers_config2_scale():
    """The table over the minimizers of 2^24 bases (k = 15, w = 10), hashed
    (top 24 bits) and as a lexicographic table over all 4^12 seeds of the
    forward 12-mers (k = 12, identity)."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    seq = inputs.dna(1 << 24, seed=1)
    t = dev(seq, torch)
    h, p = sws.minimizers(t, 15, 10)
    torch.cuda.synchronize()
    check(torch, host_u64(h), host_u32(p), 24, 40)
    h, p = sws.minimizers(t, 12, 10, canonical=False, hashed=False)
    torch.cuda.synchronize()
    check(torch, host_u64(h), host_u32(p), 24, 0)


def test_runner_reuse_smaller():
    """A runner reused for a smaller table gives the same result as a fresh one."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    rng = np.random.default_rng(9)
    r = sws.SeedTableRunner(20_000, 12)
    for count in (20_000, 5_000):
        h, p = random_entries(rng, count)
        r.launch(dev(h, torch), dev(p, torch), 52)
        torch.cuda.synchronize()
        eptr, epo, eho = oracle.seed_table(h, p, 12, 52)
        assert np.array_equal(host_u32(r.ptr).astype(np.uint64), eptr)
        assert np.array_equal(host_u32(r.pos[:count]), epo)
        assert np.array_equal(host_u64(r.hash[:count]), eho)


@pytest.mark.parametrize("k", [4, 11])
def test_kmer_counting_composition(k):
    """K-mer counting as the seed table's pointer differences (Sec. 2.4): the
    forward k-mers of a sequence with N runs, keyed by their own 2k bits.  The
    count of every k-mer value equals a histogram of the oracle's k-mers, and
    each group's positions are that k-mer's occurrences in order."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    seq = inputs.dna(200_003, seed=70 + k, n_rate=0.01)
    km = sws.kmers(dev(seq, torch), k, canonical=False, hashed=False)
    ok = km != -1  # invalid k-mers carry 2^64 - 1; the compaction is test plumbing
    pos = torch.nonzero(ok).flatten().to(torch.int32)
    keys = km[ok].contiguous()
    ptr, po, _ = sws.seed_table(keys, pos, 2 * k, 0, with_hash=False)
    torch.cuda.synchronize()
    ek = oracle.kmers(seq, k, canonical=False, hashed=False)
    valid = ek != np.uint64(2**64 - 1)
    counts = np.bincount(ek[valid].astype(np.int64), minlength=1 << (2 * k))
    got = host_u32(ptr).astype(np.int64)
    assert np.array_equal(np.diff(got), counts)
    order = np.argsort(ek[valid], kind="stable")
    assert np.array_equal(host_u32(po), np.nonzero(valid)[0][order].astype(np.uint32))


def test_minimizer_counting_forward_lexicographic():
    """Counting over minimizers (Sec. 1's application) with the Fig. 2
    semantics: forward-strand, unhashed (lexicographic) k-mers.  The seed table
    over the minimizers, keyed by the 2k-bit k-mer itself, gives each k-mer's
    number of minimizer occurrences as ptr[j + 1] - ptr[j]."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    k, w = 9, 6
    seq = inputs.dna(300_007, seed=91, n_rate=0.005)
    h, p = sws.minimizers(dev(seq, torch), k, w, canonical=False, hashed=False)
    ptr, po, _ = sws.seed_table(h, p, 2 * k, 0, with_hash=False)
    torch.cuda.synchronize()
    eh, ep = oracle.minimizers(seq, k, w, canonical=False, hashed=False)
    counts = np.bincount(eh.astype(np.int64), minlength=1 << (2 * k))
    assert np.array_equal(np.diff(host_u32(ptr).astype(np.int64)), counts)
    order = np.argsort(eh, kind="stable")
    assert np.array_equal(host_u32(po), ep[order])


def test_fourteen_million_entries():
    """A table larger than config 2's (14 M entries, 24 bits): 3419 tiles,
    427 or 428 per die."""
    torch = torch_cuda()
    rng = np.random.default_rng(11)
    h, p = random_entries(rng, 14_000_000)
    check(torch, h, p, 24, 40)
