"""The oracle's multi-threaded drivers (chunks of one sequence, groups of
reads) give exactly the single-threaded oracle's results."""
import numpy as np
import pytest

import oracle
from paper_1811_10074_amd import inputs


@pytest.mark.parametrize("k,w", [(15, 10), (3, 3), (19, 19), (1, 1), (11, 40)])
def test_chunked_equals_whole(k, w):
    for seed, n, n_rate in ((1, 50_000, 0.0), (2, 60_001, 0.02), (3, 3000, 0.3)):
        s = inputs.dna(n, seed=seed, n_rate=n_rate)
        for split in (False, True):
            eh, ep = oracle.minimizers(s, k, w, split=split)
            for chunks in (1, 2, 7, 64, 1000):
                h, p = oracle.minimizers_chunked(s, k, w, threads=4, chunks=chunks, split=split)
                assert np.array_equal(p, ep), (k, w, seed, chunks, split)
                assert np.array_equal(h, eh), (k, w, seed, chunks, split)


def test_chunked_runs_of_one_value():
    """A poly-A stretch (every window ties, the leftmost wins) across chunk
    edges, and a stretch of N (windows with no minimizer)."""
    s = np.frombuffer(b"A" * 3000 + b"N" * 500 + b"ACGT" * 700, dtype=np.uint8).copy()
    eh, ep = oracle.minimizers(s, 7, 5)
    for chunks in (3, 50, 400):
        h, p = oracle.minimizers_chunked(s, 7, 5, threads=3, chunks=chunks)
        assert np.array_equal(p, ep) and np.array_equal(h, eh), chunks


def test_batch_parallel_equals_batch():
    seqs, off = inputs.read_batch(n_short=3000, n_long=20, seed=8)
    e = oracle.minimizers_batch(seqs, off, 15, 10)
    for threads in (1, 3, 8):
        g = oracle.minimizers_batch_parallel(seqs, off, 15, 10, threads=threads)
        for a, b in zip(g, e):
            assert np.array_equal(a, b), threads
    lens = np.array([0, 0, 5, 0, 100, 0], dtype=np.int64)
    off2 = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=off2[1:])
    s2 = inputs.dna(int(off2[-1]), seed=1)
    e2 = oracle.minimizers_batch(s2, off2, 3, 2)
    g2 = oracle.minimizers_batch_parallel(s2, off2, 3, 2, threads=4)
    for a, b in zip(g2, e2):
        assert np.array_equal(a, b)
