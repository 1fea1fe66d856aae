"""Seeded synthetic inputs for tests and the benchmark.

This module only draws random data with numpy's PCG64 (``default_rng(seed)``)
in a fixed call order.  It holds none of the method's arithmetic, so both the
HIP path and the CPU oracle can be fed the same buffers.

Recipes (the paper measures hashed 15-mers of a human genome assembly, Sec. 4;
that assembly is not available here, so i.i.d. uniform sequences of the same
shape stand in for it):

* ``uniform_u32``        u32 values uniform over [0, 2^32) (plain sliding sums).
* ``affine_pairs``       (a, b) u32 pairs for the affine-map operator; with
                         ``odd=True`` a is forced odd so that products of long
                         windows do not collapse to 0 mod 2^32.
* ``adversarial``        structured u32 inputs (sorted, constant, tiny
                         alphabet, sawtooth around the window length).
* ``dna``                i.i.d. uniform A/C/G/T text, optionally with N at a
                         given rate.
* ``read_batch``         many reads of uneven length: short reads plus
                         lognormal long reads, shuffled, concatenated with
                         CSR offsets.
* ``poisson_requests``   serving workload: Poisson arrival times, a log-uniform
                         number of reads per request, read lengths from the
                         batch mix.
"""
from __future__ import annotations

import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
N_BYTE = ord("N")


def uniform_u32(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, n, dtype=np.uint32)


def affine_pairs(n: int, seed: int, odd: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2**32, (n, 2), dtype=np.uint32)
    if odd:
        x[:, 0] |= np.uint32(1)
    return x


def adversarial(kind: str, n: int, w: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.uint64)
    if kind == "ascending":
        return (i & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    if kind == "descending":
        return (np.uint64(0xFFFFFFFF) - (i & np.uint64(0xFFFFFFFF))).astype(np.uint32)
    if kind == "constant":
        return np.full(n, 0x9E3779B9, dtype=np.uint32)
    if kind == "extremes":
        return rng.choice(np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32), n)
    if kind == "small_alphabet":
        return rng.integers(0, 3, n, dtype=np.uint32)
    if kind == "sawtooth_up":
        return (i % np.uint64(w + 1)).astype(np.uint32)
    if kind == "sawtooth_down":
        return (np.uint64(w) - i % np.uint64(max(w - 1, 1))).astype(np.uint32)
    raise ValueError(kind)


ADVERSARIAL_KINDS = ("ascending", "descending", "constant", "extremes", "small_alphabet",
                     "sawtooth_up", "sawtooth_down")


def dna_codes(n: int, seed: int) -> np.ndarray:
    """n base codes in {0, 1, 2, 3}, i.i.d. uniform."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 4, n, dtype=np.uint8)


def dna(n: int, seed: int, n_rate: float = 0.0, lowercase_rate: float = 0.0) -> np.ndarray:
    """n bytes of A/C/G/T text (uint8), i.i.d. uniform; with ``n_rate`` each
    byte is 'N' with that probability; with ``lowercase_rate`` each letter is
    lower-cased with that probability."""
    out = ACGT[dna_codes(n, seed)]
    if n_rate > 0 or lowercase_rate > 0:
        rng = np.random.default_rng(seed + 0x5EED)
        if n_rate > 0:
            out[rng.random(n) < n_rate] = N_BYTE
        if lowercase_rate > 0:
            low = (rng.random(n) < lowercase_rate) & (out != N_BYTE)
            out[low] = out[low] | np.uint8(0x20)
    return out


def _dna_n_percent(rng, n: int) -> np.ndarray:
    """n bytes, each 'N' with probability 1/100, else uniform A/C/G/T."""
    out = np.empty(n, dtype=np.uint8)
    chunk = 1 << 26
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        v = rng.integers(0, 400, e - s, dtype=np.uint16)
        b = ACGT[(v & 3).astype(np.uint8)]
        b[v < 4] = N_BYTE
        out[s:e] = b
    return out


def long_read_lengths(rng, count: int) -> np.ndarray:
    """Lognormal lengths, median 8 kb, sigma 0.8, clipped to [1 kb, 100 kb]."""
    ln = rng.lognormal(mean=np.log(8000.0), sigma=0.8, size=count)
    return np.clip(np.round(ln), 1000, 100000).astype(np.int64)


def read_batch(n_short: int = 2_000_000, n_long: int = 100_000, short_len: int = 150,
               seed: int = 3):
    """Uneven read batch: n_short reads of short_len bases plus n_long lognormal
    reads, shuffled, 1% N.  Returns (seqs uint8[total], offsets uint64[nreads+1])."""
    rng = np.random.default_rng(seed)
    lens = np.concatenate([np.full(n_short, short_len, dtype=np.int64),
                           long_read_lengths(rng, n_long)])
    lens = lens[rng.permutation(lens.size)]
    offsets = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    seqs = _dna_n_percent(rng, int(offsets[-1]))
    return seqs, offsets


def poisson_requests(rate: float = 200.0, duration_s: float = 60.0, max_reads: int = 4096,
                     short_len: int = 150, p_short: float = 2.0 / 2.1, seed: int = 4,
                     max_requests: int | None = None):
    """Serving workload.  Returns a list of (arrival_s, seqs uint8[], offsets
    uint64[]) in arrival order."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s or (max_requests is not None and len(reqs) >= max_requests):
            break
        count = int(min(max_reads, np.floor(np.exp(rng.random() * np.log(max_reads + 1)))))
        count = max(count, 1)
        short = rng.random(count) < p_short
        lens = np.where(short, short_len, long_read_lengths(rng, count)).astype(np.int64)
        offsets = np.zeros(count + 1, dtype=np.uint64)
        np.cumsum(lens, out=offsets[1:])
        seqs = _dna_n_percent(rng, int(offsets[-1]))
        reqs.append((t, seqs, offsets))
    return reqs
