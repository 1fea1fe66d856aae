"""Tiny pure-Python brute force, a second formulation that checks oracle.c.

TEST INFRASTRUCTURE ONLY.  Written for inputs of a few dozen elements; it works
on Python integers and strings, not on the C code's arrays and loops.

* ``sliding_sum``: Eq. 2 of Sec. 2.2 as ``functools.reduce`` over each slice.
* ``kmer_strings`` / ``kmer_value``: Sec. 2.4 treats a k-mer as a sliding sum of
  bases under string concatenation; here the k-mers are literal substrings, the
  reverse complement is a translated and reversed string, the canonical k-mer
  is the string-wise smaller one, and the value is the base-4 reading of the
  string with A<C<G<T (lexicographic order, Sec. 2.4).
* ``minimizers``: Sec. 2.4 / Fig. 2, windows of w consecutive k-mers, the
  smallest (value, position) pair per window via ``min``, adjacent equal pairs
  stored once.
"""
from __future__ import annotations

import functools

MASK32 = (1 << 32) - 1
MASK64 = (1 << 64) - 1

_DIGIT = {"A": "0", "C": "1", "G": "2", "T": "3"}
_COMPLEMENT = str.maketrans("ACGT", "TGCA")


def op_fn(op: str):
    if op == "add":
        return lambda u, v: (u + v) & MASK32
    if op == "min":
        return min
    if op == "max":
        return max
    if op == "affine":
        # compose the maps z -> a*z + b: (a, b) then (c, d) gives (a*c, a*d + b)
        return lambda u, v: ((u[0] * v[0]) & MASK32, (u[0] * v[1] + u[1]) & MASK32)
    raise ValueError(op)


def sliding_sum(op: str, w: int, xs):
    """xs: list of ints (or of (a, b) tuples for affine)."""
    f = op_fn(op)
    return [functools.reduce(f, xs[i:i + w]) for i in range(len(xs) - w + 1)]


def hash64(v: int) -> int:
    """The fixed xorshift-multiply mix over Python integers."""
    c1, c2 = 0x9E3779B97F4A7C15, 0x243F6A8885A308D3
    v ^= v >> 32
    v = (v * c1) & MASK64
    v ^= v >> 29
    v = (v * c2) & MASK64
    v ^= v >> 32
    return v


def kmer_strings(seq: str, k: int):
    """All substrings of length k, upper-cased, with None for those that hold
    a byte outside ACGT."""
    out = []
    for i in range(len(seq) - k + 1):
        s = seq[i:i + k].upper()
        out.append(s if all(ch in _DIGIT for ch in s) else None)
    return out


def revcomp(s: str) -> str:
    return s.translate(_COMPLEMENT)[::-1]


def kmer_value(s: str, canonical: bool = True, hashed: bool = True) -> int:
    if canonical:
        s = min(s, revcomp(s))
    v = int("".join(_DIGIT[ch] for ch in s), 4)
    return hash64(v) if hashed else v


def kmers(seq: str, k: int, canonical: bool = True, hashed: bool = True):
    return [MASK64 if s is None else kmer_value(s, canonical, hashed)
            for s in kmer_strings(seq, k)]


def window_minima(seq: str, k: int, w: int, canonical: bool = True, hashed: bool = True):
    """For each window p, the minimum (value, pos) pair or None."""
    strs = kmer_strings(seq, k)
    keys = [None if s is None else (kmer_value(s, canonical, hashed), i)
            for i, s in enumerate(strs)]
    res = []
    for p in range(len(keys) - w + 1):
        valid = [key for key in keys[p:p + w] if key is not None]
        res.append(min(valid) if valid else None)
    return res


def minimizers(seq: str, k: int, w: int, canonical: bool = True, hashed: bool = True):
    """List of (value, pos) pairs stored in the seed position table."""
    out = []
    prev = None
    for m in window_minima(seq, k, w, canonical, hashed):
        if m is not None and m != prev:
            out.append(m)
        prev = m
    return out
