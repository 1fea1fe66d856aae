"""Checks that pin the CPU oracle to facts other than itself.

Every check takes a loaded oracle library (``oracle.load()`` or a deliberately
mutated build) and raises AssertionError on a mismatch.  The facts come from
the paper (Eq. 2, the scalar- and vector-input forms of Sec. 3.1, the Fig. 2
worked example), from closed forms
(prefix differences for +, global extrema, products), from library routines
(numpy's sliding-window views), from mathematics (the hash constants), and from
brute force on tiny inputs.  ``ALL_PINS`` lists them so that a test can show
each planted oracle mistake is caught by at least one.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
M32 = (1 << 32) - 1
M64 = (1 << 64) - 1
IDENT = {"add": 0, "min": M32, "max": 0, "affine": (1, 0)}


# ---------------------------------------------------------------- helpers
def _to_list(op, x):
    return [tuple(int(v) for v in r) for r in x] if op == "affine" else [int(v) for v in x]


def _from_list(op, ys):
    if op == "affine":
        return np.array(ys, dtype=np.uint32).reshape(-1, 2)
    return np.array(ys, dtype=np.uint32)


def _fold(f, vals):
    acc = vals[0]
    for v in vals[1:]:
        acc = f(acc, v)
    return acc


def carried_state(op, w, xs, i):
    """The state Sec. 3.1 carries from one input to the next: before x_i
    arrives, entry t (t = 0 .. w-2) holds x_{i-w+1+t} (+) ... (+) x_{i-1}, the
    part of each pending window already seen (the identity where it reaches
    before x_0)."""
    f, e = brute.op_fn(op), IDENT[op]
    return [_fold(f, [e] + xs[max(0, i - w + 1 + t):i]) for t in range(w - 1)]


def scalar_input_outputs(op, w, xs):
    """The scalar-input form of Sec. 3.1 restated as a state machine: one
    input at a time, the window that ends at x_i is entry 0 of the state
    combined with x_i, and every pending partial window takes x_i on its
    right.  The state is checked against its definition at every step."""
    f = brute.op_fn(op)
    n = len(xs)
    if n < w:
        return []
    state = carried_state(op, w, xs, w - 1)
    out = []
    for i in range(w - 1, n):
        assert state == carried_state(op, w, xs, i), ("state", op, w, i)
        out.append(f(state[0], xs[i]) if w > 1 else xs[i])
        # windows still pending after x_i: those ending at x_{i+1} .. x_{i+w-1}
        state = [f(v, xs[i]) for v in state[1:]] + ([xs[i]] if w > 1 else [])
    return out


def block_input_outputs(op, w, xs, P):
    """The vector-input form of Sec. 3.1 restated by splitting each window at
    a block boundary: blocks of P >= w inputs start at w-1, w-1+P, ...; the
    window ending at x_j in the block that starts at b is the carried part
    before b (the state entry for that window) followed by the in-block prefix
    x_b .. x_j, or lies wholly inside the block.  The state passed on is the
    definition of carried_state at the next block start."""
    f, e = brute.op_fn(op), IDENT[op]
    n = len(xs)
    if n < w:
        return []
    out = [None] * (n - w + 1)
    b = w - 1
    state = carried_state(op, w, xs, b)
    while b < n:
        blk = [xs[j] if j < n else e for j in range(b, b + P)]
        pref = []
        for v in blk:                     # in-block prefixes x_b .. x_j
            pref.append(v if not pref else f(pref[-1], v))
        for q in range(P):
            j = b + q
            if j >= n:
                break
            start = j - w + 1
            if start < b:                 # spans the block start
                y = f(state[q], pref[q]) if w > 1 else pref[q]
            else:                         # wholly inside the block
                y = _fold(f, blk[start - b:q + 1])
            out[start] = y
        b += P
        state = carried_state(op, w, xs, b)
    return out


def golden_ratio_c1():
    """floor(2^64 * (sqrt(5) - 1) / 2) with exact integer arithmetic."""
    return (math.isqrt(5 << 128) - (1 << 64)) >> 1


def pi_fraction_c2():
    """floor(2^64 * (pi - 3)) from Machin's formula in 2^-128 fixed point."""
    S = 1 << 128

    def arctan_inv(x):
        total, k, term = 0, 0, S // x
        while term:
            total += term // (2 * k + 1) if k % 2 == 0 else -(term // (2 * k + 1))
            term //= x * x
            k += 1
        return total

    pi = 16 * arctan_inv(5) - 4 * arctan_inv(239)
    return (pi >> 64) - (3 << 64)


def py_mix64_inverse(y: int) -> int:
    """Inverse of the hash with constants derived here from mathematics."""
    c1i = pow(golden_ratio_c1(), -1, 1 << 64)
    c2i = pow(pi_fraction_c2(), -1, 1 << 64)
    y ^= y >> 32
    y = (y * c2i) & M64
    y ^= (y >> 29) ^ (y >> 58)
    y = (y * c1i) & M64
    y ^= y >> 32
    return y


def read_golden(name):
    facts = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            facts[key] = vals
    return facts


# ---------------------------------------------------------------- sliding sum pins
def pin_sliding_bruteforce(lib):
    """Exhaustive tiny inputs versus functools.reduce over each slice."""
    alphabet = [0, 1, 2, 1 << 31, M32]
    for op in ("add", "min", "max"):
        for n in range(0, 5):
            for xs in itertools.product(alphabet, repeat=n):
                x = np.array(xs, dtype=np.uint32)
                for w in range(1, n + 2):
                    got = oracle.sliding_sum(op, w, x, lib=lib)
                    exp = _from_list(op, brute.sliding_sum(op, w, list(xs)))
                    assert np.array_equal(got, exp), (op, xs, w)
    rng = np.random.default_rng(11)
    pairs = [(a, b) for a in (0, 1, 2, 3, M32) for b in (0, 1, 5, M32)]
    for n in range(1, 8):
        for _ in range(20):
            xs = [pairs[j] for j in rng.integers(0, len(pairs), n)]
            x = np.array(xs, dtype=np.uint32).reshape(n, 2)
            for w in range(1, n + 1):
                got = oracle.sliding_sum("affine", w, x, lib=lib)
                exp = _from_list("affine", brute.sliding_sum("affine", w, xs))
                assert np.array_equal(got, exp), (xs, w)


def pin_add_prefix_difference(lib):
    """+ mod 2^32 is invertible: y_i = Pfx_{i+w} - Pfx_i with Pfx exclusive."""
    rng = np.random.default_rng(12)
    x = rng.integers(0, 1 << 32, 3000, dtype=np.uint32)
    pfx = np.concatenate([np.zeros(1, np.uint64), np.cumsum(x.astype(np.uint64))])
    for w in (1, 2, 3, 16, 100, 1024, 3000):
        got = oracle.sliding_sum("add", w, x, lib=lib)
        exp = ((pfx[w:] - pfx[:-w]) & np.uint64(M32)).astype(np.uint32)
        assert np.array_equal(got, exp), w


def pin_minmax_library(lib):
    """min/max windows equal numpy's reductions over sliding-window views;
    w = n gives the global extremum and w = 1 the input itself."""
    rng = np.random.default_rng(13)
    x = rng.integers(0, 1 << 32, 2000, dtype=np.uint32)
    for w in (1, 2, 5, 16, 333, 2000):
        v = sliding_window_view(x, w)
        assert np.array_equal(oracle.sliding_sum("min", w, x, lib=lib), v.min(axis=1)), w
        assert np.array_equal(oracle.sliding_sum("max", w, x, lib=lib), v.max(axis=1)), w
    assert oracle.sliding_sum("min", 2000, x, lib=lib)[0] == x.min()
    assert np.array_equal(oracle.sliding_sum("max", 1, x, lib=lib), x)


def pin_minmax_deque(lib):
    """The O(N) deque gives the same min/max windows as numpy's reductions over
    sliding-window views and as the fold: on random values with many ties, on
    increasing, decreasing and constant runs (the queue's longest and shortest
    states), for w from 1 to n and w > n (no output)."""
    rng = np.random.default_rng(15)
    cases = [rng.integers(0, 4, 700, dtype=np.uint32),
             rng.integers(0, 1 << 32, 700, dtype=np.uint32),
             np.arange(700, dtype=np.uint32), np.arange(700, 0, -1).astype(np.uint32),
             np.full(700, 9, dtype=np.uint32),
             np.concatenate([np.arange(300), np.arange(300, 0, -1), np.zeros(100)]).astype(np.uint32)]
    for x in cases:
        for w in (1, 2, 3, 7, 64, 699, 700):
            v = sliding_window_view(x, w)
            for op, red in (("min", v.min), ("max", v.max)):
                got = oracle.sliding_extremum_deque(op, w, x, lib=lib)
                assert np.array_equal(got, red(axis=1)), (op, w)
                assert np.array_equal(got, oracle.sliding_sum(op, w, x, lib=lib)), (op, w)
        assert oracle.sliding_extremum_deque("min", 701, x, lib=lib).size == 0
    for bad in ("add", "affine"):
        try:
            oracle.sliding_extremum_deque(bad, 4, cases[0], lib=lib)
        except ValueError:
            continue
        raise AssertionError("deque accepted " + bad)


def pin_affine_prefix(lib):
    """For odd multipliers the prefix formulation equals the fold of Eq. 2 at
    every window length, including w = 1 (the input), w = n (one output) and
    multipliers near 2^32; an even multiplier is refused."""
    rng = np.random.default_rng(16)
    for n in (1, 2, 9, 300):
        a = rng.integers(0, 1 << 31, n, dtype=np.uint64).astype(np.uint32) * 2 + 1
        a[::7] = 0xFFFFFFFF
        b = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        x = np.stack([a, b], axis=1)
        for w in sorted({1, 2, 3, 8, n // 2 + 1, n}):
            if w > n:
                continue
            got = oracle.affine_windows_by_prefix(w, x, lib=lib)
            assert np.array_equal(got, oracle.sliding_sum("affine", w, x, lib=lib)), (n, w)
    x = np.array([[3, 1], [4, 1], [5, 9]], dtype=np.uint32)
    try:
        oracle.affine_windows_by_prefix(2, x, lib=lib)
    except ValueError:
        return
    raise AssertionError("an even multiplier was accepted")


def pin_minmax_composition(lib):
    """Idempotent ops compose: S_a(S_b(x)) = S_{a+b-1}(x)."""
    rng = np.random.default_rng(14)
    x = rng.integers(0, 1000, 500, dtype=np.uint32)
    for op in ("min", "max"):
        for a, b in ((2, 3), (5, 5), (1, 7), (16, 17)):
            lhs = oracle.sliding_sum(op, a, oracle.sliding_sum(op, b, x, lib=lib), lib=lib)
            rhs = oracle.sliding_sum(op, a + b - 1, x, lib=lib)
            assert np.array_equal(lhs, rhs), (op, a, b)


def pin_affine_reductions(lib):
    """a = 1 reduces to + on b; b = 0 reduces to a product of the a's; and every
    output, applied as a map, equals applying the w maps one after another,
    innermost (rightmost) first."""
    rng = np.random.default_rng(15)
    n = 400
    b = rng.integers(0, 1 << 32, n, dtype=np.uint32)
    a = rng.integers(0, 1 << 32, n, dtype=np.uint32) | np.uint32(1)
    for w in (1, 2, 7, 64):
        ones = np.stack([np.ones(n, np.uint32), b], axis=1)
        y = oracle.sliding_sum("affine", w, ones, lib=lib)
        assert np.all(y[:, 0] == 1)
        assert np.array_equal(y[:, 1], oracle.sliding_sum("add", w, b, lib=lib)), w
        prods = np.stack([a, np.zeros(n, np.uint32)], axis=1)
        y = oracle.sliding_sum("affine", w, prods, lib=lib)
        assert np.all(y[:, 1] == 0)
        for i in range(0, n - w + 1, 37):
            p = 1
            for j in range(i, i + w):
                p = (p * int(a[j])) & M32
            assert int(y[i, 0]) == p, (w, i)
        x = np.stack([a, b], axis=1)
        y = oracle.sliding_sum("affine", w, x, lib=lib)
        for i in range(0, n - w + 1, 29):
            z = int(rng.integers(0, 1 << 32))
            v = z
            for j in range(i + w - 1, i - 1, -1):
                v = (int(a[j]) * v + int(b[j])) & M32
            assert (int(y[i, 0]) * z + int(y[i, 1])) & M32 == v, (w, i)


def pin_paper_algorithms(lib):
    """The two vector forms of Sec. 3.1, restated from the windows they
    combine: one input at a time through the carried state of partial
    windows, and one block of P >= w inputs at a time by splitting windows at
    the block start.  Both give the oracle's outputs, every op."""
    rng = np.random.default_rng(16)
    for op in ("add", "min", "max", "affine"):
        for n in (1, 5, 23, 64):
            if op == "affine":
                x = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint32)
                x[:, 0] |= 1
            else:
                x = rng.integers(0, 1 << 32, n, dtype=np.uint32)
            xs = _to_list(op, x)
            for w in (1, 2, 3, 5, 8):
                exp = oracle.sliding_sum(op, w, x, lib=lib)
                assert np.array_equal(_from_list(op, scalar_input_outputs(op, w, xs)), exp), (op, n, w)
                for P in (w, w + 2, 16):
                    if P < w:
                        continue
                    assert np.array_equal(_from_list(op, block_input_outputs(op, w, xs, P)), exp), (op, n, w, P)


# ---------------------------------------------------------------- hash pins
def pin_mix64(lib):
    """The C hash inverts with constants derived from sqrt(5) and pi; the C
    inverse inverts it; 0 is a fixed point."""
    assert golden_ratio_c1() == 0x9E3779B97F4A7C15
    assert pi_fraction_c2() == 0x243F6A8885A308D3
    rng = np.random.default_rng(17)
    x = rng.integers(0, M64, 100_000, dtype=np.uint64, endpoint=True)
    h = oracle.mix64(x, lib=lib)
    assert np.array_equal(oracle.mix64(h, inverse=True, lib=lib), x)
    assert np.array_equal(oracle.mix64(oracle.mix64(x, inverse=True, lib=lib), lib=lib), x)
    for v in list(x[:200]) + [0, 1, M64, (1 << 30) - 1, (1 << 38) - 1]:
        assert py_mix64_inverse(oracle.mix64(int(v), lib=lib)) == int(v)
    assert oracle.mix64(0, lib=lib) == 0
    assert np.unique(h).size == h.size


# ---------------------------------------------------------------- k-mer pins
def _random_seq(rng, n, n_rate=0.1, lower_rate=0.1):
    letters = np.frombuffer(b"ACGT", dtype=np.uint8)[rng.integers(0, 4, n)]
    letters = letters.copy()
    letters[rng.random(n) < n_rate] = ord("N")
    low = (rng.random(n) < lower_rate) & (letters != ord("N"))
    letters[low] |= 0x20
    return letters.tobytes().decode()


def pin_kmers_strings(lib):
    """k-mer values equal the base-4 reading of literal substrings, the reverse
    complement the translated reversed substring."""
    rng = np.random.default_rng(18)
    for k in (1, 2, 3, 5, 9, 15, 16, 19, 31):
        for _ in range(4):
            s = _random_seq(rng, int(rng.integers(0, 80)))
            for can, hsh in itertools.product((True, False), repeat=2):
                got = oracle.kmers(s, k, canonical=can, hashed=hsh, lib=lib)
                exp = np.array(brute.kmers(s, k, can, hsh), dtype=np.uint64)
                assert np.array_equal(got, exp), (k, s, can, hsh)


def pin_kmer_strand_symmetry(lib):
    """Canonical k-mers do not depend on the strand: the k-mer at i of s equals
    the k-mer at n-k-i of the reverse complement of s; forward k-mers follow
    the shift-or recurrence fwd_{i+1} = (fwd_i * 4 + code) mod 4^k."""
    rng = np.random.default_rng(19)
    codes = {"A": 0, "C": 1, "G": 2, "T": 3}
    for k in (1, 4, 15, 21, 31):
        s = _random_seq(rng, 300, n_rate=0.0, lower_rate=0.0)
        rc = brute.revcomp(s)
        a = oracle.kmers(s, k, hashed=False, lib=lib)
        b = oracle.kmers(rc, k, hashed=False, lib=lib)
        assert np.array_equal(a, b[::-1]), k
        f = oracle.kmers(s, k, canonical=False, hashed=False, lib=lib)
        mask = (1 << (2 * k)) - 1
        for i in range(len(f) - 1):
            assert int(f[i + 1]) == ((int(f[i]) << 2) | codes[s[i + k]]) & mask, (k, i)
        fr = oracle.kmers(rc, k, canonical=False, hashed=False, lib=lib)
        assert np.array_equal(np.minimum(f, fr[::-1]), a), k


# ---------------------------------------------------------------- minimizer pins
def pin_fig2_worked_example(lib):
    """Sec. 2.4 / Fig. 2: k=3, w=3, forward lexicographic minimizers."""
    g = read_golden("fig2_worked_example.txt")
    k, w, seq = int(g["k"][0]), int(g["w"][0]), g["sequence"][0]
    nwin = len(seq) - k - w + 2
    assert nwin == int(g["windows"][0])
    for method in ("naive", "deque"):
        h, p = oracle.minimizers(seq, k, w, canonical=False, hashed=False, method=method, lib=lib)
        assert sorted(p.tolist()) == [int(v) for v in g["stored_positions"]], method
        dropped = sorted(set(range(len(seq) - k + 1)) - set(p.tolist()))
        assert dropped == [int(v) for v in g["dropped_positions"]], method
        s_str, s_pos = g["shared_minimizer"][0], int(g["shared_minimizer"][1])
        val = int("".join(str("ACGT".index(c)) for c in s_str), 4)
        assert (val, s_pos) in list(zip(h.tolist(), p.tolist())), method
    # the shared windows really share: their minima are equal and stored once
    mins = brute.window_minima(seq, k, w, canonical=False, hashed=False)
    i1, i2 = (int(v) for v in g["shared_windows"])
    assert mins[i1] == mins[i2] == (val, s_pos)


def _np_minimizers(vals, w):
    """Library formulation: argmin over sliding-window views picks the
    leftmost minimum; invalid k-mers carry the all-ones value and a window
    whose minimum is an invalid k-mer is empty."""
    nk = vals.size
    if nk < w:
        return [], []
    valid = vals != np.uint64(M64)
    keyv = np.where(valid, vals, np.uint64(M64))
    v = sliding_window_view(keyv, w)
    arg = v.argmin(axis=1) + np.arange(v.shape[0])
    nonempty = valid[arg] | (sliding_window_view(valid, w).any(axis=1))
    # a window whose only candidates tie at the all-ones hash: pick the first valid
    fix = nonempty & ~valid[arg]
    for p in np.nonzero(fix)[0]:
        arg[p] = p + int(np.argmax(valid[p:p + w]))
    hs, ps = [], []
    prev = None
    for p in range(v.shape[0]):
        if not nonempty[p]:
            prev = None
            continue
        m = int(arg[p])
        if m != prev:
            hs.append(int(vals[m]))
            ps.append(m)
        prev = m
    return hs, ps


def pin_minimizers_bruteforce(lib):
    """All 4^n sequences, n <= 6, plus random ones with N, versus brute force."""
    for n in range(0, 7):
        for t in itertools.product("ACGT", repeat=n):
            s = "".join(t)
            for k in (1, 2, 3):
                for w in (1, 2, 3, 4):
                    exp = brute.minimizers(s, k, w, canonical=False, hashed=False)
                    h, p = oracle.minimizers(s, k, w, canonical=False, hashed=False, lib=lib)
                    assert list(zip(h.tolist(), p.tolist())) == exp, (s, k, w)
    rng = np.random.default_rng(20)
    for _ in range(300):
        s = _random_seq(rng, int(rng.integers(0, 40)), n_rate=0.08)
        k, w = int(rng.integers(1, 6)), int(rng.integers(1, 7))
        can, hsh = bool(rng.integers(0, 2)), bool(rng.integers(0, 2))
        exp = brute.minimizers(s, k, w, can, hsh)
        for method in ("naive", "deque"):
            h, p = oracle.minimizers(s, k, w, can, hsh, method=method, lib=lib)
            assert list(zip(h.tolist(), p.tolist())) == exp, (s, k, w, can, hsh, method)


def pin_minimizers_invariants(lib):
    """On longer random inputs (with N runs and repeats): naive == deque ==
    the sliding-window-view formulation; every window's minimum is stored with
    a position inside the window; positions strictly increase; w = 1 stores
    every valid k-mer."""
    rng = np.random.default_rng(21)
    for trial in range(6):
        n = 3000
        s = _random_seq(rng, n, n_rate=0.02 * trial)
        if trial == 5:
            s = "A" * 200 + "ACGT" * 100 + "T" * 150 + s[:1000]
        for k, w in ((3, 4), (15, 10), (19, 19), (5, 1), (31, 7)):
            hn, pn = oracle.minimizers(s, k, w, method="naive", lib=lib)
            hd, pd = oracle.minimizers(s, k, w, method="deque", lib=lib)
            assert np.array_equal(hn, hd) and np.array_equal(pn, pd), (trial, k, w)
            vals = oracle.kmers(s, k, lib=lib)
            eh, ep = _np_minimizers(vals, w)
            assert hn.tolist() == eh and pn.tolist() == ep, (trial, k, w)
            assert np.all(np.diff(pn.astype(np.int64)) > 0)
            if w == 1:
                assert pn.tolist() == np.nonzero(vals != np.uint64(M64))[0].tolist()


def pin_minimizer_density(lib):
    """Sec. 2.4 cites a new minimizer about every w/2 bases; for a random
    order the expected count is 1 + (W - 1) * 2 / (w + 1) over W windows."""
    rng = np.random.default_rng(22)
    s = np.frombuffer(b"ACGT", dtype=np.uint8)[rng.integers(0, 4, 400_000)].tobytes()
    for w in (10, 19):
        h, p = oracle.minimizers(s, 15, w, lib=lib)
        W = len(s) - 15 - w + 2
        expected = 1 + (W - 1) * 2.0 / (w + 1)
        assert abs(h.size / expected - 1) < 0.02, (w, h.size, expected)


def pin_batch(lib):
    """Batch mode equals the single-sequence oracle read by read."""
    rng = np.random.default_rng(23)
    lens = rng.integers(0, 60, 50)
    reads = [_random_seq(rng, int(L), n_rate=0.05) for L in lens]
    seqs = "".join(reads)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    for k, w in ((3, 3), (5, 4), (15, 10)):
        h, p, r, ro = oracle.minimizers_batch(seqs, offsets, k, w, lib=lib)
        for i, s in enumerate(reads):
            eh, ep = oracle.minimizers(s, k, w, lib=lib)
            a, b = int(ro[i]), int(ro[i + 1])
            assert np.array_equal(h[a:b], eh) and np.array_equal(p[a:b], ep), (i, k, w)
            assert np.all(r[a:b] == i)
        assert int(ro[-1]) == h.size


# ---------------------------------------------------------------- seed table pins
def _seed_code(s):
    return int("".join(str("ACGT".index(c)) for c in s), 4)


def pin_fig1_seed_table(lib):
    """Sec. 2.4 / Fig. 1 over the Fig. 2 minimizers: pointer and position tables."""
    g = read_golden("fig1_seed_table.txt")
    f2 = read_golden("fig2_worked_example.txt")
    k = int(g["k"][0])
    assert 4 ** k == int(g["seeds"][0])
    h, p = oracle.minimizers(f2["sequence"][0], k, int(f2["w"][0]), canonical=False,
                             hashed=False, lib=lib)
    hits = g["hits"]
    assert sorted(zip(h.tolist(), p.tolist())) == sorted(
        (_seed_code(hits[i]), int(hits[i + 1])) for i in range(0, len(hits), 2))
    ptr, po, ho = oracle.seed_table(h, p, 2 * k, 0, lib=lib)
    # the paper's table is ptr[1:] (entry s closes the list of s)
    paper = ptr[1:]
    first = int(g["paper_pointer_nonzero_from"][0])
    assert np.all(paper[:first] == 0) and paper[first] != 0
    pp = g["paper_pointer"]
    for i in range(0, len(pp), 2):
        assert int(paper[_seed_code(pp[i])]) == int(pp[i + 1]), pp[i]
    assert po.tolist() == [int(v) for v in g["position_table"]]
    # hits of s lie between the lookups of the seed before s and of s
    ct = _seed_code("CTT")
    a, b = int(paper[ct - 1]), int(paper[ct])
    assert po[a:b].tolist() == [2] and ho[a:b].tolist() == [ct]


def _py_seed_table(h, p, bits, shift):
    """Definition by Python's sorted(): entries ordered by (key, input index)."""
    mask = (1 << bits) - 1
    keys = [(int(x) >> shift) & mask for x in h]
    order = sorted(range(len(keys)), key=lambda i: (keys[i], i))
    ptr = [sum(1 for kk in keys if kk < j) for j in range((1 << bits) + 1)]
    return ptr, [int(p[i]) for i in order], [int(h[i]) for i in order]


def pin_seed_table_bruteforce(lib):
    """Small random tables against the sorted() definition, every bits/shift
    combination of a few widths, duplicate keys and empty input included."""
    rng = np.random.default_rng(11)
    for count in (0, 1, 2, 7, 40, 300):
        for bits, shift in ((1, 0), (3, 0), (4, 60), (6, 5), (8, 56), (10, 30)):
            h = rng.integers(0, 1 << 63, count, dtype=np.uint64) * np.uint64(2) + \
                rng.integers(0, 2, count, dtype=np.uint64)
            if count > 10:
                h[: count // 3] = h[0]  # a heavy key
            p = np.sort(rng.choice(10 * count + 1, count, replace=False)).astype(np.uint32)
            ptr, po, ho = oracle.seed_table(h, p, bits, shift, lib=lib)
            eptr, epo, eho = _py_seed_table(h, p, bits, shift)
            assert ptr.tolist() == eptr, (count, bits, shift)
            assert po.tolist() == epo and ho.tolist() == eho, (count, bits, shift)


def pin_seed_table_invariants(lib):
    """On minimizers of a random genome: the pointer table is monotone and ends
    at the count; every group holds its own key only, in ascending position;
    the table is a permutation of the input."""
    rng = np.random.default_rng(12)
    seq = _random_seq(rng, 20000, n_rate=0.01)
    h, p = oracle.minimizers(seq, 15, 10, lib=lib)
    for bits, shift in ((12, 52), (16, 0), (20, 44)):
        ptr, po, ho = oracle.seed_table(h, p, bits, shift, lib=lib)
        assert ptr[0] == 0 and int(ptr[-1]) == h.size and np.all(np.diff(ptr.astype(np.int64)) >= 0)
        keys = (ho >> np.uint64(shift)) & np.uint64((1 << bits) - 1)
        for j in rng.integers(0, 1 << bits, 200):
            a, b = int(ptr[j]), int(ptr[j + 1])
            assert np.all(keys[a:b] == j) and np.all(np.diff(po[a:b].astype(np.int64)) > 0)
        assert sorted(zip(po.tolist(), ho.tolist())) == sorted(zip(p.tolist(), h.tolist()))


def pin_split_segments(lib):
    """Split semantics (invalid bases cut the sequence): equal to the string
    brute force run on every N-free segment, positions shifted by the
    segment's start; naive and deque agree."""
    import re
    rng = np.random.default_rng(13)
    for trial in range(60):
        n = int(rng.integers(1, 70))
        seq = _random_seq(rng, n, n_rate=float(rng.choice([0.0, 0.05, 0.2])), lower_rate=0.1)
        k = int(rng.integers(1, 5))
        w = int(rng.integers(1, 6))
        for canonical, hashed in ((True, True), (False, False)):
            exp = []
            for m in re.finditer(r"[ACGTacgt]+", seq):
                for h, p in brute.minimizers(m.group(0).upper(), k, w, canonical, hashed):
                    exp.append((h, p + m.start()))
            for method in ("naive", "deque"):
                h, p = oracle.minimizers(seq, k, w, canonical=canonical, hashed=hashed,
                                         method=method, lib=lib, split=True)
                assert list(zip(h.tolist(), p.tolist())) == exp, (seq, k, w, method)


ALL_PINS = [
    pin_sliding_bruteforce, pin_add_prefix_difference, pin_minmax_library, pin_minmax_deque,
    pin_affine_prefix, pin_minmax_composition, pin_affine_reductions, pin_paper_algorithms, pin_mix64,
    pin_kmers_strings, pin_kmer_strand_symmetry, pin_fig2_worked_example,
    pin_minimizers_bruteforce, pin_minimizers_invariants, pin_minimizer_density, pin_batch,
    pin_fig1_seed_table, pin_seed_table_bruteforce, pin_seed_table_invariants,
    pin_split_segments,
]
