/*
 * oracle.c -- plain, slow, obviously correct CPU reference for sliding window
 * sums and minimizer seed tables (Snytsar & Turakhia, "Parallel approach to
 * sliding window sums", arXiv:1811.10074).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its product path may
 * include, link or call this file.  It shares no header, table, constant or
 * helper with the HIP implementation; every constant below is typed here from
 * its own definition.  Only tests, the smoke check and the benchmark's CPU
 * baseline leg use it.
 *
 * Every routine is the plain definition written out, with no blocking,
 * reordering or fusion beyond what that definition states:
 *
 *   oracle_sliding_sum        Sec. 2.2, Eq. 2: y_i = x_i (+) ... (+) x_{i+w-1},
 *                             exactly w addends, as a left fold (the naive
 *                             O(wN) algorithm of Sec. 2.2).
 *   oracle_sliding_extremum_deque
 *                             the same outputs for min and max by the
 *                             monotone deque (the O(N) "Dequeue" the paper
 *                             compares against, Sec. 2.4, Sec. 4).
 *   oracle_affine_windows_by_prefix
 *                             the affine outputs for invertible maps (odd
 *                             multipliers) from prefix compositions, O(N).
 *   oracle_kmers              Sec. 2.4: k-mers as a sliding sum of bases under
 *                             concatenation, written as the positional value
 *                             sum_j code(s_{i+j}) * 4^(k-1-j); the reverse
 *                             complement likewise; canonical = the smaller.
 *   oracle_mix64(_inv)        the fixed invertible xorshift-multiply hash used
 *                             for the k-mer hashing of Sec. 4.  The paper names
 *                             no hash: parity unpinned against the paper; it is
 *                             pinned only to its own definition (known answers
 *                             and the inverse).
 *   oracle_minimizers_naive   Sec. 2.4 / Fig. 2: for every window of w
 *                             consecutive k-mers, the minimum (hash, position)
 *                             pair, leftmost on ties; adjacent windows with the
 *                             same pair are stored once.  O(w) per window.
 *   oracle_minimizers_deque   the same result with the monotone-deque sliding
 *                             minimum the paper cites as the O(N) alternative
 *                             (Sec. 2.4, "Dequeue" in Sec. 4 / Fig. 3).
 *   oracle_minimizers_batch   the deque routine run once per read.
 *   oracle_seed_table         Sec. 2.4 / Fig. 1: the seed pointer table and
 *                             seed position table over the stored minimizers,
 *                             keyed by key(h) = (h >> shift) mod 2^bits: a
 *                             count per key, the prefix of the counts, and the
 *                             entries placed key by key in their input order.
 *
 * Readings of points the paper leaves open (stated once here, used below):
 *   - identity of each operator pads nothing: the naive fold never needs it;
 *   - bases A/C/G/T (either case) code as 0/1/2/3 (lexicographic order, Sec.
 *     2.4); any other byte is invalid and a k-mer covering it is invalid;
 *   - an invalid k-mer never wins a window; a window with no valid k-mer
 *     stores nothing; positions are 0-based k-mer start offsets;
 *   - n < w (or fewer than w k-mers) gives no output at all;
 *   - with ORC_SPLIT, invalid bases split the sequence into segments and only
 *     windows wholly inside a segment count: a window holding an invalid
 *     k-mer stores nothing, as a window with no valid k-mer does.  The result
 *     is that of each segment taken as its own sequence, positions kept;
 *   - the seed pointer table has 2^bits + 1 entries, ptr[j] = number of
 *     entries with key < j, so the hits of key j are ptr[j] .. ptr[j+1] - 1.
 *     The paper's table, whose entry for seed s ends the list of s (the
 *     lookups of the seed before s and of s bound the hits of s), is
 *     ptr[1 ..].  Within one key the entries keep their input (position)
 *     order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Operator codes understood by oracle_sliding_sum. */
#define ORC_ADD 0
#define ORC_MIN 1
#define ORC_MAX 2
#define ORC_AFFINE 3

/* Minimizer flags understood by the oracle. */
#define ORC_FORWARD 1u  /* use the forward k-mer instead of the canonical one */
#define ORC_IDENTITY 2u /* use the k-mer value itself instead of its hash    */
#define ORC_SPLIT 4u    /* invalid bases split the sequence: a window holding
                           an invalid k-mer stores nothing                    */

/* ---------------------------------------------------------------------- */
/* Sec. 2.2, Eq. 2: the sliding window sum, one left fold of w addends.     */
/* ---------------------------------------------------------------------- */

/* The affine maps f(z) = a*z + b (mod 2^32), stored as pairs (a, b).
 * (a,b) (+) (c,d) is the composition f_ab(f_cd(z)) = a*c*z + a*d + b. */
static void affine_combine(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                           uint32_t *ra, uint32_t *rb) {
    *ra = (uint32_t)(a * c);
    *rb = (uint32_t)(a * d + b);
}

/* Returns the number of outputs (n - w + 1, or 0 when n < w), or -1 when the
 * operator is unknown or w is 0.  For ORC_AFFINE, x holds n interleaved
 * (a, b) pairs and y receives pairs. */
long long oracle_sliding_sum(int op, uint64_t w, const uint32_t *x, uint64_t n,
                             uint32_t *y) {
    if (w == 0 || op < ORC_ADD || op > ORC_AFFINE) return -1;
    if (n < w) return 0;
    uint64_t count = n - w + 1;
    for (uint64_t i = 0; i < count; ++i) {
        if (op == ORC_AFFINE) {
            uint32_t a = x[2 * i], b = x[2 * i + 1];
            for (uint64_t j = 1; j < w; ++j) {
                uint32_t na, nb;
                affine_combine(a, b, x[2 * (i + j)], x[2 * (i + j) + 1], &na, &nb);
                a = na;
                b = nb;
            }
            y[2 * i] = a;
            y[2 * i + 1] = b;
        } else {
            uint32_t acc = x[i];
            for (uint64_t j = 1; j < w; ++j) {
                uint32_t v = x[i + j];
                if (op == ORC_ADD) acc = (uint32_t)(acc + v);
                else if (op == ORC_MIN) acc = v < acc ? v : acc;
                else acc = v > acc ? v : acc;
            }
            y[i] = acc;
        }
    }
    return (long long)count;
}

/* The same outputs for ORC_MIN / ORC_MAX with the monotone double-ended
 * queue the paper names as its O(N) comparison ("Dequeue", Sec. 2.4 and the
 * Sec. 4 / Fig. 3 timings): the queue holds indices whose values strictly
 * improve from back to front; a new value removes every queued value it
 * matches or beats, the front leaves once it falls out of the window, and the
 * front is each window's extremum.  Returns the output count, 0 when n < w,
 * -1 for another operator or w = 0.  Used to check the kernels at sizes where
 * the O(wN) fold is too slow. */
long long oracle_sliding_extremum_deque(int op, uint64_t w, const uint32_t *x, uint64_t n,
                                        uint32_t *y) {
    if (w == 0 || (op != ORC_MIN && op != ORC_MAX)) return -1;
    if (n < w) return 0;
    uint64_t *dq = (uint64_t *)malloc((n < w ? n : w) * sizeof(uint64_t) + sizeof(uint64_t));
    if (!dq) return -3;
    const uint64_t cap = (n < w ? n : w) + 1;  /* ring buffer of queued indices */
    uint64_t head = 0, size = 0;
    for (uint64_t i = 0; i < n; ++i) {
        while (size > 0) {
            uint32_t back = x[dq[(head + size - 1) % cap]];
            int beaten = op == ORC_MIN ? x[i] <= back : x[i] >= back;
            if (!beaten) break;
            --size;
        }
        dq[(head + size) % cap] = i;
        ++size;
        if (i + 1 >= w) {
            uint64_t first = i + 1 - w; /* the window x[first .. i] */
            while (dq[head] < first) {
                head = (head + 1) % cap;
                --size;
            }
            y[first] = x[dq[head]];
        }
    }
    free(dq);
    return (long long)(n - w + 1);
}

/* Inverse of an odd a mod 2^32 by Newton's iteration inv <- inv * (2 - a * inv):
 * a * a == 1 mod 8 for odd a, and each step doubles the correct low bits. */
static uint32_t inverse_odd(uint32_t a) {
    uint32_t inv = a;
    for (int it = 0; it < 5; ++it) inv = (uint32_t)(inv * (2u - a * inv));
    return inv;
}

/* Affine windows for inputs whose multipliers are all odd (then every map
 * z -> a z + b is invertible mod 2^32), by prefix compositions: with
 * P_j = f_0 o f_1 o ... o f_{j-1}, the window W_i = f_i o ... o f_{i+w-1}
 * satisfies P_{i+w} = P_i o W_i, so W_i = P_i^{-1} o P_{i+w}.  Two running
 * prefixes (at i and at i + w) and the running inverse of the first make it
 * O(N).  Returns the output count, 0 when n < w, -1 for w = 0, -2 when a
 * multiplier is even.  A check of the kernels at sizes where the fold of
 * oracle_sliding_sum is too slow; pinned to the fold. */
long long oracle_affine_windows_by_prefix(uint64_t w, const uint32_t *x, uint64_t n,
                                          uint32_t *y) {
    if (w == 0) return -1;
    if (n < w) return 0;
    for (uint64_t i = 0; i < n; ++i)
        if ((x[2 * i] & 1u) == 0) return -2;
    /* P_w = f_0 o ... o f_{w-1} */
    uint32_t pb_a = 1, pb_b = 0;
    for (uint64_t j = 0; j < w; ++j) {
        uint32_t na, nb;
        affine_combine(pb_a, pb_b, x[2 * j], x[2 * j + 1], &na, &nb);
        pb_a = na;
        pb_b = nb;
    }
    uint32_t qa = 1, qb = 0; /* P_i^{-1}, starting from P_0 = identity */
    for (uint64_t i = 0; i + w <= n; ++i) {
        affine_combine(qa, qb, pb_a, pb_b, &y[2 * i], &y[2 * i + 1]);
        if (i + w == n) break;
        /* P_{i+1}^{-1} = f_i^{-1} o P_i^{-1}, with (a, b)^{-1} = (a^{-1}, -a^{-1} b) */
        uint32_t ia = inverse_odd(x[2 * i]);
        uint32_t ib = (uint32_t)(0u - ia * x[2 * i + 1]);
        uint32_t na, nb;
        affine_combine(ia, ib, qa, qb, &na, &nb);
        qa = na;
        qb = nb;
        /* P_{i+w+1} = P_{i+w} o f_{i+w} */
        affine_combine(pb_a, pb_b, x[2 * (i + w)], x[2 * (i + w) + 1], &na, &nb);
        pb_a = na;
        pb_b = nb;
    }
    return (long long)(n - w + 1);
}

/* ---------------------------------------------------------------------- */
/* The hash: x ^= x>>32; x *= C1; x ^= x>>29; x *= C2; x ^= x>>32 (mod 2^64) */
/* C1 = floor(2^64 * (golden ratio - 1)), C2 = floor(2^64 * (pi - 3)).       */
/* ---------------------------------------------------------------------- */
static const uint64_t ORC_C1 = 0x9E3779B97F4A7C15ull;
static const uint64_t ORC_C2 = 0x243F6A8885A308D3ull;
static const uint64_t ORC_C1_INV = 0xF1DE83E19937733Dull; /* C1 * C1_INV == 1 */
static const uint64_t ORC_C2_INV = 0xFBF07FAC8BAA8F5Bull; /* C2 * C2_INV == 1 */

uint64_t oracle_mix64(uint64_t x) {
    x ^= x >> 32;
    x *= ORC_C1;
    x ^= x >> 29;
    x *= ORC_C2;
    x ^= x >> 32;
    return x;
}

/* Undo each step in reverse order.  y ^= y>>29 is undone by
 * y ^= (y>>29) ^ (y>>58), since two applications of the shift reach past 64. */
uint64_t oracle_mix64_inv(uint64_t y) {
    y ^= y >> 32;
    y *= ORC_C2_INV;
    y ^= (y >> 29) ^ (y >> 58);
    y *= ORC_C1_INV;
    y ^= y >> 32;
    return y;
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.4: bases, k-mers, canonical k-mers.                              */
/* ---------------------------------------------------------------------- */

/* A=0, C=1, G=2, T=3 (either case); -1 for every other byte. */
int oracle_base_code(uint8_t c) {
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

/* The k-mer starting at i, its validity, forward value and reverse-complement
 * value, each straight from the positional definition. */
static int kmer_at(const uint8_t *seq, uint64_t i, uint32_t k, uint64_t *fwd,
                   uint64_t *rc) {
    uint64_t f = 0, r = 0, place = 1;
    for (uint32_t j = 0; j < k; ++j) {
        int c = oracle_base_code(seq[i + j]);
        if (c < 0) return 0;
        f = f * 4u + (uint64_t)c;             /* sum_j code * 4^(k-1-j)    */
        r = r + (uint64_t)(3 - c) * place;    /* sum_j (3 - code) * 4^j    */
        place *= 4u;
    }
    *fwd = f;
    *rc = r;
    return 1;
}

/* The value a k-mer contributes under the flags: forward or canonical, then
 * hashed or not. */
static uint64_t kmer_value(uint64_t fwd, uint64_t rc, uint32_t flags) {
    uint64_t v = fwd;
    if (!(flags & ORC_FORWARD) && rc < fwd) v = rc;
    if (!(flags & ORC_IDENTITY)) v = oracle_mix64(v);
    return v;
}

/* out[i] = value of the k-mer at i, or UINT64_MAX when it covers an invalid
 * base.  Returns n - k + 1 (0 when n < k), or -1 for k outside [1, 31]. */
long long oracle_kmers(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t flags,
                       uint64_t *out) {
    if (k < 1 || k > 31) return -1;
    if (n < k) return 0;
    uint64_t nk = n - k + 1;
    for (uint64_t i = 0; i < nk; ++i) {
        uint64_t f, r;
        out[i] = kmer_at(seq, i, k, &f, &r) ? kmer_value(f, r, flags) : UINT64_MAX;
    }
    return (long long)nk;
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.4 / Fig. 2: minimizers of windows of w consecutive k-mers.        */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint64_t h;
    uint64_t pos;
    int valid;
} orc_key;

/* Hash (or value) and validity of every k-mer of seq[0, n). */
static orc_key *all_keys(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t flags,
                         uint64_t *nk_out) {
    uint64_t nk = n >= k ? n - k + 1 : 0;
    orc_key *keys = (orc_key *)malloc((nk ? nk : 1) * sizeof(orc_key));
    if (!keys) return NULL;
    for (uint64_t i = 0; i < nk; ++i) {
        uint64_t f, r;
        keys[i].pos = i;
        keys[i].valid = kmer_at(seq, i, k, &f, &r);
        keys[i].h = keys[i].valid ? kmer_value(f, r, flags) : 0;
    }
    *nk_out = nk;
    return keys;
}

/* Lexicographic order on (hash, position): a is strictly smaller than b. */
static int key_less(const orc_key *a, const orc_key *b) {
    if (a->h != b->h) return a->h < b->h;
    return a->pos < b->pos;
}

/* The previous window's minimum, compared as a whole (hash and position). */
typedef struct {
    uint64_t h;
    uint64_t pos;
    int some; /* 0: no previous window, or the previous window was empty */
} orc_prev;

/* Store one window minimum unless it equals the previous window's. */
static void emit(uint64_t h, uint64_t pos, orc_prev *prev, uint64_t *count,
                 uint64_t *out_hash, uint32_t *out_pos, uint32_t *out_read,
                 uint32_t read, uint64_t cap) {
    int same = prev->some && prev->h == h && prev->pos == pos;
    prev->h = h;
    prev->pos = pos;
    prev->some = 1;
    if (same) return;
    if (*count < cap) {
        out_hash[*count] = h;
        out_pos[*count] = (uint32_t)pos;
        if (out_read) out_read[*count] = read;
    }
    *count += 1;
}

static int check_args(uint32_t k, uint32_t w, uint32_t flags) {
    return k >= 1 && k <= 31 && w >= 1 &&
           (flags & ~(ORC_FORWARD | ORC_IDENTITY | ORC_SPLIT)) == 0;
}

/* O(w) per window.  Returns the number of minimizers (entries beyond cap are
 * counted but not written), or -1 for bad arguments / -3 when out of memory. */
long long oracle_minimizers_naive(const uint8_t *seq, uint64_t n, uint32_t k,
                                  uint32_t w, uint32_t flags, uint64_t *out_hash,
                                  uint32_t *out_pos, uint64_t cap) {
    if (!check_args(k, w, flags)) return -1;
    uint64_t nk;
    orc_key *keys = all_keys(seq, n, k, flags, &nk);
    if (!keys) return -3;
    uint64_t count = 0;
    orc_prev prev = {0, 0, 0};
    if (nk >= w) {
        for (uint64_t p = 0; p + w <= nk; ++p) {
            const orc_key *best = NULL;
            int holds_invalid = 0;
            for (uint64_t j = p; j < p + w; ++j) {
                if (!keys[j].valid) {
                    holds_invalid = 1;
                    continue;
                }
                if (best == NULL || key_less(&keys[j], best)) best = &keys[j];
            }
            if ((flags & ORC_SPLIT) && holds_invalid) best = NULL;
            if (best == NULL) { /* no valid k-mer: nothing stored */
                prev.some = 0;
                continue;
            }
            emit(best->h, best->pos, &prev, &count, out_hash, out_pos, NULL, 0, cap);
        }
    }
    free(keys);
    return (long long)count;
}

/* Windows of one read, deque variant.  Appends to the outputs at *count. */
static int deque_windows(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t w,
                         uint32_t flags, uint64_t *out_hash, uint32_t *out_pos,
                         uint32_t *out_read, uint32_t read, uint64_t cap,
                         uint64_t *count) {
    uint64_t nk;
    orc_key *keys = all_keys(seq, n, k, flags, &nk);
    if (!keys) return -3;
    uint64_t *dq = (uint64_t *)malloc((nk ? nk : 1) * sizeof(uint64_t));
    if (!dq) {
        free(keys);
        return -3;
    }
    uint64_t head = 0, tail = 0; /* deque = dq[head, tail), keys increasing */
    orc_prev prev = {0, 0, 0};
    uint64_t next_clean = 0; /* first window start after the latest invalid k-mer */
    for (uint64_t i = 0; i < nk; ++i) {
        if (keys[i].valid) {
            while (tail > head && key_less(&keys[i], &keys[dq[tail - 1]])) --tail;
            dq[tail++] = i;
        } else {
            next_clean = i + 1;
        }
        if (i + 1 >= w) {
            uint64_t p = i + 1 - w; /* window p covers k-mers p .. i */
            while (tail > head && dq[head] < p) ++head;
            /* no valid k-mer in the window, or (split) an invalid one */
            if (tail == head || ((flags & ORC_SPLIT) && p < next_clean)) {
                prev.some = 0;
                continue;
            }
            const orc_key *m = &keys[dq[head]];
            emit(m->h, m->pos, &prev, count, out_hash, out_pos, out_read, read, cap);
        }
    }
    free(dq);
    free(keys);
    return 0;
}

/* Amortized O(1) per window (monotone deque).  Same contract as the naive
 * routine. */
long long oracle_minimizers_deque(const uint8_t *seq, uint64_t n, uint32_t k,
                                  uint32_t w, uint32_t flags, uint64_t *out_hash,
                                  uint32_t *out_pos, uint64_t cap) {
    if (!check_args(k, w, flags)) return -1;
    uint64_t count = 0;
    int rc = deque_windows(seq, n, k, w, flags, out_hash, out_pos, NULL, 0, cap, &count);
    return rc ? rc : (long long)count;
}

/* Reads r = 0 .. nreads-1 occupy seqs[offsets[r], offsets[r+1]).  Each read is
 * handled on its own: positions are relative to the read start and no window
 * spans two reads.  read_offsets[r] receives the index of read r's first
 * minimizer and read_offsets[nreads] the total.  Returns the total count. */
long long oracle_minimizers_batch(const uint8_t *seqs, const uint64_t *offsets,
                                  uint32_t nreads, uint32_t k, uint32_t w,
                                  uint32_t flags, uint64_t *out_hash,
                                  uint32_t *out_pos, uint32_t *out_read,
                                  uint64_t cap, uint64_t *read_offsets) {
    if (!check_args(k, w, flags)) return -1;
    uint64_t count = 0;
    for (uint32_t r = 0; r < nreads; ++r) {
        if (offsets[r + 1] < offsets[r]) return -1;
        read_offsets[r] = count;
        int rc = deque_windows(seqs + offsets[r], offsets[r + 1] - offsets[r], k, w,
                               flags, out_hash, out_pos, out_read, r, cap, &count);
        if (rc) return rc;
    }
    read_offsets[nreads] = count;
    return (long long)count;
}

/* Element-wise mix64 (inverse = 0) or its inverse (inverse = 1) over an array. */
void oracle_mix64_array(const uint64_t *x, uint64_t n, int inverse, uint64_t *y) {
    for (uint64_t i = 0; i < n; ++i) y[i] = inverse ? oracle_mix64_inv(x[i]) : oracle_mix64(x[i]);
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.4 / Fig. 1: seed pointer table and seed position table.          */
/* ---------------------------------------------------------------------- */

/* Entries i = 0 .. count-1 are (hash[i], pos[i]) in input order; their key is
 * (hash[i] >> shift) mod 2^bits.  Writes ptr[0 .. 2^bits] (ptr[j] = entries
 * with key < j), and pos_out / hash_out (hash_out may be NULL) with the
 * entries grouped by key, ascending, each group in input order.  Returns 0,
 * or -1 for bits outside 1..32, shift + bits > 64, or a failed allocation. */
int oracle_seed_table(const uint64_t *hash, const uint32_t *pos, uint64_t count,
                      uint32_t bits, uint32_t shift, uint64_t *ptr, uint32_t *pos_out,
                      uint64_t *hash_out) {
    if (bits < 1 || bits > 32 || shift + bits > 64) return -1;
    const uint64_t nkeys = 1ull << bits;
    const uint64_t mask = nkeys - 1;
    uint64_t *next = (uint64_t *)calloc(nkeys, sizeof(uint64_t));
    if (!next) return -1;
    /* counts per key */
    for (uint64_t i = 0; i < count; ++i) next[(hash[i] >> shift) & mask] += 1;
    /* ptr[j] = sum of the counts of keys below j */
    uint64_t run = 0;
    for (uint64_t j = 0; j < nkeys; ++j) {
        ptr[j] = run;
        run += next[j];
        next[j] = ptr[j]; /* where the next entry of key j goes */
    }
    ptr[nkeys] = run;
    /* entries in input order, each to the next free slot of its key */
    for (uint64_t i = 0; i < count; ++i) {
        const uint64_t j = (hash[i] >> shift) & mask;
        pos_out[next[j]] = pos[i];
        if (hash_out) hash_out[next[j]] = hash[i];
        next[j] += 1;
    }
    free(next);
    return 0;
}
