// genome.hip -- 2-bit packing, k-mers and minimizer seeds (Sec. 2.4, Fig. 2)
// on gfx950.
//
// Sec. 2.4 reads k-mers as a sliding sum of bases under concatenation and a
// minimizer table as a sliding minimum over k-mers.  One fused pass per tile
// does every step with no intermediate array in HBM:
//
//   1. stage the tile's bases in LDS as 2-bit codes plus an invalid bit
//      (from ASCII or from the packed layout);
//   2. each lane forms the k-mers of its 16 positions: the forward value by
//      the shift-or recurrence f_{i+1} = (f_i << 2 | c_{i+k}) mod 4^k (the
//      sliding concatenation), the reverse complement by the mirrored
//      recurrence, the canonical k-mer as the smaller, then mix64;
//      validity of every k-mer is an OR over k invalid bits, done by doubling
//      with two overlapping halves (the idempotent case of Sec. 3.1 on bits);
//   3. the sliding minimum over w keys (value, position): the block
//      prefix/suffix scheme of the sliding-sum kernels with the
//      "leftmost minimum" operator, which is associative;
//   4. a window's minimizer is stored iff it exists and its position differs
//      from the previous window's (same position <=> same pair);
//   5. ordered compaction: a scan of the per-lane store counts, then a
//      decoupled look-back over the tiles (tile order = workgroup order, so a
//      tile only waits for tiles of workgroups dispatched before its own),
//      then coalesced stores from an LDS staging area.
//
// Tile geometry: 16 positions per lane, P = 16 * NT key positions per tile
// starting at K0 = p0 - 16, where p0 (a multiple of 16) is the first window
// the tile stores; it owns windows [p0, p0 + TW).  The 16 extra keys give
// the window before p0, whose minimizer the dedup test needs.
#include "sws_device.hpp"
#include "sws_internal.hpp"
#include "sws_scan.hpp"

#include <mutex>

namespace sws {

constexpr int kR = 16;                    // positions per lane
constexpr uint32_t kInvalidTag = 0x8000u; // tag bit: key of an invalid k-mer

// ---------------------------------------------------------------------------
// Bases.
// ---------------------------------------------------------------------------

// A/a=0 C/c=1 G/g=2 T/t=3: bits 1..2 of the byte, xor-folded.
__device__ __forceinline__ uint32_t base_code(uint32_t b) { return ((b >> 1) ^ (b >> 2)) & 3u; }
__device__ __forceinline__ bool base_valid(uint32_t b) {
    const uint32_t u = b & 0xDFu;
    return u == 'A' || u == 'C' || u == 'G' || u == 'T';
}

// Four ASCII bytes at once.  c: per byte, the code (bits 1..2 of the byte,
// xor-folded) in bits 0..1.  d: per byte, the upper-cased byte xor
// "ACGT"[code] (one byte permute builds the expected bytes), zero exactly for
// a base letter.
__device__ __forceinline__ void ascii4_parts(uint32_t x, uint32_t& c, uint32_t& d) {
    c = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
    d = (x & 0xDFDFDFDFu) ^ __builtin_amdgcn_perm(0u, 0x54474341u, c);  // 'T' 'G' 'C' 'A'
}

// 0x80 in every byte of d that is not zero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t d) {
    return (((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u;
}

// The four 2-bit codes of c, byte i's at bits 31 - 2i .. 30 - 2i of the
// product (first byte highest): the multiplier's terms 2^30, 2^20, 2^10, 2^0
// move byte i's code (at bit 8i) to bit 30 - 2i, and every other partial
// product lands in bits 0..21 or past bit 31 without overlapping another, so
// no carry reaches bits 24..31.
__device__ __forceinline__ uint32_t codes4_high(uint32_t c) { return c * 0x40100401u; }

// Bit i (i = 0..3) set when byte i of the nonzero_bytes mask z is: after the
// shift byte i's flag sits at bit 8i, and the multiplier's terms 2^21, 2^14,
// 2^7, 2^0 move it to bit 21 + i; every other partial product lands in bits
// 0..16, 29..31 or past bit 31, none overlapping another.
__device__ __forceinline__ uint32_t invalid4(uint32_t z) {
    return (((z >> 7) * 0x00204081u) >> 21) & 0xFu;
}

// 16 bases held as 16 bytes: the code word (first base in bits 31..30) and 16
// invalid bits (bit i = byte i).  Invalid bytes get code 0.  A lane whose 16
// bytes are all base letters skips the invalid bookkeeping.
__device__ __forceinline__ void ascii16_bytes(const uint4& q, uint32_t& code, uint32_t& inv) {
    uint32_t c0, c1, c2, c3, d0, d1, d2, d3;
    ascii4_parts(q.x, c0, d0);
    ascii4_parts(q.y, c1, d1);
    ascii4_parts(q.z, c2, d2);
    ascii4_parts(q.w, c3, d3);
    inv = 0;
    if ((d0 | d1 | d2 | d3) != 0u) {
        const uint32_t z0 = nonzero_bytes(d0), z1 = nonzero_bytes(d1);
        const uint32_t z2 = nonzero_bytes(d2), z3 = nonzero_bytes(d3);
        inv = invalid4(z0) | (invalid4(z1) << 4) | (invalid4(z2) << 8) | (invalid4(z3) << 12);
        // 0x03 in each invalid byte: clear its code
        c0 &= ~((z0 >> 6) | (z0 >> 7));
        c1 &= ~((z1 >> 6) | (z1 >> 7));
        c2 &= ~((z2 >> 6) | (z2 >> 7));
        c3 &= ~((z3 >> 6) | (z3 >> 7));
    }
    // bits 31..24 of each product, bytes 0..3 of the code word from the top
    const uint32_t p0 = codes4_high(c0), p1 = codes4_high(c1);
    const uint32_t p2 = codes4_high(c2), p3 = codes4_high(c3);
    code = __builtin_amdgcn_perm(p0, p1, 0x07030C0Cu) | __builtin_amdgcn_perm(p2, p3, 0x0C0C0703u);
}

// 16 bases starting at `base` (may be negative or run past n): the code word
// (first base in bits 31..30) and 16 invalid bits (bit i = base + i).  Bases
// outside [0, n) are invalid with code 0.  Invalid bases get code 0.
__device__ __forceinline__ void ascii16(const uint8_t* __restrict__ seq, int64_t base, uint64_t n,
                                        bool aligned, uint32_t& code, uint32_t& inv) {
    if (aligned && base >= 0 && (uint64_t)base + 16 <= n) {
        // one 16-byte load, four bytes per operation
        ascii16_bytes(*reinterpret_cast<const uint4*>(seq + base), code, inv);
        return;
    }
    uint32_t word[4];
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int64_t g = base + i * 4 + b;
                const uint32_t byte = (g >= 0 && (uint64_t)g < n) ? (uint32_t)seq[g] : 0u;
                v |= byte << (8 * b);
            }
            word[i] = v;
        }
    }
    code = 0;
    inv = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t b = (word[i >> 2] >> (8 * (i & 3))) & 0xFFu;
        const bool ok = base_valid(b);
        code |= (ok ? base_code(b) : 0u) << (30 - 2 * i);
        inv |= (ok ? 0u : 1u) << i;
    }
}

// The same 16 bases from the packed layout (base a multiple of 16).
__device__ __forceinline__ void packed16(const uint32_t* __restrict__ packed,
                                         const uint32_t* __restrict__ invalid, int64_t base,
                                         uint64_t n, uint32_t& code, uint32_t& inv) {
    if (base < 0 || (uint64_t)base >= n) {
        code = 0;
        inv = 0xFFFFu;
        return;
    }
    const uint64_t wi = (uint64_t)base >> 4;
    code = packed[wi];
    inv = invalid ? (invalid[wi >> 1] >> (16 * (wi & 1))) & 0xFFFFu : 0u;
    const uint64_t left = n - (uint64_t)base;
    if (left < 16) {
        inv |= (0xFFFFu << left) & 0xFFFFu;
        code &= ~(0xFFFFFFFFu >> (2 * left));
    }
}

// ---------------------------------------------------------------------------
// Hash.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 32;
    x *= 0x9E3779B97F4A7C15ull;
    x ^= x >> 29;
    x *= 0x243F6A8885A308D3ull;
    x ^= x >> 32;
    return x;
}

// mix64 of a value below 2^32 (k <= 16), in 32-bit pieces: the first
// xor-shift is the identity, and the first product is one 32 x 32 -> 64
// multiply by the constant's low word plus one low multiply by its high word.
__device__ __forceinline__ uint64_t mix64_u32(uint32_t x) {
    const uint64_t p = (uint64_t)x * 0x7F4A7C15ull;
    const uint32_t hi = (uint32_t)(p >> 32) + x * 0x9E3779B9u;
    uint64_t y = ((uint64_t)hi << 32) | (uint32_t)p;
    y ^= y >> 29;
    y *= 0x243F6A8885A308D3ull;
    y ^= y >> 32;
    return y;
}

__device__ __forceinline__ uint32_t revpairs32(uint32_t x) {
    x = __builtin_bitreverse32(x);
    return ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);
}
__device__ __forceinline__ uint64_t revpairs64(uint64_t x) {
    x = __builtin_bitreverse64(x);
    return ((x >> 1) & 0x5555555555555555ull) | ((x & 0x5555555555555555ull) << 1);
}

// k-mer values (canonical or forward, hashed or not) of the 16 positions of
// lane t, from the LDS code/invalid words t, t+1, t+2.  bad: bit e set iff the
// k-mer at position e covers an invalid base.  clean (wave-uniform): no base
// the wave staged is invalid, so bad is 0 without looking.
template <bool KM64, int FLAGS = -1>
__device__ __forceinline__ void lane_kmers(const uint32_t* s_code, const uint32_t* s_inv, int t,
                                           uint32_t k, bool canon_rt, bool hashed_rt, bool clean,
                                           uint64_t (&val)[kR], uint32_t& bad) {
    // FLAGS >= 0 fixes the flags at compile time (bit 0 forward, bit 1 identity)
    const bool canon = FLAGS >= 0 ? (FLAGS & 1) == 0 : canon_rt;
    const bool hashed = FLAGS >= 0 ? (FLAGS & 2) == 0 : hashed_rt;
    const uint32_t w0 = s_code[t], w1 = s_code[t + 1], w2 = s_code[t + 2];
    bad = 0;
    if (!clean) {
        const uint64_t M = (uint64_t)s_inv[t] | ((uint64_t)s_inv[t + 1] << 16) |
                           ((uint64_t)s_inv[t + 2] << 32);
        uint64_t A = M;
        uint32_t len = 1;
        while (2u * len <= k) {
            A |= A >> len;
            len *= 2u;
        }
        bad = (uint32_t)((A | (A >> (k - len))) & 0xFFFFu);
    }

    const uint64_t hi = ((uint64_t)w0 << 32) | w1;
    if (KM64) {
        // The 48 bases of words t .. t + 2 hold every k-mer of the run (bases
        // e .. e + k - 1 <= 45).  The 64 bits from base e on, shifted right by
        // 64 - 2k, are k-mer e's forward value; in R2:R1:R0, the reverse
        // complement of all 48 bases (base i complemented at bits 2i + 1 ..
        // 2i), its reverse complement is the 2k bits from bit 2e.  Funnel
        // shifts by constants, no recurrence between positions.
        const uint32_t R0 = revpairs32(~w0), R1 = revpairs32(~w1), R2 = revpairs32(~w2);
        const uint32_t mhi = (1u << (2u * k - 32u)) - 1u;  // k >= 17
        const uint32_t fsh = 64u - 2u * k;
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const uint32_t uh = e == 0 ? w0 : __builtin_amdgcn_alignbit(w0, w1, 32 - 2 * e);
            const uint32_t ul = e == 0 ? w1 : __builtin_amdgcn_alignbit(w1, w2, 32 - 2 * e);
            const uint64_t fwd = (((uint64_t)uh << 32) | ul) >> fsh;
            const uint32_t rl = e == 0 ? R0 : __builtin_amdgcn_alignbit(R1, R0, 2 * e);
            const uint32_t rh = (e == 0 ? R1 : __builtin_amdgcn_alignbit(R2, R1, 2 * e)) & mhi;
            const uint64_t rc = ((uint64_t)rh << 32) | rl;
            const uint64_t cv = (canon && rc < fwd) ? rc : fwd;
            val[e] = hashed ? mix64(cv) : cv;
        }
    } else {
        // The 32 bases of words t, t + 1 hold every k-mer of the run (bases
        // e .. e + k - 1 <= 30).  In G = hi >> (34 - 2k) k-mer e's forward
        // value is the 2k bits from bit 30 - 2e; in R, the reverse complement
        // of all 32 bases (base i complemented at bits 2i + 1 .. 2i), k-mer
        // e's reverse complement is the 2k bits from bit 2e.  Each is one
        // funnel shift and a mask, with no recurrence between positions.
        const uint32_t mask = k == 16u ? 0xFFFFFFFFu : ((1u << (2u * k)) - 1u);
        const uint64_t G = hi >> (34u - 2u * k);
        const uint64_t R = revpairs64(~hi);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const uint32_t fwd = (uint32_t)(G >> (30 - 2 * e)) & mask;
            const uint32_t rc = (uint32_t)(R >> (2 * e)) & mask;
            const uint32_t cv = (canon && rc < fwd) ? rc : fwd;
            val[e] = hashed ? mix64_u32(cv) : (uint64_t)cv;
        }
    }
}

// Stage the code/invalid words of bases [K0, K0 + 16 * nw) into LDS.
template <int IN>
__device__ __forceinline__ void stage_bases(const GenomeInput& in, int64_t K0, int nw,
                                            uint32_t* s_code, uint32_t* s_inv, int tid, int nt) {
    for (int i = tid; i < nw; i += nt) {
        uint32_t code, inv;
        const int64_t base = K0 + 16 * (int64_t)i;
        if (IN == kInAscii) ascii16(in.seq, base, in.n, in.aligned != 0, code, inv);
        else packed16(in.packed, in.invalid, base, in.n, code, inv);
        s_code[i] = code;
        s_inv[i] = inv;
    }
}

// The 16-base word of a lane in a wavefront tile, split in two phases so
// that the global load of the next tile can be in flight while the current
// one is computed: `fetch` issues the load into registers, `commit` converts
// and stores it into LDS.  Lane l holds the tile's word l.
struct RawWords {
    uint4 a;  // ASCII: 16 bytes; 2-bit: .x code word, .y invalid bits
};

template <int IN>
__device__ __forceinline__ void fetch_words(const GenomeInput& in, int64_t K0, int lane,
                                            RawWords& r) {
    const int64_t b0 = K0 + 16 * (int64_t)lane;
    if (IN == kInAscii) {
        const bool fast0 = in.aligned && b0 >= 0 && (uint64_t)b0 + 16 <= in.n;
        r.a = fast0 ? *reinterpret_cast<const uint4*>(in.seq + b0) : make_uint4(0, 0, 0, 0);
    } else {
        uint32_t c, v;
        packed16(in.packed, in.invalid, b0, in.n, c, v);
        r.a = make_uint4(c, v, 0, 0);
    }
}

__device__ __forceinline__ void ascii_word(const GenomeInput& in, int64_t base, const uint4& q,
                                           uint32_t& code, uint32_t& inv) {
    if (in.aligned && base >= 0 && (uint64_t)base + 16 <= in.n) {
        ascii16_bytes(q, code, inv);
    } else {
        ascii16(in.seq, base, in.n, false, code, inv);  // edges and unaligned input
    }
}

// Returns the word's invalid bits.
template <int IN>
__device__ __forceinline__ uint32_t commit_words(const GenomeInput& in, int64_t K0, int lane,
                                                 const RawWords& r, uint32_t* code, uint32_t* inv) {
    uint32_t c = r.a.x, v = r.a.y;
    if (IN == kInAscii) ascii_word(in, K0 + 16 * (int64_t)lane, r.a, c, v);
    code[lane] = c;
    inv[lane] = v;
    return v;
}

// ---------------------------------------------------------------------------
// pack2bit: one lane per 16 bases.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack2bit_kernel(const uint8_t* __restrict__ seq, uint64_t n,
                                                       uint32_t* __restrict__ packed,
                                                       uint32_t* __restrict__ invalid, int aligned,
                                                       uint64_t nwords) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t code = 0, inv = 0;
    if (i < nwords) {
        ascii16(seq, (int64_t)(i * 16), n, aligned != 0, code, inv);
        const uint64_t left = n - i * 16;
        if (left < 16) inv &= (1u << left) - 1u;  // bits past n are zero
        packed[i] = code;
    }
    const int lane = lane_id();
    const uint32_t other = shfl(inv, lane, 1);
    if (invalid && i < nwords && (i & 1) == 0) invalid[i >> 1] = inv | (other << 16);
}

// ---------------------------------------------------------------------------
// kmers: one tile of 16 * NT positions per workgroup.  The tile's bases are
// staged in LDS as 16-base words; thread t then forms the k-mers at tile
// positions t, t + NT, t + 2 NT, ... each from the two words it spans (three
// for k > 16), so that every store instruction writes 64 consecutive values
// straight from registers.
// ---------------------------------------------------------------------------
// LDS index with one pad word per 16 (runs of 16 per thread, conflict-free).
__device__ __forceinline__ uint32_t pad16(uint32_t i) { return i + (i >> 4); }

// The k-mer value (canonical or forward, hashed or not; all ones when it
// covers an invalid base) at tile position q, from the staged words.
template <bool KM64>
__device__ __forceinline__ uint64_t kmer_at(const uint32_t* s_code, const uint32_t* s_inv,
                                            uint32_t q, uint32_t k, bool canon, bool hashed) {
    const uint32_t j = q >> 4, r = q & 15u;  // word, base within it
    uint64_t cv;
    bool bad;
    if (KM64) {  // bases r .. r + k - 1 <= 46 of words j, j + 1, j + 2
        const uint64_t hi = ((uint64_t)s_code[j] << 32) | s_code[j + 1];
        const uint64_t win = r == 0u ? hi : (hi << (2u * r)) | (s_code[j + 2] >> (32u - 2u * r));
        const uint64_t fwd = win >> (64u - 2u * k);
        const uint64_t rc = revpairs64(~fwd) >> (64u - 2u * k);
        cv = (canon && rc < fwd) ? rc : fwd;
        const uint64_t M = (uint64_t)s_inv[j] | ((uint64_t)s_inv[j + 1] << 16) |
                           ((uint64_t)s_inv[j + 2] << 32);
        bad = ((M >> r) & ((2ull << (k - 1u)) - 1ull)) != 0ull;
    } else {  // bases r .. r + k - 1 <= 30 of words j, j + 1
        const uint64_t pair = ((uint64_t)s_code[j] << 32) | s_code[j + 1];
        const uint32_t fwd = (uint32_t)((pair << (2u * r)) >> (64u - 2u * k));
        const uint32_t rc = revpairs32(~fwd) >> (32u - 2u * k);
        cv = (canon && rc < fwd) ? rc : fwd;
        const uint32_t M = s_inv[j] | (s_inv[j + 1] << 16);
        bad = ((M >> r) & ((1u << k) - 1u)) != 0u;
    }
    return bad ? ~0ull : (hashed ? mix64(cv) : cv);
}

// PAIRS (out 16-byte aligned): a thread forms two neighbouring k-mers and
// writes them with one 16-byte store.  The stores are nontemporal: the output
// is written once and not read back by this kernel, and streaming it past the
// caches measured 0.66 of the plain stores' time.
template <int NT, int IN, bool KM64, bool PAIRS>
__global__ __launch_bounds__(NT) void kmers_kernel(GenomeInput in, uint32_t k, uint32_t flags,
                                                   uint64_t nk, uint64_t* __restrict__ out) {
    constexpr int P = NT * kR;
    constexpr int NW = NT + 2;  // the tile's P bases and the (k - 1)-base tail
    __shared__ uint32_t s_code[NW], s_inv[NW];
    const int tid = (int)threadIdx.x;
    const int64_t K0 = (int64_t)blockIdx.x * P;
    stage_bases<IN>(in, K0, NW, s_code, s_inv, tid, NT);
    __syncthreads();
    const bool canon = (flags & 1u) == 0u, hashed = (flags & 2u) == 0u;
    if (PAIRS) {
        typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < kR / 2; ++i) {
            const uint32_t q = 2u * (uint32_t)(i * NT + tid);  // tile position, even
            const uint64_t g = (uint64_t)K0 + q;
            if (g >= nk) break;
            u64x2 v;
            v.x = kmer_at<KM64>(s_code, s_inv, q, k, canon, hashed);
            v.y = kmer_at<KM64>(s_code, s_inv, q + 1u, k, canon, hashed);
            if (g + 1 < nk) __builtin_nontemporal_store(v, (u64x2*)(out + g));
            else __builtin_nontemporal_store(v.x, out + g);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kR; ++i) {
            const uint32_t q = (uint32_t)(i * NT + tid);  // tile position
            const uint64_t g = (uint64_t)K0 + q;
            if (g >= nk) break;
            __builtin_nontemporal_store(kmer_at<KM64>(s_code, s_inv, q, k, canon, hashed), out + g);
        }
    }
}

// ---------------------------------------------------------------------------
// Minimizers.
// ---------------------------------------------------------------------------

// Leftmost minimum of keys.  FULL compares (value, tag) -- needed only when a
// valid key may carry the all-ones value (hashed k >= 30); otherwise values
// alone decide, and ties keep the left (earlier) operand.
template <bool FULL>
struct OpKeyMin {
    using T = Key;
    static __device__ __forceinline__ Key identity() {
        Key r;
        r.lo = 0xFFFFFFFFu;
        r.hi = 0xFFFFFFFFu;
        r.tag = 0xFFFFu;
        return r;
    }
    static __device__ __forceinline__ bool less(const Key& a, const Key& b) {
        const uint64_t ha = ((uint64_t)a.hi << 32) | a.lo;
        const uint64_t hb = ((uint64_t)b.hi << 32) | b.lo;
        if (FULL) return ha < hb || (ha == hb && a.tag < b.tag);
        return ha < hb;
    }
    static __device__ __forceinline__ Key combine(Key l, Key r) { return less(r, l) ? r : l; }
};


__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t lo = shfl((uint32_t)v, lane, d);
        const uint32_t hi = shfl((uint32_t)(v >> 32), lane, d);
        v += ((uint64_t)hi << 32) | lo;  // lanes past 63 wrap; lane 0 ends with the total
    }
    return v;
}

// Exclusive prefix of a look-back participant's store count over the
// participants before it (decoupled look-back, one wavefront).  Each first
// publishes its own count (AGGREGATE), then reads the status words of the LB
// (<= 64) participants before it in one round: if every one back to the
// nearest with an INCLUSIVE prefix has published, their counts plus that
// prefix give the answer; otherwise it waits and re-reads.  Without an
// INCLUSIVE word among the LB it moves LB further back.  Called by all 64
// lanes of one wave; returns the prefix in every lane.
//
// A status word is flag (2 bits: AGGREGATE 1, INCLUSIVE 2) | epoch (30 bits) |
// count (32 bits); a word whose epoch is not this call's reads as unpublished,
// so a workspace needs no clearing between calls (the epoch of the last call
// sits in the workspace header; a zero-filled header starts at epoch 1).
//
// Status words sit one per 64-byte line (kStatusStride words apart): the
// words of neighbouring participants are written and polled by different
// compute units at device scope, and sharing a line serializes those
// accesses.  The status traffic and the distance to the nearest INCLUSIVE
// word both grow with the number of participants, so the w <= 32 path makes
// a workgroup of wave tiles one participant.
constexpr uint32_t kEpochMask = (1u << 30) - 1u;

// This call's epoch, from the last call's (1 .. 2^30 - 1; never 0, so that a
// zero-filled error word never matches it).
__device__ __forceinline__ uint32_t call_epoch(const uint64_t* epoch_word) {
    return (uint32_t)(*epoch_word % kEpochMask) + 1u;
}

template <int LB = kWave>
__device__ uint64_t tile_lookback(uint64_t* status, uint64_t tile, uint64_t total, uint32_t* err,
                                  uint32_t epoch, int lane) {
    const uint64_t kAgg = 1ull << 62, kInc = 2ull << 62, kVal = 0xFFFFFFFFull;
    const uint64_t tag = (uint64_t)epoch << 32;
    if (tile == 0) {
        if (lane == 0)
            __hip_atomic_store(&status[0], kInc | tag | total, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (lane == 0)
        __hip_atomic_store(&status[tile * kStatusStride], kAgg | tag | total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;
    uint32_t spins = 0;
    // LB predecessors per round.  The narrower window suits the batched
    // kernel (0.497 against 0.531 ms at 32); the single-sequence kernel is
    // faster with all 64 (0.1715 against 0.1778 ms at 32).
    const uint64_t win = LB >= kWave ? ~0ull : ((1ull << LB) - 1ull);
    for (;;) {
        const int64_t j = base - lane;
        // before participant 0 there is nothing: read as an INCLUSIVE prefix of 0
        uint64_t s = 0;
        if (lane < LB)
            s = j >= 0 ? __hip_atomic_load(&status[(uint64_t)j * kStatusStride],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : kInc | tag;
        // a word of another call's epoch has not been published in this one
        const uint64_t f = ((s >> 32) & kEpochMask) == epoch ? s >> 62 : 0ull;
        const uint64_t inc = __ballot(f == 2) & win;
        const uint64_t notready = __ballot(f == 0) & win;
        const int first = inc ? __builtin_ctzll(inc) : LB;  // nearest INCLUSIVE lane
        const uint64_t need = first >= LB - 1 ? win : ((2ull << first) - 1ull);
        if (notready & need) {
            // Bounded wait: a predecessor that never publishes (which a correct
            // launch cannot produce) flags an error instead of hanging.
            if (++spins > (1u << 20)) {
                if (lane == 0)
                    __hip_atomic_store(err, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        const uint64_t mine = lane <= first && lane < LB ? (s & kVal) : 0ull;
        excl += lane_value_u64(wave_sum_u64(mine, lane), 0);
        if (first < LB) break;
        base -= LB;
    }
    if (lane == 0)
        __hip_atomic_store(&status[tile * kStatusStride], kInc | tag | (excl + total),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return excl;
}

// The count the last tile reports: the total, or all ones if some tile of
// this call gave up waiting for a predecessor (an internal error the caller
// must see).  The last tile also records the call's epoch: every tile read the
// old one before it published, and the last tile has seen every publication.
__device__ __forceinline__ uint64_t final_count(uint32_t* err, uint64_t* epoch_word,
                                                uint32_t epoch, uint64_t total) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool failed = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
    *epoch_word = epoch;
    return failed ? ~0ull : total;
}

template <int NT, int IN, bool KM64, bool FULL>
__global__ __launch_bounds__(NT) void minimizer_kernel(GenomeInput in, MinimizerArgs a) {
    using Op = OpKeyMin<FULL>;
    constexpr int P = NT * kR;
    constexpr int NW = NT + 2;
    constexpr int NWV = NT / kWave;
    constexpr uint32_t WS = kWave * kR;  // keys per wave
    __shared__ uint32_t s_code[NW], s_inv[NW];
    __shared__ uint64_t s_h[P + P / 16];   // prefix minima, later the staged output values
    __shared__ uint16_t s_tag[P + P / 16]; // their tags, later the staged output positions
    __shared__ Key s_carryF[NWV], s_carryB[NWV];
    __shared__ uint32_t s_lastTag[NWV];
    __shared__ uint32_t s_wsum[NWV];
    __shared__ uint64_t s_excl;

    const int tid = (int)threadIdx.x;
    const int lane = lane_id();
    const int wv = tid >> 6;
    const uint32_t w = a.w;

    // tile order = workgroup order (see minimizer_wave_kernel)
    const uint64_t tile = blockIdx.x;
    const int64_t p0 = (int64_t)(tile * a.tw);
    const int64_t K0 = p0 - 16;

    // 1. bases
    stage_bases<IN>(in, K0, NW, s_code, s_inv, tid, NT);
    __syncthreads();

    // 2. keys
    Key pf[kR], sf[kR];
    {
        uint64_t val[kR];
        uint32_t bad;
        lane_kmers<KM64>(s_code, s_inv, tid, a.k, (a.flags & 1u) == 0u, (a.flags & 2u) == 0u, false, val,
                         bad);
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const uint32_t j = (uint32_t)tid * kR + e;
            const bool inv = (bad >> e) & 1u;
            pf[e].lo = inv ? 0xFFFFFFFFu : (uint32_t)val[e];
            pf[e].hi = inv ? 0xFFFFFFFFu : (uint32_t)(val[e] >> 32);
            pf[e].tag = j | (inv ? kInvalidTag : 0u);
            sf[e] = pf[e];
        }
    }

    // 3. sliding minimum: in-segment prefix/suffix minima, segments of w keys
    //    aligned to multiples of w inside the tile
    const uint32_t span = (w + kR - 1) / kR;
    const uint32_t m0 = ((uint32_t)tid * kR) % w;
    const HeadMask<kR> heads = lane_heads<kR>(m0, w, head_pattern<kR>(w));
    slab_prefix<Op, kR>(pf, heads, span, lane, Op::identity());
    slab_suffix<Op, kR>(sf, heads, span, lane);
    if (lane == kWave - 1) s_carryF[wv] = pf[kR - 1];
    if (lane == 0) s_carryB[wv] = sf[0];
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        const uint32_t j = (uint32_t)tid * kR + e;
        s_h[pad16(j)] = ((uint64_t)pf[e].hi << 32) | pf[e].lo;
        s_tag[pad16(j)] = (uint16_t)pf[e].tag;
    }
    __syncthreads();
    // the wave's last segment continues into the next wave (w <= keys per wave)
    if (wv < NWV - 1) {
        const uint32_t wend = (uint32_t)(wv + 1) * WS;
        const uint32_t last = (wend - 1u) % w;
        if (last != w - 1u) {
            const Key c = s_carryB[wv + 1];
            const uint32_t head = wend - 1u - last;
#pragma unroll
            for (int e = 0; e < kR; ++e)
                if ((uint32_t)tid * kR + e >= head) sf[e] = Op::combine(sf[e], c);
        }
    }
    uint32_t mtag[kR];
    {
        uint32_t m = m0;
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const uint32_t j = (uint32_t)tid * kR + e;
            const uint32_t q = j + w - 1u;
            Key r;
            if (q < (uint32_t)P) {
                const uint64_t h = s_h[pad16(q)];
                r.lo = (uint32_t)h;
                r.hi = (uint32_t)(h >> 32);
                r.tag = s_tag[pad16(q)];
                // prefix minima of a segment that started in the previous wave
                // a segment that started in the previous wave takes that wave's
                // carried prefix; q mod w = (j - 1) mod w
                const uint32_t qw = q / WS;
                const uint32_t qhead = q - (m == 0u ? w - 1u : m - 1u);
                if (qhead < qw * WS) r = Op::combine(s_carryF[qw - 1], r);
                if (m != 0u) r = Op::combine(sf[e], r);
            } else {
                r = Op::identity();
            }
            // keep the key itself (value in sf) for the output stage
            sf[e] = r;
            mtag[e] = r.tag;
            m = (m + 1u == w) ? 0u : m + 1u;
        }
    }
    if (lane == kWave - 1) s_lastTag[wv] = mtag[kR - 1];
    __syncthreads();

    // 4. dedup: store window p iff it has a minimizer at a new position
    uint32_t emit = 0;
    {
        uint32_t prev = shfl(mtag[kR - 1], lane, -1);
        if (lane == 0) prev = wv > 0 ? s_lastTag[wv - 1] : 0xFFFFFFFFu;
#pragma unroll
        for (int e = 0; e < kR; ++e) {
            const uint32_t j = (uint32_t)tid * kR + e;
            const int64_t p = K0 + (int64_t)j;
            const bool owned = j >= 16u && j < 16u + a.tw && p < (int64_t)a.nwin;
            const bool valid = (mtag[e] & kInvalidTag) == 0u;
            const bool fresh = p == 0 || mtag[e] != prev;
            emit |= (owned && valid && fresh ? 1u : 0u) << e;
            prev = mtag[e];
        }
    }

    // 5. ordered compaction
    const uint32_t cnt = (uint32_t)__builtin_popcount(emit);
    uint32_t incl = wave_inclusive_sum(cnt);
    if (lane == kWave - 1) s_wsum[wv] = incl;
    __syncthreads();  // also: every read of s_h / s_tag above is complete
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int i = 0; i < NWV; ++i) {
        const uint32_t v = s_wsum[i];
        wbase += i < wv ? v : 0u;
        total += v;
    }
    uint32_t slot = wbase + incl - cnt;
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        if ((emit >> e) & 1u) {
            s_h[slot] = ((uint64_t)sf[e].hi << 32) | sf[e].lo;
            s_tag[slot] = (uint16_t)(sf[e].tag & 0x7FFFu);
            ++slot;
        }
    }
    uint32_t epoch = 0;
    if (wv == 0) {
        epoch = call_epoch(a.epoch);
        const uint64_t e = tile_lookback(a.status, tile, total, a.err, epoch, lane);
        if (lane == 0) s_excl = e;
    }
    __syncthreads();
    const uint64_t excl = s_excl;
    for (uint32_t i = (uint32_t)tid; i < total; i += NT) {
        const uint64_t g = excl + i;
        if (g < a.capacity) {
            a.out_hash[g] = s_h[i];
            a.out_pos[g] = (uint32_t)(K0 + (int64_t)s_tag[i]);
        }
    }
    if (tid == 0 && tile == a.ntiles - 1)
        *a.d_count = final_count(a.err, a.epoch, epoch, excl + total);
}

// ---------------------------------------------------------------------------
// Minimizers, one wavefront per tile (w <= 32).
//
// Each wavefront owns a tile of 1024 key positions (16 per lane) and does every
// step alone: no workgroup barrier after the tile id is known.  For w <= 8 the
// window minimum uses the doubling of Sec. 3.1 for an idempotent operator:
// with m^(1) = key, m^(2s)_e = min(m^(s)_e, m^(s)_{e+s}), and 2^L the largest
// power of two not above w, the minimum over [e, e+w) is min(m^(2^L)_e,
// m^(2^L)_{e+w-2^L}) -- the two halves overlap, which min allows.  The levels
// run in registers (a lane takes the s values it needs past its run from the
// next lane).  For 9 <= w <= 32 block prefix/suffix scans over the lanes' runs
// take fewer combines (window_min).  Every min keeps the left operand on
// ties, so the leftmost position wins.
// ---------------------------------------------------------------------------
//
// A wave stages exactly the 1024 bases [K0, K0 + 1024), one 16-base word per
// lane.  The k-mers at positions past 1024 - k would need bases beyond them:
// they read the two LDS words after the tile, which are never written, so
// their keys are unspecified, and the tile owns only windows whose keys all
// start at or below 1024 - k (wave_tile_windows).
constexpr int kWaveKeys = kWave * kR;  // 1024 keys per wave tile
constexpr uint32_t kStage = 512;       // outputs per round of a wave's store compaction
constexpr int kWaveWords = kWaveKeys / 16 + 2;  // the two words past the tile: read, never written

// The value of the next lane (lane 63 reads lane 0) and of the previous lane
// (lane 0 reads lane 63), by the whole-wave DPP rotates: the move runs in the
// VALU instead of a round trip through the LDS crossbar.  Every lane of the
// wave must be active.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x134, 0xF, 0xF, false);  // wave_rol:1
}
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xF, 0xF, false);  // wave_ror:1
}
__device__ __forceinline__ Key from_next_lane(const Key& v) {
    Key r;
    r.lo = from_next_lane(v.lo);
    r.hi = from_next_lane(v.hi);
    r.tag = from_next_lane(v.tag);
    return r;
}

template <bool FULL>
__device__ __forceinline__ Key key_min(const Key& l, const Key& r) {
    return OpKeyMin<FULL>::combine(l, r);
}

// One doubling step in registers: m[e] = min(m[e], m[e + S]); a lane reads
// m[e + S] past its run from the next lane (values taken before any update).
template <int S, bool FULL>
__device__ __forceinline__ void doubling_step(Key (&m)[kR]) {
    Key nb[S];
#pragma unroll
    for (int t = 0; t < S; ++t) nb[t] = from_next_lane(m[t]);
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        const Key r = (e + S < kR) ? m[e + S] : nb[e + S - kR];
        m[e] = key_min<FULL>(m[e], r);
    }
}

// The last step shifts by w - 2^L, known only at run time: a uniform switch
// over the possible values (w <= 8: at most 3) keeps every register index
// static.
template <bool FULL>
__device__ __forceinline__ void doubling_shift(Key (&m)[kR], uint32_t shift) {
    switch (shift) {
    case 1: doubling_step<1, FULL>(m); break;
    case 2: doubling_step<2, FULL>(m); break;
    case 3: doubling_step<3, FULL>(m); break;
    default: break;
    }
}

// Windows of 9 to 32 keys: the block prefix/suffix scheme of Sec. 2.2, with
// each lane's run of 16 keys as a block.  A window that leaves the run is a
// suffix of the run combined with a prefix of the next run (w <= 17), or with
// the whole next run and a prefix of the one after (w > 17); a window inside
// the run (w <= 16) crosses its middle, so it is a suffix of the first half
// combined with a prefix of the second.  Per position this takes about 3
// combines where the doubling takes ceil(log2 w) (4 at w = 10, 5 at w = 19).
// Every combine keeps the earlier keys on the left, so ties still go to the
// leftmost position.
//
// Order of work, to keep few keys live: the prefixes first (the previous lane
// takes them as they form), then the suffixes from the end of the run, each
// output written in place as soon as its suffix exists.
template <int W, bool FULL>
__device__ __forceinline__ void window_min_runs(Key (&m)[kR]) {
    static_assert(W >= 9 && W <= 32, "windows of 9 to 32 keys");
    if (W <= 16) {
        Key pn[W - 1];  // the next run's prefixes: keys 0 .. j, j <= W - 2
        Key pb[8];      // this run's keys 8 .. 8 + i
        Key p = m[0];
        pn[0] = from_next_lane(p);
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            p = key_min<FULL>(p, m[j]);
            if (j <= W - 2) pn[j] = from_next_lane(p);
        }
        pb[0] = m[8];
#pragma unroll
        for (int i = 1; i < 8; ++i) pb[i] = key_min<FULL>(pb[i - 1], m[8 + i]);
#pragma unroll
        for (int j = 8; j <= W - 2; ++j) pn[j] = from_next_lane(key_min<FULL>(p, pb[j - 8]));
        // windows e >= 17 - W leave the run: keys e .. 15, then the next
        // run's keys 0 .. e + W - 17
        Key sb = m[15];
        m[15] = key_min<FULL>(sb, pn[W - 2]);
#pragma unroll
        for (int e = 14; e >= 8; --e) {
            sb = key_min<FULL>(m[e], sb);
            m[e] = key_min<FULL>(sb, pn[e + W - 17]);
        }
        // sb: keys 8 .. 15.  Windows e <= 16 - W (e <= 7) stay in the run:
        // keys e .. 7, then keys 8 .. e + W - 1.
        Key sa = m[7];
#pragma unroll
        for (int e = 7; e >= 0; --e) {
            if (e < 7) sa = key_min<FULL>(m[e], sa);
            if (e >= 17 - W) m[e] = key_min<FULL>(key_min<FULL>(sa, sb), pn[e + W - 17]);
            else m[e] = key_min<FULL>(sa, pb[e + W - 9]);
        }
    } else {
        constexpr int NN = W > 17 ? W - 17 : 1;
        Key pn[kR];   // the next run's prefixes: keys 0 .. j
        Key pnn[NN];  // the prefixes of the run after next, j <= W - 18
        Key p = m[0];
        pn[0] = from_next_lane(p);
#pragma unroll
        for (int j = 1; j < kR; ++j) {
            p = key_min<FULL>(p, m[j]);
            pn[j] = from_next_lane(p);
        }
#pragma unroll
        for (int j = 0; j < W - 17; ++j) pnn[j] = from_next_lane(pn[j]);
        // window e: keys e .. 15, the next run's keys 0 .. e + W - 17 (all
        // 16 of them when e + W - 17 > 15, then the run after next's keys
        // 0 .. e + W - 33)
        Key sfx = m[kR - 1];
#pragma unroll
        for (int e = kR - 1; e >= 0; --e) {
            if (e < kR - 1) sfx = key_min<FULL>(m[e], sfx);
            if (e <= 32 - W) m[e] = key_min<FULL>(sfx, pn[e + W - 17]);
            else m[e] = key_min<FULL>(key_min<FULL>(sfx, pn[kR - 1]), pnn[e + W - 33]);
        }
    }
}

// The minimum of every window of w keys (1 <= w <= 32) starting in the run,
// in place: doubling for w <= 8, runs for larger w (a uniform switch keeps
// every register index static).
template <bool FULL>
__device__ __forceinline__ void window_min(Key (&m)[kR], uint32_t w) {
    if (w <= 8u) {
        uint32_t L = 1;
        if (2u <= w) { doubling_step<1, FULL>(m); L = 2; }
        if (4u <= w) { doubling_step<2, FULL>(m); L = 4; }
        if (8u <= w) { doubling_step<4, FULL>(m); L = 8; }
        doubling_shift<FULL>(m, w - L);  // 0 <= w - L < L <= 8
        return;
    }
    switch (w) {
#define SWS_RUNS_CASE(W) \
    case W: window_min_runs<W, FULL>(m); break;
    SWS_RUNS_CASE(9) SWS_RUNS_CASE(10) SWS_RUNS_CASE(11) SWS_RUNS_CASE(12)
    SWS_RUNS_CASE(13) SWS_RUNS_CASE(14) SWS_RUNS_CASE(15) SWS_RUNS_CASE(16)
    SWS_RUNS_CASE(17) SWS_RUNS_CASE(18) SWS_RUNS_CASE(19) SWS_RUNS_CASE(20)
    SWS_RUNS_CASE(21) SWS_RUNS_CASE(22) SWS_RUNS_CASE(23) SWS_RUNS_CASE(24)
    SWS_RUNS_CASE(25) SWS_RUNS_CASE(26) SWS_RUNS_CASE(27) SWS_RUNS_CASE(28)
    SWS_RUNS_CASE(29) SWS_RUNS_CASE(30) SWS_RUNS_CASE(31) SWS_RUNS_CASE(32)
#undef SWS_RUNS_CASE
    default: break;
    }
}

// Bit e set when window e's minimum sits at another position than window
// e - 1's (window -1: the previous lane's last).  Built from the last window
// down: each step doubles the bits so far and adds the next comparison, so
// window e ends at bit e.
__device__ __forceinline__ uint32_t changed_bits(const Key (&m)[kR]) {
    uint32_t r = 0;
#pragma unroll
    for (int e = kR - 1; e > 0; --e) r = r + r + (m[e].tag != m[e - 1].tag ? 1u : 0u);
    return r + r + (m[0].tag != from_prev_lane(m[kR - 1].tag) ? 1u : 0u);
}

// OR over the `len` bits following each of bits 0..15: bit e of the result is
// set iff some bit in [e+1, e+len] of x is.  len <= 62 - 15.
__device__ __forceinline__ uint32_t or_after(uint64_t x, uint32_t len) {
    if (len == 0) return 0;
    uint64_t A = x >> 1;
    uint32_t l = 1;
    while (2u * l <= len) {
        A |= A >> l;
        l *= 2u;
    }
    return (uint32_t)((A | (A >> (len - l))) & 0xFFFFu);
}

// Invalid k-mer bits of a lane's run and of the next two lanes' runs (bit e:
// k-mer 16 lane + e), enough for every window that starts in the run (w <= 32).
__device__ __forceinline__ uint64_t run_bits3(uint32_t bad) {
    const uint32_t b1 = from_next_lane(bad), b2 = from_next_lane(b1);
    return (uint64_t)bad | ((uint64_t)b1 << 16) | ((uint64_t)b2 << 32);
}

// Split semantics (flag 4): invalid bases cut the sequence into segments and
// a window holding an invalid k-mer stores nothing.  Bit e of the result is
// set when window 16 lane + e (k-mers e .. e + w - 1) holds one.
__device__ __forceinline__ uint32_t window_holds_invalid(uint64_t ext, uint32_t w) {
    return ((uint32_t)ext | or_after(ext, w - 1u)) & 0xFFFFu;
}

// Bit e set when window 16 lane + e has no valid k-mer at all (it stores
// nothing under either semantics).
__device__ __forceinline__ uint32_t window_all_invalid(uint64_t ext, uint32_t w) {
    const uint64_t ok = ~ext;
    return ~((uint32_t)ok | or_after(ok, w - 1u)) & 0xFFFFu;
}

// Bits of the windows 16 lane + e that a tile stores: 16 <= j < hi (uniform).
__device__ __forceinline__ uint32_t owned_bits(int64_t hi, int lane) {
    const int32_t h = (int32_t)(hi < 16 ? 16 : (hi > kWaveKeys ? kWaveKeys : hi));
    const int32_t b = lane * kR;
    const int32_t lo_rel = min(max(16 - b, 0), 16), hi_rel = min(max(h - b, 0), 16);
    return ((1u << hi_rel) - 1u) & ~((1u << lo_rel) - 1u);
}

// Bit e set when the window before window 16 lane + e holds an invalid
// k-mer: the window after such a window is never a duplicate.
__device__ __forceinline__ uint32_t previous_window_bits(uint32_t wbad) {
    return ((wbad << 1) | ((from_prev_lane(wbad) >> 15) & 1u)) & 0xFFFFu;
}

// The keys of a lane's 16 positions: value and tag = tile position.  With
// any_bad (wave-uniform) the k-mers flagged in bad become invalid keys:
// all-ones without FULL (no valid k-mer reaches it, so one never wins), the
// invalid tag bit with FULL.
template <bool FULL>
__device__ __forceinline__ void make_keys(const uint64_t (&val)[kR], uint32_t bad, bool any_bad,
                                          uint32_t tbase, Key (&m)[kR]) {
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        m[e].lo = (uint32_t)val[e];
        m[e].hi = (uint32_t)(val[e] >> 32);
        m[e].tag = tbase + e;
    }
    if (!any_bad) return;
#pragma unroll
    for (int e = 0; e < kR; ++e) {
        if (FULL) {
            const bool iv = (bad >> e) & 1u;
            m[e].lo = iv ? 0xFFFFFFFFu : m[e].lo;
            m[e].hi = iv ? 0xFFFFFFFFu : m[e].hi;
            m[e].tag |= iv ? kInvalidTag : 0u;
        } else {
            const uint32_t ivm = 0u - ((bad >> e) & 1u);
            m[e].lo |= ivm;
            m[e].hi |= ivm;
        }
    }
}

// Both input layouts run 4 waves per SIMD (at most 128 VGPRs; the window
// minimum of w > 8 holds up to 32 keys at once).
template <int NT, int IN, bool KM64, bool FULL, int FLAGS>
__global__ __launch_bounds__(NT) void minimizer_wave_kernel(GenomeInput in, MinimizerArgs a) {
    constexpr int NWV = NT / kWave;
    static_assert(NWV <= kWave, "one lane per wave of the workgroup");
    __shared__ uint32_t s_code[NWV][kWaveWords], s_inv[NWV][kWaveWords];
    __shared__ uint32_t s_cnt[NWV];  // stores per wave tile
    __shared__ uint64_t s_base;      // stores before the workgroup
    __shared__ uint64_t s_stage_hash[NWV][kStage];
    __shared__ uint32_t s_stage_pos[NWV][kStage];

    const int lane = lane_id();
    const int wv = wave_id();
    const uint32_t w = a.w;
    uint32_t* code = s_code[wv];
    uint32_t* inv = s_inv[wv];

    // Tile order = workgroup order.  The workgroup's wave tiles are
    // consecutive; their counts are added in LDS and one wave does the
    // look-back for the workgroup, which waits only for workgroups dispatched
    // before it, so the lowest unfinished one never waits and every one
    // finishes.  (One look-back per workgroup rather than per wave: the status
    // words are read through to memory, and their traffic and the distance to
    // the nearest inclusive prefix both grow with the number of participants.)
    const uint64_t cur = (uint64_t)blockIdx.x * NWV + (uint64_t)wv;
    const bool have = cur < a.ntiles;  // waves past the last tile only join the barriers
    const int64_t p0 = (int64_t)(cur * a.tw);
    const int64_t K0 = p0 - 16;
    Key m[kR];
    uint32_t emit = 0;
    if (have) {
        RawWords raw;
        fetch_words<IN>(in, K0, lane, raw);
        // 1. bases
        const uint32_t inv_word = commit_words<IN>(in, K0, lane, raw, code, inv);
        wave_lds_sync();
        // a wave whose 1024 bases are all valid skips every invalid-bit step
        // (the keys past 1024 - k, whose k-mers run into the unwritten words,
        // belong to no window the tile stores)
        const bool clean = __ballot(inv_word != 0u) == 0ull;

        // 2. keys.  Without FULL an invalid k-mer gets the all-ones key, which
        //    no valid k-mer reaches, so it never wins against one; whether a
        //    window holds any valid k-mer comes from the invalid bits.
        uint32_t wnone = 0;  // windows without a valid k-mer
        uint32_t wbad = 0;   // split semantics: windows holding an invalid k-mer
        {
            uint64_t val[kR];
            uint32_t bad;
            lane_kmers<KM64, FLAGS>(code, inv, lane, a.k, (a.flags & 1u) == 0u,
                                    (a.flags & 2u) == 0u, clean, val, bad);
            const bool split = FLAGS != 0 && (a.flags & kSplitFlag);
            if ((!FULL || split) && !clean) {
                const uint64_t ext = run_bits3(bad);
                if (!FULL) wnone = window_all_invalid(ext, w);
                if (split) wbad = window_holds_invalid(ext, w);
            }
            make_keys<FULL>(val, bad, !clean, (uint32_t)lane * kR, m);
        }

        // 3. window minimum
        window_min<FULL>(m, w);

        // 4. dedup, as bit masks over the lane's 16 windows: window j is
        //    stored iff owned, valid and its minimum sits at another position
        //    than the previous window's (the first window of the sequence has
        //    no previous one)
        {
            uint32_t fresh = changed_bits(m);
            if (p0 == 0 && lane == 1) fresh |= 1u;  // window 0 is j = 16
            if (FLAGS != 0 && (a.flags & kSplitFlag))
                fresh |= previous_window_bits(wbad);
            uint32_t valid = ~(wnone | wbad);
            if (FULL) {
#pragma unroll
                for (int e = 0; e < kR; ++e)
                    valid &= ~(((m[e].tag & kInvalidTag) != 0u ? 1u : 0u) << e);
            }
            const int64_t lim = (int64_t)a.nwin - K0;
            emit = fresh & valid & owned_bits(lim < 16 + (int64_t)a.tw ? lim : 16 + (int64_t)a.tw,
                                              lane);
        }
    }

    // 5. ordered compaction: lane prefix, workgroup sum, look-back, stores
    //    from registers
    const uint32_t cnt = (uint32_t)__builtin_popcount(emit);
    uint32_t incl = wave_inclusive_sum(cnt);
    if (lane == kWave - 1) s_cnt[wv] = incl;
    __syncthreads();
    if (wv == 0) {
        const uint32_t c = lane < NWV ? s_cnt[lane] : 0u;
        const uint64_t block_total = lane_value_u64(wave_sum_u64(c, lane), 0);
        const uint32_t epoch = call_epoch(a.epoch);
        const uint64_t ex = tile_lookback(a.status, blockIdx.x, block_total, a.err, epoch, lane);
        if (lane == 0) {
            s_base = ex;
            if (blockIdx.x == gridDim.x - 1)
                *a.d_count = final_count(a.err, a.epoch, epoch, ex + block_total);
        }
    }
    __syncthreads();
    if (have) {
        // Compaction through a wave-private LDS buffer: lane l writes its
        // outputs at their ranks within the wave, then the wave copies the
        // buffer out with consecutive lanes on consecutive outputs.  Stored
        // straight from the lanes' runs, each store instruction would scatter
        // a few values per lane over the wave's whole output range; this way
        // measured 0.89 of that time (0.85 from 2-bit input).  A wave with
        // more than kStage outputs takes several rounds.
        uint64_t* sh = s_stage_hash[wv];
        uint32_t* sp = s_stage_pos[wv];
        uint64_t gw = s_base;  // the wave's first output
        for (int v = 0; v < wv; ++v) gw += s_cnt[v];
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
        uint32_t lim = total;  // outputs past the capacity are dropped
        if (gw + total > a.capacity) lim = gw >= a.capacity ? 0u : (uint32_t)(a.capacity - gw);
        const uint32_t pos0 = (uint32_t)K0;  // positions are below 2^32
        const uint32_t tmask = FULL ? 0x7FFFu : 0xFFFFFFFFu;
        if (total <= kStage) {  // one round, the usual case: every rank fits
            uint32_t j = incl - cnt;
#pragma unroll
            for (int e = 0; e < kR; ++e) {
                if ((emit >> e) & 1u) {
                    sh[j] = ((uint64_t)m[e].hi << 32) | m[e].lo;
                    sp[j] = pos0 + (m[e].tag & tmask);
                    ++j;
                }
            }
            wave_lds_sync();
            for (uint32_t r = (uint32_t)lane; r < lim; r += kWave) {
                a.out_hash[gw + r] = sh[r];
                a.out_pos[gw + r] = sp[r];
            }
        } else {
            for (uint32_t c = 0; c < lim; c += kStage) {
                uint32_t j = incl - cnt - c;  // rank - c, mod 2^32
#pragma unroll
                for (int e = 0; e < kR; ++e) {
                    if ((emit >> e) & 1u) {
                        if (j < kStage) {
                            sh[j] = ((uint64_t)m[e].hi << 32) | m[e].lo;
                            sp[j] = pos0 + (m[e].tag & tmask);
                        }
                        ++j;
                    }
                }
                wave_lds_sync();
                const uint32_t nc = min(kStage, lim - c);
                for (uint32_t r = (uint32_t)lane; r < nc; r += kWave) {
                    a.out_hash[gw + c + r] = sh[r];
                    a.out_pos[gw + c + r] = sp[r];
                }
                wave_lds_sync();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Batched minimizers: many reads of uneven length, one launch.
//
// The reads are concatenated; every base position p is a candidate window.
// Window p belongs to the read containing p and exists iff it ends inside that
// read (p + w + k - 1 <= read end); a k-mer exists iff it ends inside its read
// and covers no invalid base; dedup restarts at each read start.  Tiles are
// the single-sequence wavefront tiles over the concatenation.  A tile learns
// the read boundaries it overlaps as a bitmap of read starts in LDS (plus a
// rank -> (read, start) table), and tests "does a read start inside (i, i+L]"
// with the same OR-by-doubling used for invalid bases.  Outputs are read-major
// because the concatenation is; the tile that owns a read's start position
// writes that read's output offset.
// ---------------------------------------------------------------------------
constexpr int kTileRange = kWaveKeys + 64;   // positions whose boundaries a tile needs
constexpr int kBitmapWords = kTileRange / 32 + 2;
// Reads a tile keeps in its LDS table (id, start); a tile overlapping more
// (reads shorter than about 9 bases on average) finds the rest by a binary
// search over the offsets.
constexpr uint32_t kReadSlots = 128;
// Outputs per round of the batched kernel's store compaction.
constexpr uint32_t kBatchStage = 384;

// Read containing the first base of each tile: a read covering tiles whose
// first base (q * tw - 16, clamped at 0) lies in it writes its index there.
__global__ void batch_first_read_kernel(const uint64_t* __restrict__ offsets, uint32_t nreads,
                                        uint32_t tw, uint64_t ntiles,
                                        uint32_t* __restrict__ first_read) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nreads;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = offsets[r], e = offsets[r + 1];
        if (e <= s) continue;
        const uint64_t qa = s == 0 ? 0 : (s + 16 + tw - 1) / tw;
        uint64_t qb = (e + 16 + tw - 1) / tw;
        if (qb > ntiles) qb = ntiles;
        for (uint64_t q = qa; q < qb; ++q) first_read[q] = (uint32_t)r;
    }
}

template <int NT, bool KM64, bool FULL, int FLAGS>
__global__ __launch_bounds__(NT) void minimizer_batch_kernel(GenomeInput in, BatchArgs a) {
    constexpr int NWV = NT / kWave;
    __shared__ uint32_t s_code[NWV][kWaveWords], s_inv[NWV][kWaveWords];
    __shared__ uint32_t s_bits[NWV][kBitmapWords];
    __shared__ uint32_t s_rid[NWV][kReadSlots];
    __shared__ uint32_t s_rstart[NWV][kReadSlots];
    __shared__ uint32_t s_lexcl[NWV][kWave], s_lemit[NWV][kWave];
    // per lane run: listed read starts before it, and its 16 read-start bits
    __shared__ uint32_t s_lstart[NWV][kWave], s_lbits[NWV][kWave];
    __shared__ uint32_t s_cnt[NWV];  // stores per wave tile
    __shared__ uint64_t s_base;      // stores before the workgroup
    __shared__ uint64_t s_stage_hash[NWV][kBatchStage];
    __shared__ uint32_t s_stage_pos[NWV][kBatchStage];

    const int lane = lane_id();
    const int wv = wave_id();
    const uint32_t w = a.w, k = a.k;
    uint32_t* code = s_code[wv];
    uint32_t* inv = s_inv[wv];
    uint32_t* bits = s_bits[wv];
    uint32_t* rid = s_rid[wv];
    uint32_t* rstart = s_rstart[wv];

    // the workgroup's wave tiles are one look-back participant (as in
    // minimizer_wave_kernel)
    const uint64_t cur = (uint64_t)blockIdx.x * NWV + (uint64_t)wv;
    const bool has_tile = cur < a.ntiles;  // waves past the last tile only join the barriers
    const int64_t p0 = (int64_t)(cur * a.tw);
    const int64_t K0 = p0 - 16;
    uint32_t r0 = 0, pre = 0, emit = 0, cnt = 0, incl = 0, sincl = 0, starts = 0;
    uint32_t nlisted = 0;  // reads the tile overlaps (the table keeps kReadSlots)
    uint32_t wbad = 0;   // split semantics: windows holding an invalid k-mer
    uint32_t wnone = 0;  // windows without a valid k-mer (FULL = false)
    uint64_t B = 0;
    Key m[kR];
    if (has_tile) {
        RawWords raw;
        fetch_words<kInAscii>(in, K0, lane, raw);

        // read boundaries of [K0, K0 + kTileRange)
        for (int i = lane; i < kBitmapWords; i += kWave) bits[i] = 0u;
        wave_lds_sync();
        const int64_t rng_end = K0 + kTileRange;
        r0 = a.first_read[cur];
        uint32_t listed = 0;  // pre: the first listed read starts before the tile
        for (uint64_t base_r = r0;; base_r += kWave) {
            const uint64_t r = base_r + (uint64_t)lane;
            const bool have = r < a.nreads;
            const int64_t rs = have ? (int64_t)a.offsets[r] : (int64_t)a.total;
            const int64_t re = have ? (int64_t)a.offsets[r + 1] : (int64_t)a.total;
            const bool take = have && re > rs && re > K0 && rs < rng_end;
            const uint64_t tmask = __ballot(take);
            if (take) {
                const uint32_t idx = listed + (uint32_t)__builtin_popcountll(tmask & ((1ull << lane) - 1ull));
                if (idx < kReadSlots) {
                    rid[idx] = (uint32_t)r;
                    rstart[idx] = (uint32_t)rs;
                }
                if (rs >= K0) {
                    const uint32_t b = (uint32_t)(rs - K0);
                    atomicOr(&bits[b >> 5], 1u << (b & 31));
                } else {
                    pre = 1;
                }
            }
            listed += (uint32_t)__builtin_popcountll(tmask);
            if (__ballot(!have || rs >= rng_end)) break;
        }
        pre = __ballot(pre != 0) ? 1u : 0u;
        nlisted = listed;
        if (lane == 0 && (int64_t)a.total >= K0 && (int64_t)a.total < rng_end) {
            const uint32_t b = (uint32_t)((int64_t)a.total - K0);  // end of the last read
            atomicOr(&bits[b >> 5], 1u << (b & 31));
        }
        wave_lds_sync();
        // this lane's 64 boundary bits from tile position 16 * lane
        {
            const uint32_t wi = (uint32_t)lane >> 1;
            const uint64_t W = (uint64_t)bits[wi] | ((uint64_t)bits[wi + 1] << 32);
            B = (lane & 1) ? ((W >> 16) | ((uint64_t)bits[wi + 2] << 48)) : W;
        }
        const uint32_t kcross = or_after(B, k - 1u);      // k-mer e spans a read start
        const uint32_t wcross = or_after(B, k + w - 2u);  // window e spans a read start

        // bases and keys
        const uint32_t inv_word = commit_words<kInAscii>(in, K0, lane, raw, code, inv);
        wave_lds_sync();
        const bool clean = __ballot(inv_word != 0u) == 0ull;  // as in minimizer_wave_kernel
        {
            uint64_t val[kR];
            uint32_t bad;
            lane_kmers<KM64, FLAGS>(code, inv, lane, k, (a.flags & 1u) == 0u, (a.flags & 2u) == 0u,
                                    clean, val, bad);
            bad |= kcross;
            const bool split = FLAGS != 0 && (a.flags & kSplitFlag);
            if (!FULL || split) {
                const uint64_t ext = run_bits3(bad);
                if (!FULL) wnone = window_all_invalid(ext, w);
                if (split) wbad = window_holds_invalid(ext, w);
            }
            make_keys<FULL>(val, bad, true, (uint32_t)lane * kR, m);
        }
        window_min<FULL>(m, w);

        // dedup, restarting at read starts (bit masks as in the single-sequence
        // kernel)
        {
            uint32_t fresh = changed_bits(m) | ((uint32_t)B & 0xFFFFu);
            if (FLAGS != 0 && (a.flags & kSplitFlag))
                fresh |= previous_window_bits(wbad);
            uint32_t valid = ~(wnone | wbad | wcross);
            if (FULL) {
#pragma unroll
                for (int e = 0; e < kR; ++e)
                    valid &= ~(((m[e].tag & kInvalidTag) != 0u ? 1u : 0u) << e);
            }
            const int64_t lim = (int64_t)a.total - K0;
            emit = fresh & valid & owned_bits(lim < 16 + (int64_t)a.tw ? lim : 16 + (int64_t)a.tw,
                                              lane);
        }
        cnt = (uint32_t)__builtin_popcount(emit);
        starts = (uint32_t)__builtin_popcountll(B & 0xFFFFull);
        incl = wave_inclusive_sum(cnt);
        sincl = wave_inclusive_sum(starts);
        s_lexcl[wv][lane] = incl - cnt;
        s_lemit[wv][lane] = emit;
        s_lstart[wv][lane] = pre + sincl - starts;
        s_lbits[wv][lane] = (uint32_t)B & 0xFFFFu;
    }

    const uint32_t total = lane_value(incl, kWave - 1);
    if (lane == 0) s_cnt[wv] = total;
    __syncthreads();
    if (wv == 0) {
        const uint32_t c = lane < NWV ? s_cnt[lane] : 0u;
        const uint64_t block_total = lane_value_u64(wave_sum_u64(c, lane), 0);
        const uint32_t epoch = call_epoch(a.epoch);
        const uint64_t ex = tile_lookback<32>(a.status, blockIdx.x, block_total, a.err, epoch, lane);
        if (lane == 0) {
            s_base = ex;
            if (blockIdx.x == gridDim.x - 1)
                a.read_out[a.nreads] = final_count(a.err, a.epoch, epoch, ex + block_total);
        }
    }
    __syncthreads();
    if (!has_tile) return;  // no barrier follows
    uint64_t excl = s_base;
    for (int v = 0; v < wv; ++v) excl += s_cnt[v];
    // Compaction through wave-private LDS, as in minimizer_wave_kernel: lane
    // l writes its outputs at their ranks within the wave, then consecutive
    // lanes store consecutive outputs.  More than kBatchStage outputs take
    // several rounds.
    const uint32_t total_w = lane_value(incl, kWave - 1);
    uint32_t lim = total_w;  // outputs past the capacity are dropped
    if (excl + total_w > a.capacity) lim = excl >= a.capacity ? 0u : (uint32_t)(a.capacity - excl);
    uint64_t* sh = s_stage_hash[wv];
    uint32_t* sp = s_stage_pos[wv];
    for (uint32_t c = 0; c < lim; c += kBatchStage) {
        // stage each output's hash and tile position (the lanes' runs stay
        // in registers: only unrolled loops touch them)
        uint32_t j = incl - cnt - c;  // rank - c, mod 2^32
        if (total_w <= kBatchStage) {  // one round, the usual case: every rank fits
#pragma unroll
            for (int e = 0; e < kR; ++e) {
                if ((emit >> e) & 1u) {
                    sh[j] = ((uint64_t)m[e].hi << 32) | m[e].lo;
                    sp[j] = m[e].tag & (FULL ? 0x7FFFu : 0xFFFFu);
                    ++j;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < kR; ++e) {
                if ((emit >> e) & 1u) {
                    if (j < kBatchStage) {
                        sh[j] = ((uint64_t)m[e].hi << 32) | m[e].lo;
                        sp[j] = m[e].tag & (FULL ? 0x7FFFu : 0xFFFFu);
                    }
                    ++j;
                }
            }
        }
        wave_lds_sync();
        // resolve positions to reads and store, consecutive lanes on
        // consecutive outputs.  The read of tile position t is the listed
        // read of rank (starts before t's lane run) + (starts in the run up
        // to t) - 1.
        const uint32_t nc = min(kBatchStage, lim - c);
        for (uint32_t q = (uint32_t)lane; q < nc; q += kWave) {
            const uint32_t t = sp[q];
            const uint32_t l = t >> 4, e = t & 15u;
            const uint32_t rk = s_lstart[wv][l] +
                                (uint32_t)__builtin_popcount(s_lbits[wv][l] & ((2u << e) - 1u)) - 1u;
            const uint32_t pos = (uint32_t)(K0 + (int64_t)t);
            uint32_t rr, rs;
            if (rk < kReadSlots && rk < nlisted) {
                rr = rid[rk];
                rs = rstart[rk];
            } else {
                // past the table: the read holding pos is the last one
                // starting at or before it (offsets[r0] <= the tile's first
                // base <= pos < total)
                uint64_t lo = r0, hi = a.nreads;  // offsets[lo] <= pos < offsets[hi]
                while (hi - lo > 1) {
                    const uint64_t mid = lo + (hi - lo) / 2;
                    if (a.offsets[mid] <= (uint64_t)pos) lo = mid;
                    else hi = mid;
                }
                rr = (uint32_t)lo;
                rs = (uint32_t)a.offsets[lo];
            }
            a.out_hash[excl + c + q] = sh[q];
            a.out_pos[excl + c + q] = pos - rs;
            a.out_read[excl + c + q] = rr;
        }
        wave_lds_sync();
    }
    // output offsets of the reads that start in the windows this tile owns
    const bool last = cur == a.ntiles - 1;
    const int64_t own_end = last ? INT64_MAX : p0 + (int64_t)a.tw;
    for (uint64_t base_r = r0;; base_r += kWave) {
        const uint64_t r = base_r + (uint64_t)lane;
        const bool have = r < a.nreads;
        const int64_t rs = have ? (int64_t)a.offsets[r] : INT64_MAX;
        if (have && rs >= p0 && rs < own_end) {
            const int64_t j = rs - K0;
            uint32_t before = total;
            if (j < 16 + (int64_t)a.tw) {
                const uint32_t l = (uint32_t)(j >> 4), e = (uint32_t)(j & 15);
                before = s_lexcl[wv][l] + (uint32_t)__builtin_popcount(s_lemit[wv][l] & ((1u << e) - 1u));
            }
            a.read_out[r] = excl + before;
        }
        if (__ballot(!have || rs >= own_end)) break;
    }
}

__global__ void zero_words_kernel(uint64_t* __restrict__ p, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
int launch_zero(uint64_t* p, uint64_t words, hipStream_t s) {
    const uint64_t blocks = (words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), 0, s, p,
                       words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pack2bit(const uint8_t* seq, uint64_t n, uint32_t* packed, uint32_t* invalid,
                    hipStream_t s) {
    const uint64_t nwords = (n + 15) / 16;
    // one extra lane when nwords is odd so the pair (i, i+1) always exists
    const uint64_t lanes = (nwords + 1) & ~1ull;
    const uint64_t blocks = (lanes + 255) / 256;
    const int aligned = ((uintptr_t)seq & 15u) == 0;
    hipLaunchKernelGGL(pack2bit_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seq, n, packed,
                       invalid, aligned, nwords);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int NT, bool PAIRS>
static void launch_kmers_variant(const GenomeInput& in, uint32_t k, uint32_t flags, uint64_t nk,
                                 uint64_t* out, hipStream_t s) {
    const unsigned blocks = (unsigned)((nk + NT * kR - 1) / (NT * kR));
    if (k <= 16) {
        if (in.kind == kInAscii)
            hipLaunchKernelGGL((kmers_kernel<NT, kInAscii, false, PAIRS>), dim3(blocks), dim3(NT), 0, s, in, k, flags, nk, out);
        else
            hipLaunchKernelGGL((kmers_kernel<NT, kIn2bit, false, PAIRS>), dim3(blocks), dim3(NT), 0, s, in, k, flags, nk, out);
    } else {
        if (in.kind == kInAscii)
            hipLaunchKernelGGL((kmers_kernel<NT, kInAscii, true, PAIRS>), dim3(blocks), dim3(NT), 0, s, in, k, flags, nk, out);
        else
            hipLaunchKernelGGL((kmers_kernel<NT, kIn2bit, true, PAIRS>), dim3(blocks), dim3(NT), 0, s, in, k, flags, nk, out);
    }
}

int launch_kmers(const GenomeInput& in, uint32_t k, uint32_t flags, uint64_t* out, hipStream_t s) {
    constexpr int NT = 256;
    const uint64_t nk = in.n - k + 1;
    if (((uintptr_t)out & 15u) == 0u) launch_kmers_variant<NT, true>(in, k, flags, nk, out, s);
    else launch_kmers_variant<NT, false>(in, k, flags, nk, out, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int NT, bool KM64, bool FULL>
static void launch_batch_variant(const GenomeInput& in, const BatchArgs& a, hipStream_t s) {
    constexpr int NWV = NT / kWave;
    const unsigned grid = (unsigned)((a.ntiles + NWV - 1) / NWV);
    if (a.flags == 0u)
        hipLaunchKernelGGL((minimizer_batch_kernel<NT, KM64, FULL, 0>), dim3(grid), dim3(NT), 0, s,
                           in, a);
    else
        hipLaunchKernelGGL((minimizer_batch_kernel<NT, KM64, FULL, -1>), dim3(grid), dim3(NT), 0,
                           s, in, a);
}

int launch_minimizers_batch(const GenomeInput& in, BatchArgs a, uint32_t nt, void* workspace,
                            hipStream_t s, bool kept) {
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    a.err = reinterpret_cast<uint32_t*>(ws + 8);
    a.status = reinterpret_cast<uint64_t*>(ws + kWsStatusOffset);
    a.epoch = reinterpret_cast<uint64_t*>(ws + 16);
    a.first_read = reinterpret_cast<uint32_t*>(ws + kWsStatusOffset + 8 * kStatusStride * a.ntiles);
    // a kept workspace holds an earlier call's epoch and status words, which
    // the epoch tells apart from this call's (as in launch_minimizers); the
    // read table is rewritten below either way
    if (!kept && launch_zero(reinterpret_cast<uint64_t*>(ws),
                             kWsStatusOffset / 8 + kStatusStride * a.ntiles, s) != 0)
        return -1;
    const uint64_t rb = ((uint64_t)a.nreads + 255) / 256;
    hipLaunchKernelGGL(batch_first_read_kernel, dim3((unsigned)(rb < 4096 ? (rb ? rb : 1) : 4096)),
                       dim3(256), 0, s, a.offsets, a.nreads, a.tw, a.ntiles, a.first_read);
    const bool km64 = a.k > 16;
    const bool full = a.k >= 30 && (a.flags & 2u) == 0u;
    if (nt == 128) {
        if (!km64) launch_batch_variant<128, false, false>(in, a, s);
        else if (!full) launch_batch_variant<128, true, false>(in, a, s);
        else launch_batch_variant<128, true, true>(in, a, s);
    } else if (nt == 512) {
        if (!km64) launch_batch_variant<512, false, false>(in, a, s);
        else if (!full) launch_batch_variant<512, true, false>(in, a, s);
        else launch_batch_variant<512, true, true>(in, a, s);
    } else if (nt == 64) {
        if (!km64) launch_batch_variant<64, false, false>(in, a, s);
        else if (!full) launch_batch_variant<64, true, false>(in, a, s);
        else launch_batch_variant<64, true, true>(in, a, s);
    } else {
        if (!km64) launch_batch_variant<256, false, false>(in, a, s);
        else if (!full) launch_batch_variant<256, true, false>(in, a, s);
        else launch_batch_variant<256, true, true>(in, a, s);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

uint64_t batch_workspace_bytes(uint64_t ntiles) {
    return kWsStatusOffset + (8ull * kStatusStride + 4ull) * ntiles;
}

// Windows a wave tile stores: its 1024 keys less the 16 before its first
// window, the w - 1 keys the last window reaches past its start and the
// k - 1 keys whose k-mers run past the tile's bases; a multiple of 16.
uint32_t wave_tile_windows(uint32_t k, uint32_t w) {
    const uint32_t need = 16u + (w - 1u) + (k - 1u);
    if ((uint32_t)kWaveKeys < need + 16u) return 0;
    return ((uint32_t)kWaveKeys - need) & ~15u;
}

uint32_t batch_tile_windows(uint32_t k, uint32_t w) { return wave_tile_windows(k, w); }

uint32_t minimizer_tile_windows(uint32_t nt, uint32_t w) {
    const uint32_t P = nt * kR;
    if (P < 32u + w) return 0;
    return (P - 16u - (w - 1u)) & ~15u;
}

uint32_t minimizer_wave_max_window() { return 32; }

// Windows stored per tile: one wavefront's 1024 keys when w <= 32, else the
// workgroup's 16 * nt keys.
uint32_t minimizer_windows_per_tile(uint32_t nt, uint32_t k, uint32_t w) {
    return w <= minimizer_wave_max_window() ? wave_tile_windows(k, w)
                                            : minimizer_tile_windows(nt, w);
}

uint64_t minimizer_workspace_bytes(uint64_t ntiles) {
    return kWsStatusOffset + 8ull * kStatusStride * ntiles;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free minimizer entry point: the look-back header
// and status words live in this file-scope array instead of a caller
// workspace.  Each GPU holds its own copy, at its own address, until the
// process ends; host code must never pass the array's name to a kernel (on
// the host it is a stand-in, not a device address), only the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices];  // per device, filled on first use
}  // namespace

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device] == nullptr) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return nullptr;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
            (void)hipGetLastError();  // leave no sticky error behind for the caller
            return nullptr;
        }
        g_scratch_addr[device] = p;
    }
    return g_scratch_addr[device];
}

template <int NT, int IN, bool KM64, bool FULL>
static void launch_wave_variant(const GenomeInput& in, const MinimizerArgs& a, hipStream_t s) {
    constexpr int NWV = NT / kWave;
    const unsigned grid = (unsigned)((a.ntiles + NWV - 1) / NWV);
    // canonical + hashed (flags 0) is compiled with the flags fixed
    if (a.flags == 0u)
        hipLaunchKernelGGL((minimizer_wave_kernel<NT, IN, KM64, FULL, 0>), dim3(grid), dim3(NT), 0,
                           s, in, a);
    else
        hipLaunchKernelGGL((minimizer_wave_kernel<NT, IN, KM64, FULL, -1>), dim3(grid), dim3(NT),
                           0, s, in, a);
}

template <int NT, int IN>
static void launch_min_wave(const GenomeInput& in, const MinimizerArgs& a, bool km64, bool full,
                            hipStream_t s) {
    if (!km64) launch_wave_variant<NT, IN, false, false>(in, a, s);
    else if (!full) launch_wave_variant<NT, IN, true, false>(in, a, s);
    else launch_wave_variant<NT, IN, true, true>(in, a, s);
}

template <int NT, int IN>
static void launch_min_nt(const GenomeInput& in, const MinimizerArgs& a, bool km64, bool full,
                          hipStream_t s) {
    const dim3 grid((unsigned)a.ntiles), block(NT);
    if (!km64)
        hipLaunchKernelGGL((minimizer_kernel<NT, IN, false, false>), grid, block, 0, s, in, a);
    else if (!full)
        hipLaunchKernelGGL((minimizer_kernel<NT, IN, true, false>), grid, block, 0, s, in, a);
    else
        hipLaunchKernelGGL((minimizer_kernel<NT, IN, true, true>), grid, block, 0, s, in, a);
}

int launch_minimizers(const GenomeInput& in, MinimizerArgs a, uint32_t nt, void* workspace,
                      hipStream_t s, bool kept) {
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    a.err = reinterpret_cast<uint32_t*>(ws + 8);
    a.epoch = reinterpret_cast<uint64_t*>(ws + 16);
    a.status = reinterpret_cast<uint64_t*>(ws + kWsStatusOffset);
    // one status word per look-back participant: a workgroup of wave tiles on
    // the w <= 32 path, a tile (= workgroup) otherwise
    const bool wave_path = a.w <= minimizer_wave_max_window();
    const uint64_t parts = wave_path ? (a.ntiles + kWaveTileGroup - 1) / kWaveTileGroup : a.ntiles;
    // a kept workspace holds the last call's epoch and status words, which
    // the epoch tells apart from this call's: nothing to clear
    if (!kept && launch_zero(reinterpret_cast<uint64_t*>(ws),
                             kWsStatusOffset / 8 + kStatusStride * parts, s) != 0)
        return -1;
    const bool km64 = a.k > 16;
    const bool full = a.k >= 30 && (a.flags & 2u) == 0u;
    if (wave_path) {
        constexpr int NT = kWaveTileGroup * kWave;
        if (in.kind == kInAscii) launch_min_wave<NT, kInAscii>(in, a, km64, full, s);
        else launch_min_wave<NT, kIn2bit>(in, a, km64, full, s);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    // the block kernel is built for 256-thread tiles only; a.tw was computed
    // for that width
    if (nt != 256) return -1;
    if (in.kind == kInAscii) launch_min_nt<256, kInAscii>(in, a, km64, full, s);
    else launch_min_nt<256, kIn2bit>(in, a, km64, full, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sws
