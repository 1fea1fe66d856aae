// sliding.hip -- sliding window sums y_i = x_i (+) ... (+) x_{i+w-1}
// (Sec. 2.2, Eq. 2) on gfx950.
//
// Generic path (any associative operator; Sec. 3.1, Alg. 2 with the vector
// length taken equal to w).  Cut the index space into segments of w elements
// starting at multiples of w.  With Pf the in-segment prefix and Sf the
// in-segment suffix,
//     y_i = Pf_{i+w-1}                 if i starts a segment,
//     y_i = Sf_i (+) Pf_{i+w-1}        otherwise,
// since the window [i, i+w-1] is the tail of i's segment followed by the head
// of the next one.  That is three operator applications per output whatever w
// is; only associativity is used and the left operand is always the earlier
// element, so non-commutative operators keep the order of Eq. 2.
//
// Mapping: every wavefront streams its own contiguous run of "slabs" of
// S = 64*R elements; lane l holds elements [l*R, l*R+R) of a slab in
// registers.  Prefix and suffix sums are serial inside a lane; across lanes a
// segmented Hillis-Steele scan with log2(ceil(w/R)) shuffle steps carries the
// partial sums of segments that span lanes (w <= S, so a segment spans at most
// two slabs).  Across slabs the carried state is one value each way: the
// prefix at the end of the previous slab (the paper's vector Y of Alg. 2) and
// the suffix at the start of the next slab, which patches the last segment
// of the current slab.  Prefix sums of two consecutive slabs sit in a per-wave
// LDS ring, from which each lane reads Pf_{i+w-1}.  No workgroup barrier, no
// global scratch; HBM sees each element read once and each output written once.
//
// Ring layout: rows of R elements (one lane's run), each padded by one
// element, so lane l's writes of element e and its reads of Pf_{i+w-1} are
// both one row apart across lanes and free of bank conflicts.  Rows 0..63 and
// 64..127 are the two slab regions; rows from 128 on repeat the first rows of
// region 0, so that the reads of a slab in region 1 never wrap.  A read
// address is then the lane's row base plus a wave-uniform offset.  The region
// that is dead at each moment doubles as the staging area through which
// coalesced 16-byte loads and stores are redistributed into lane runs.
//
// Log path (MIN and MAX only; Sec. 3.1, the commutative case).  With
// m^(1) = x, m^(2s)_i = m^(s)_i (+) m^(s)_{i+s} and 2^t the largest power of two
// not above w, y_i = m^(2^t)_i (+) m^(2^t)_{i+w-2^t}; the two halves overlap,
// which idempotence allows.  floor(log2 w) + 1 applications per output.  A
// workgroup loads a tile plus its (w-1)-element halo into LDS and runs the
// doubling levels between two LDS buffers.
#include "sws_device.hpp"
#include "sws_internal.hpp"
#include "sws_scan.hpp"

#include <type_traits>
#include <utility>

namespace sws {

// ---------------------------------------------------------------------------
// Generic path.
// ---------------------------------------------------------------------------
// Coalesced movement of one slab between HBM and a lane's run of R elements:
// lane l loads/stores the 16-byte chunks l, l + 64, l + 128, ... of the slab
// (every instruction covers 1 KB of contiguous memory) and the chunks change
// hands through a per-wave LDS staging area holding one 16-byte pad per four
// lane runs (64 * kChunks + 16 chunks: one ring region).
template <class T, int R>
struct SlabIO {
    static constexpr int kChunks = (int)(R * sizeof(T) / 16);  // chunks per lane run
    static constexpr int kStageWords = (kWave * kChunks + 16) * 4;

    static __device__ __forceinline__ uint32_t stage_off(int chunk) {  // in u32 words
        return (uint32_t)(chunk + chunk / (4 * kChunks)) * 4u;
    }

    // raw[i] = chunk (i * 64 + lane) of the slab starting at element p0.
    // CHECK = false: the caller guarantees an aligned slab wholly below n, and
    // the loads are straight-line code.  CHECK = true: elements at or past n
    // read as the identity.
    template <bool CHECK>
    static __device__ __forceinline__ void load(const T* __restrict__ x, uint64_t n, uint64_t p0,
                                                int lane, bool vec, T ident, u32x4 (&raw)[kChunks]) {
        const uint64_t per = 16 / sizeof(T);
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const uint64_t e0 = p0 + (uint64_t)(i * kWave + lane) * per;
            if (!CHECK || (vec && e0 + per <= n)) {
                raw[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(x + e0));
            } else {
                const uint32_t* xw = reinterpret_cast<const uint32_t*>(x);
                const uint32_t* iw = reinterpret_cast<const uint32_t*>(&ident);
                constexpr int wpe = (int)(sizeof(T) / 4);  // words per element
                u32x4 c;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t e = e0 + (uint64_t)(q / wpe);
                    c[q] = e < n ? xw[e * wpe + (q % wpe)] : iw[q % wpe];
                }
                raw[i] = c;
            }
        }
    }

    // Chunks below nchunks of the slab at element p0 (wholly below n), the
    // rest as the identity: the slab after a wave's last one is needed only
    // up to its first w - 1 elements.
    template <bool NT = true>
    static __device__ __forceinline__ void load_head(const T* __restrict__ x, uint64_t p0, int lane,
                                                     uint32_t nchunks, T ident,
                                                     u32x4 (&raw)[kChunks]) {
        const uint64_t per = 16 / sizeof(T);
        const uint32_t* iw = reinterpret_cast<const uint32_t*>(&ident);
        constexpr int wpe = (int)(sizeof(T) / 4);
        u32x4 id;
#pragma unroll
        for (int q = 0; q < 4; ++q) id[q] = iw[q % wpe];
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const uint32_t c = (uint32_t)(i * kWave + lane);
            const u32x4* src = reinterpret_cast<const u32x4*>(x + p0 + (uint64_t)c * per);
            raw[i] = c < nchunks ? (NT ? __builtin_nontemporal_load(src) : *src) : id;
        }
    }

    // raw chunks -> this lane's run, through the staging area
    static __device__ __forceinline__ void to_run(uint32_t* stage, int lane,
                                                  const u32x4 (&raw)[kChunks], T (&v)[R]) {
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<u32x4*>(stage + stage_off(i * kWave + lane)) = raw[i];
        wave_lds_sync();
        u32x4 q[kChunks];
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            q[i] = *reinterpret_cast<const u32x4*>(stage + stage_off(lane * kChunks + i));
        const T* t = reinterpret_cast<const T*>(q);
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = t[e];
        wave_lds_sync();
    }

    // this lane's run -> coalesced stores of the slab at element p0; with
    // CHECK = false the slab is aligned and wholly below limit.
    template <bool CHECK>
    static __device__ __forceinline__ void store(T* __restrict__ y, uint64_t limit, uint64_t p0,
                                                 int lane, bool vec, uint32_t* stage,
                                                 const T (&v)[R]) {
        const u32x4* q = reinterpret_cast<const u32x4*>(v);
        wave_lds_sync();  // earlier reads of the staging area have completed
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<u32x4*>(stage + stage_off(lane * kChunks + i)) = q[i];
        wave_lds_sync();
        const uint64_t per = 16 / sizeof(T);
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const u32x4 c = *reinterpret_cast<const u32x4*>(stage + stage_off(i * kWave + lane));
            const uint64_t e0 = p0 + (uint64_t)(i * kWave + lane) * per;
            if (!CHECK || (vec && e0 + per <= limit)) {
                __builtin_nontemporal_store(c, reinterpret_cast<u32x4*>(y + e0));
            } else {
                uint32_t* yw = reinterpret_cast<uint32_t*>(y);
                constexpr int wpe = (int)(sizeof(T) / 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint64_t e = e0 + (uint64_t)(q / wpe);
                    if (e < limit) yw[e * wpe + (q % wpe)] = c[q];
                }
            }
        }
        wave_lds_sync();
    }
};

// Suffix sums at segment heads are never read (a window starting at a head is
// one whole segment, Pf alone); storing the identity there lets every output
// take the form Sf (+) Pf.
template <int R, class T>
__device__ __forceinline__ void heads_to_identity(T (&sf)[R], HeadMask<R> h, T ident) {
#pragma unroll
    for (int e = 0; e < R; ++e)
        if (head_bit<R>(h, e)) sf[e] = ident;
}

// Ring rows a window of w needs: two regions of 64 rows plus the repeated
// rows read past row 127, rounded up to a multiple of 4 (keeps every region
// 16-byte aligned).
template <int R>
__host__ __device__ constexpr uint32_t ring_rows(uint32_t w) {
    return (128u + (R + w - 2u) / R + 3u) & ~3u;
}

// PFX: the prefix-difference form for an invertible operator (+ mod 2^32):
// y_i = P_{i+w-1} - P_{i-1} with P a running prefix local to the wave (an
// offset common to both terms cancels).  The ring then holds P, the suffix
// registers hold the exclusive prefix, and the segment masks are unused.
template <class Op, int R, int WAVES, bool PFX = false, bool EARLY_HALO = false>
__global__ __launch_bounds__(WAVES * kWave) void sliding_generic_kernel(
    const typename Op::T* __restrict__ x, uint64_t n, uint32_t w, typename Op::T* __restrict__ y,
    uint64_t count, uint64_t total_slabs, uint64_t slabs_per_wave, int vec, uint32_t rows) {
    using T = typename Op::T;
    using IO = SlabIO<T, R>;
    static_assert(!PFX || sizeof(T) == 4, "the prefix-difference form is for + on u32");
    constexpr uint32_t S = kWave * R;
    constexpr uint32_t RS = R + 1;              // ring row stride (elements)
    constexpr uint32_t REGION = kWave * RS;     // elements per slab region
    static_assert(IO::kStageWords * 4 <= REGION * sizeof(T), "staging fits a region");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = lane_id();
    const int wv = wave_id();
    T* ring = reinterpret_cast<T*>(lds_raw) + (size_t)wv * rows * RS;
    auto stage_of = [&](uint32_t region) {
        return reinterpret_cast<uint32_t*>(ring + region * REGION);
    };
    const uint64_t gw = (uint64_t)blockIdx.x * WAVES + (uint64_t)wv;
    const uint64_t s0 = gw * slabs_per_wave;
    if (s0 >= total_slabs) return;
    const uint64_t s1 = s0 + slabs_per_wave < total_slabs ? s0 + slabs_per_wave : total_slabs;

    const uint32_t span = PFX ? (uint32_t)kWave : (w + R - 1) / R;
    const uint32_t head_chunks = (uint32_t)(((w - 1u) * sizeof(T) + 15u) / 16u);  // first w - 1 elements
    const uint32_t mirror = (R + w - 2u) / R;  // rows of region 0 repeated from row 128
    const uint32_t lane_row = (uint32_t)lane * RS;
    const uint32_t lane_mod = (uint32_t)(((uint64_t)lane * R) % w);
    const uint32_t slab_mod_step = S % w;
    const HeadMask<R> pat = head_pattern<R>(w);
    const T ident = Op::identity();
    const bool v16 = vec != 0;

    // Which steps run unchecked (see the loop at the end): the step that
    // prefetches the next wave's first slab (MODE 3) runs when the wave has
    // two slabs or more and both bounds reach its last slab.
    const uint64_t by_count = count / S;  // s + 1 <= count / S: outputs in range
    const uint64_t by_n = n / S >= 3 ? n / S - 2 : 0;  // s + 3 <= n / S
    const bool mode3 = v16 && s0 + 2 <= s1 && by_n >= s1 - 1 && by_count >= s1 - 1;
    // EARLY_HALO: that slab's first w - 1 elements (this wave's halo) are
    // loaded now, through the caches, while the next wave (the workgroup's
    // other wave, or the next workgroup's first) loads the same lines as its
    // first slab, rather than at this wave's end, when they have long left
    // the caches.  They wait in registers (16 VGPRs at R = 16).
    u32x4 halo[EARLY_HALO ? IO::kChunks : 1];
    if constexpr (EARLY_HALO) {
        if (mode3) IO::template load_head<false>(x, s1 * (uint64_t)S, lane, head_chunks, ident, halo);
    }

    // slab A = s0: prefix sums into ring half 0, suffix sums in registers
    uint32_t mA = (uint32_t)((s0 * (uint64_t)S) % w);
    HeadMask<R> headsA;
    T sfA[R];
    T carryA;
    u32x4 raw[IO::kChunks];
    IO::template load<true>(x, n, s0 * S, lane, v16, ident, raw);
    {
        T v[R];
        IO::to_run(stage_of(1), lane, raw, v);
        uint32_t m0 = mA + lane_mod;
        m0 = m0 >= w ? m0 - w : m0;
        headsA = PFX ? (HeadMask<R>)0 : lane_heads<R>(m0, w, pat);
#pragma unroll
        for (int e = 0; e < R; ++e) sfA[e] = v[e];
        slab_prefix<Op, R>(v, headsA, span, lane, ident);
#pragma unroll
        for (int e = 0; e < R; ++e) ring[lane_row + e] = v[e];
        carryA = lane_value(v[R - 1], kWave - 1);
        if constexpr (PFX) {
#pragma unroll
            for (int e = 0; e < R; ++e) sfA[e] = v[e] - sfA[e];  // exclusive prefix
        } else {
            slab_suffix<Op, R>(sfA, headsA, span, lane);
            heads_to_identity<R>(sfA, headsA, ident);
        }
    }
    // slab B; when it is the next wave's first slab, only its first w - 1
    // elements enter this wave's outputs
    const uint64_t halo_n = s1 * (uint64_t)S + w - 1u < n ? s1 * (uint64_t)S + w - 1u : n;
    IO::template load<true>(x, s0 + 1 == s1 ? halo_n : n, (s0 + 1) * S, lane, v16, ident, raw);
    uint32_t half = 0;  // ring half holding slab A's prefix sums

    // One step: slab A = s gets its outputs, slab B = s + 1 (in raw) becomes A.
    // MODE 0: every access in range and slab s + 2 is loaded into raw;
    // MODE 1: every access in range, nothing left to load (the last slab of
    // the wave); MODE 2: accesses checked against n and count; MODE 3: as
    // MODE 0 with slab s + 2 the next wave's first, of which only the first
    // w - 1 elements are loaded.
    auto step = [&](uint64_t s, auto mode) {
        constexpr int MODE = decltype(mode)::value;
        constexpr bool CHECK = MODE == 2;
        const uint64_t baseA = s * S;
        uint32_t mB = mA + slab_mod_step;
        mB = mB >= w ? mB - w : mB;
        T sfB[R];
        HeadMask<R> headsB;
        {
            T v[R];
            IO::to_run(stage_of(half ^ 1u), lane, raw, v);  // B's region is free
            // prefetch slab s + 2 while B and A are computed
            if (MODE == 0)
                IO::template load<false>(x, n, baseA + 2 * (uint64_t)S, lane, v16, ident, raw);
            else if (MODE == 3) {
                if constexpr (EARLY_HALO) {
#pragma unroll
                    for (int i = 0; i < IO::kChunks; ++i) raw[i] = halo[i];
                } else {
                    IO::load_head(x, baseA + 2 * (uint64_t)S, lane, head_chunks, ident, raw);
                }
            }
            else if (MODE == 2 && s + 1 < s1)
                IO::template load<true>(x, s + 2 == s1 ? halo_n : n, baseA + 2 * (uint64_t)S,
                                        lane, v16, ident, raw);
            uint32_t m0 = mB + lane_mod;
            m0 = m0 >= w ? m0 - w : m0;
            headsB = PFX ? (HeadMask<R>)0 : lane_heads<R>(m0, w, pat);
#pragma unroll
            for (int e = 0; e < R; ++e) sfB[e] = v[e];
            slab_prefix<Op, R>(v, headsB, span, lane, carryA);
            T* rowB = ring + (half ^ 1u) * REGION + lane_row;
#pragma unroll
            for (int e = 0; e < R; ++e) rowB[e] = v[e];
            if (half == 1u && (uint32_t)lane < mirror) {  // B in region 0: repeat its first rows
#pragma unroll
                for (int e = 0; e < R; ++e) rowB[2 * REGION + e] = v[e];
            }
            carryA = lane_value(v[R - 1], kWave - 1);
            if constexpr (PFX) {
#pragma unroll
                for (int e = 0; e < R; ++e) sfB[e] = v[e] - sfB[e];  // exclusive prefix
            } else {
                slab_suffix<Op, R>(sfB, headsB, span, lane);
                heads_to_identity<R>(sfB, headsB, ident);
            }
        }
        // the last segment of A continues into B: append B's leading suffix
        // (B's first element is not a head here, so sfB[0] in lane 0 is real)
        if constexpr (!PFX) {
            const T c = lane_value(sfB[0], 0);
            const uint32_t last = (mA + S - 1u) % w;
            if (last != w - 1u) {
                const uint32_t head_rel = S - 1u - last;
#pragma unroll
                for (int e = 0; e < R; ++e)
                    if ((uint32_t)lane * R + e > head_rel) sfA[e] = Op::combine(sfA[e], c);
            }
        }
        wave_lds_sync();
        // outputs of slab A: y_i = Pf_{i+w-1} at a head, Sf_i (+) Pf_{i+w-1}
        // elsewhere; sfA holds the identity at heads, so one form serves both
        {
            T out[R];
            // Pf_{i+w-1} for element e of this lane: row base + (c + e) + (c + e) / R
            // past the start of A's region, c = w - 1 (uniform)
            const T* rowA = ring + half * REGION + lane_row;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                const uint32_t q = w - 1u + (uint32_t)e;
                if constexpr (PFX) out[e] = rowA[q + q / R] - sfA[e];  // P_{i+w-1} - P_{i-1}
                else out[e] = Op::combine(sfA[e], rowA[q + q / R]);
            }
            IO::template store<CHECK>(y, count, baseA, lane, v16, stage_of(half), out);
        }
#pragma unroll
        for (int e = 0; e < R; ++e) sfA[e] = sfB[e];
        headsA = headsB;
        mA = mB;
        half ^= 1u;
    };
    // Steps whose prefetch (slab s + 2) lies below n and whose outputs (slab
    // s) lie below count, on aligned buffers, run without bounds checks; the
    // last step of a wave loads nothing, and the last waves check every
    // access.  The first unchecked step is peeled so that both ways into the
    // loop leave the same memory operations in flight (the prefetch, then the
    // stores); the wait for the prefetched slab then need not wait for the
    // stores.
    using M0 = std::integral_constant<int, 0>;
    using M1 = std::integral_constant<int, 1>;
    using M2 = std::integral_constant<int, 2>;
    using M3 = std::integral_constant<int, 3>;
    uint64_t s = s0;
    if (v16) {
        uint64_t pf_end = by_n < by_count ? by_n : by_count;
        if (pf_end > s1 - 1) pf_end = s1 - 1;
        if (s < pf_end) {
            // pf_end <= s1 - 1; the step s1 - 2 prefetches the next wave's slab
            const uint64_t full_end = pf_end == s1 - 1 ? s1 - 2 : pf_end;
            if (s < full_end) {
                step(s++, M0());
                for (; s < full_end; ++s) step(s, M0());
            }
            if (s < pf_end) step(s++, M3());
        }
    }
    for (; s < s1; ++s) {
        if (v16 && s < by_count && s + 1 == s1) step(s, M1());
        else step(s, M2());
    }
}

// ---------------------------------------------------------------------------
// Log path (MIN / MAX).
// ---------------------------------------------------------------------------
// LDS index of tile position i: one pad word per 16, so that threads reading
// runs of 16 consecutive positions (one run per thread) hit distinct banks.
__device__ __forceinline__ uint32_t log_pad(uint32_t i) { return i + (i >> 4); }

constexpr int kLogRun = 16;  // positions per thread run in the register levels

// One doubling level on a register window: v[e] = v[e] (+) v[e + S].
template <class Op, int S, int N>
__device__ __forceinline__ void log_level(uint32_t (&v)[N]) {
#pragma unroll
    for (int e = 0; e + S < N; ++e) v[e] = Op::combine(v[e], v[e + S]);
}

template <class Op, int NT>
__global__ __launch_bounds__(NT) void sliding_log_kernel(const uint32_t* __restrict__ x, uint64_t n,
                                                         uint32_t w, uint32_t* __restrict__ y,
                                                         uint64_t count, uint32_t tile, int vec) {
    constexpr int RR = kLogRun;
    extern __shared__ uint32_t lds[];
    const uint32_t L = tile + w - 1u;           // tile plus its halo
    uint32_t* bufA = lds;
    uint32_t* bufB = lds + log_pad(L) + 1u;
    const uint64_t t0 = (uint64_t)blockIdx.x * tile;
    // load the tile and halo; aligned 16-byte chunks wholly below n take one
    // vector load each (t0 is a multiple of 4, a chunk never crosses a pad)
    const uint32_t nv = vec ? L / 4u : 0u;
    for (uint32_t c = threadIdx.x; c < nv; c += NT) {
        const uint64_t g = t0 + 4u * c;
        u32x4 q;
        if (g + 4u <= n) {
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(x + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = g + k < n ? x[g + k] : Op::identity();
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) bufA[log_pad(4u * c + k)] = q[k];
    }
    for (uint32_t i = 4u * nv + threadIdx.x; i < L; i += NT) {
        const uint64_t g = t0 + i;
        bufA[log_pad(i)] = g < n ? x[g] : Op::identity();
    }
    __syncthreads();
    uint32_t p2 = 1;  // largest power of two not above w
    while (p2 * 2u <= w) p2 *= 2u;
    // Levels with shifts below RR in registers: a thread takes a run of RR
    // positions plus the RR - 1 after it and leaves m^(Q) of its run in bufB,
    // Q = min(p2, RR), on the positions [0, L - Q + 1) later levels read.
    const uint32_t q = p2 < (uint32_t)RR ? p2 : (uint32_t)RR;
    const uint32_t nq = L - q + 1u;
    for (uint32_t j = threadIdx.x; j * RR < nq; j += NT) {
        uint32_t v[2 * RR];
#pragma unroll
        for (int e = 0; e < 2 * RR; ++e) {
            const uint32_t p = j * RR + (uint32_t)e;
            v[e] = p < L ? bufA[log_pad(p)] : Op::identity();
        }
        if (q > 1u) log_level<Op, 1>(v);
        if (q > 2u) log_level<Op, 2>(v);
        if (q > 4u) log_level<Op, 4>(v);
        if (q > 8u) log_level<Op, 8>(v);
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            const uint32_t p = j * RR + (uint32_t)e;
            if (p < nq) bufB[log_pad(p)] = v[e];
        }
    }
    __syncthreads();
    // Levels with shifts of RR and more through LDS: windows of 2s on the
    // positions [0, L - 2s + 1).
    uint32_t* src = bufB;
    uint32_t* dst = bufA;
    for (uint32_t s = q; s < p2; s *= 2u) {
        const uint32_t len = L - 2u * s + 1u;
        for (uint32_t i = threadIdx.x; i < len; i += NT)
            dst[log_pad(i)] = Op::combine(src[log_pad(i)], src[log_pad(i + s)]);
        __syncthreads();
        uint32_t* t = src;
        src = dst;
        dst = t;
    }
    const uint32_t shift = w - p2;
    // outputs four at a time, one 16-byte store per full aligned chunk
    for (uint32_t c = threadIdx.x; 4u * c < tile; c += NT) {
        const uint64_t g = t0 + 4u * c;
        u32x4 r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = 4u * c + k;
            r[k] = Op::combine(src[log_pad(i)], src[log_pad(i + shift)]);
        }
        if (vec && g + 4u <= count) {
            __builtin_nontemporal_store(r, reinterpret_cast<u32x4*>(y + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (g + k < count) y[g + k] = r[k];
        }
    }
}

// Log path for w <= 1024, one wavefront per tile and no workgroup barrier.  A
// wave takes 64 R consecutive inputs with coalesced 16-byte loads, turns them
// around in its own LDS region so that each lane holds R consecutive ones, and
// runs the doubling levels 1, 2, 4, ... in registers: a level's shift of S
// positions reaches S / R lanes up, whose values come by shuffle, all taken
// before the level writes.  The windows of 2^L go back through the region and
// the last, runtime-length step reads them at i and i + (w - 2^L) while the
// outputs leave with coalesced stores.  Tiles overlap by the halo H = w - 1
// rounded up to 32, so a tile stores 64 R - H outputs; an output reads only
// inputs of its own tile (the wrapped values the last lanes receive feed only
// windows past the tile's share).
constexpr uint32_t kLogWaveSmall = 64;    // w <= this: R = 16
constexpr uint32_t kLogWaveMaxWindow = 1024;  // w <= this: R = 32

// LDS word of tile position i: runs of 16 at a stride of 20 words, so that the
// 16-byte accesses of a lane's run (and of 4 consecutive positions) stay
// aligned and spread over the banks.
__device__ __forceinline__ uint32_t log_wave_pad(uint32_t i) { return i + 4u * (i >> 4); }

template <class Op, int R, int S>
__device__ __forceinline__ void log_wave_step(uint32_t (&v)[R], int lane) {
    uint32_t r[R];
#pragma unroll
    for (int e = 0; e < R; ++e) {
        const int j = e + S;
        r[e] = j < R ? v[j] : shfl(v[j % R], lane, j / R);
    }
#pragma unroll
    for (int e = 0; e < R; ++e) v[e] = Op::combine(v[e], r[e]);
}

__host__ __device__ constexpr uint32_t log_wave_outputs(uint32_t inputs, uint32_t w) {
    // a multiple of 32 outputs, so that tiles meet on 128-byte line boundaries
    // (rounding to 16 left half lines shared by neighbouring tiles' stores and
    // measured 4-6% slower at w = 4 and 16)
    return inputs - ((w - 1u + 31u) & ~31u);
}

template <class Op, int R>
__global__ __launch_bounds__(256) void sliding_log_wave_kernel(const uint32_t* __restrict__ x,
                                                              uint64_t n, uint32_t w,
                                                              uint32_t* __restrict__ y,
                                                              uint64_t count, uint64_t ntiles,
                                                              int vec) {
    constexpr int NWV = 256 / kWave;
    constexpr uint32_t IN = kWave * R;  // inputs per wave tile
    constexpr int C = (int)IN / 256;    // coalesced 16-byte accesses per lane
    __shared__ __align__(16) uint32_t region[NWV][IN / 16 * 20];
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t tile = (uint64_t)blockIdx.x * NWV + (uint64_t)wv;
    if (tile >= ntiles) return;  // whole waves only; no workgroup barrier follows
    uint32_t* buf = region[wv];
    const uint32_t tw = log_wave_outputs(IN, w);
    const uint64_t t0 = tile * tw;
    // 1. coalesced loads: positions 256 c + 4 lane
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t i = 256u * c + 4u * lane;
        const uint64_t g = t0 + i;
        u32x4 q;
        if (vec && g + 4u <= n) {
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(x + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = g + k < n ? x[g + k] : Op::identity();
        }
        *reinterpret_cast<u32x4*>(buf + log_wave_pad(i)) = q;
    }
    wave_lds_sync();
    // 2. lane l takes positions R l .. R l + R - 1
    uint32_t v[R];
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
        const u32x4 q = *reinterpret_cast<const u32x4*>(buf + log_wave_pad(R * lane + 4u * c));
#pragma unroll
        for (int k = 0; k < 4; ++k) v[4 * c + k] = q[k];
    }
    // 3. levels 1, 2, 4, ... while 2s <= w
    uint32_t p2 = 1;
    if (2u <= w) { log_wave_step<Op, R, 1>(v, lane); p2 = 2; }
    if (4u <= w) { log_wave_step<Op, R, 2>(v, lane); p2 = 4; }
    if (8u <= w) { log_wave_step<Op, R, 4>(v, lane); p2 = 8; }
    if (16u <= w) { log_wave_step<Op, R, 8>(v, lane); p2 = 16; }
    if (32u <= w) { log_wave_step<Op, R, 16>(v, lane); p2 = 32; }
    if (64u <= w) { log_wave_step<Op, R, 32>(v, lane); p2 = 64; }
    if (R >= 32) {
        if (128u <= w) { log_wave_step<Op, R, 64>(v, lane); p2 = 128; }
        if (256u <= w) { log_wave_step<Op, R, 128>(v, lane); p2 = 256; }
        if (512u <= w) { log_wave_step<Op, R, 256>(v, lane); p2 = 512; }
        if (1024u <= w) { log_wave_step<Op, R, 512>(v, lane); p2 = 1024; }
    }
    // 4. the windows of p2 back into the region (the reads of step 2 are
    //    done: a wave's LDS operations complete in order)
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
        u32x4 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = v[4 * c + k];
        *reinterpret_cast<u32x4*>(buf + log_wave_pad(R * lane + 4u * c)) = q;
    }
    wave_lds_sync();
    // 5. y_i = m_i (+) m_{i + shift}, four consecutive outputs per lane and
    //    access (tw is a multiple of 32, so a group of four is all in or out)
    const uint32_t shift = w - p2;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t i = 256u * c + 4u * lane;
        if (i >= tw) continue;
        const uint64_t g = t0 + i;
        u32x4 q = *reinterpret_cast<const u32x4*>(buf + log_wave_pad(i));
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = Op::combine(q[k], buf[log_wave_pad(i + k + shift)]);
        if (vec && g + 4u <= count) {
            __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(y + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (g + k < count) y[g + k] = q[k];
        }
    }
}

template <class Op, int R>
static int launch_log_wave(const uint32_t* x, uint64_t n, uint32_t w, uint32_t* y, uint64_t count,
                           int vec, hipStream_t s) {
    const uint64_t tw = log_wave_outputs(kWave * R, w);
    const uint64_t ntiles = (count + tw - 1) / tw;
    const uint64_t blocks = (ntiles + 3) / 4;
    hipLaunchKernelGGL((sliding_log_wave_kernel<Op, R>), dim3((unsigned)blocks), dim3(256), 0, s,
                       x, n, w, y, count, ntiles, vec);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Prefix-difference path (+ only) for w <= 64, on the same one-wave tiles as
// the log path: 1024 inputs per wave turned around in LDS into runs of 16 per
// lane, tiles overlapping by the halo H = w - 1 rounded up to 32.  The running
// prefix P covers the tile (a common offset cancels in the difference); it
// goes back to the LDS region and y_i = P_{i+w-1} - P_{i-1} (P_{-1} = 0) leaves
// with coalesced stores.  (The block prefix/suffix form on these tiles was
// measured slower than the streaming kernel above and is not used.)
constexpr uint32_t kPrefixTileMaxWindow = 64;

__global__ __launch_bounds__(256) void sliding_prefix_tile_kernel(const uint32_t* __restrict__ x,
                                                                 uint64_t n, uint32_t w,
                                                                 uint32_t* __restrict__ y,
                                                                 uint64_t count, uint64_t ntiles,
                                                                 int vec) {
    constexpr int R = kLogRun;
    constexpr int NWV = 256 / kWave;
    constexpr uint32_t IN = kWave * R;  // inputs per wave tile
    constexpr int C = (int)IN / 256;    // coalesced 16-byte accesses per lane
    __shared__ __align__(16) uint32_t region[NWV][IN / 16 * 20];
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t tile = (uint64_t)blockIdx.x * NWV + (uint64_t)wv;
    if (tile >= ntiles) return;  // whole waves only; no workgroup barrier follows
    uint32_t* buf = region[wv];
    const uint32_t tw = log_wave_outputs(IN, w);
    const uint64_t t0 = tile * tw;
    // 1. coalesced loads: positions 256 c + 4 lane
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t i = 256u * c + 4u * lane;
        const uint64_t g = t0 + i;
        u32x4 q;
        if (vec && g + 4u <= n) {
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(x + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = g + k < n ? x[g + k] : 0u;
        }
        *reinterpret_cast<u32x4*>(buf + log_wave_pad(i)) = q;
    }
    wave_lds_sync();
    // 2. lane l takes positions R l .. R l + R - 1 and forms the tile prefix
    uint32_t v[R];
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
        const u32x4 q = *reinterpret_cast<const u32x4*>(buf + log_wave_pad(R * lane + 4u * c));
#pragma unroll
        for (int k = 0; k < 4; ++k) v[4 * c + k] = q[k];
    }
    slab_prefix<OpAdd, R>(v, (HeadMask<R>)0, (uint32_t)kWave, lane, 0u);
    // 3. back into LDS (the reads of step 2 are done: a wave's LDS operations
    //    complete in order)
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
        u32x4 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k] = v[4 * c + k];
        *reinterpret_cast<u32x4*>(buf + log_wave_pad(R * lane + 4u * c)) = q;
    }
    wave_lds_sync();
    // 4. four consecutive outputs per lane and access (tw is a multiple of 32)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const uint32_t i = 256u * c + 4u * lane;
        if (i >= tw) continue;
        const uint64_t g = t0 + i;
        u32x4 q;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t before = i + k == 0u ? 0u : buf[log_wave_pad(i + k - 1u)];
            q[k] = buf[log_wave_pad(i + k + w - 1u)] - before;
        }
        if (vec && g + 4u <= count) {
            __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(y + g));
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (g + k < count) y[g + k] = q[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Scalar-input path (Alg. 1 of Sec. 3.1), w <= 64, any associative operator.
//
// A vector of G lanes (G = 16 for w <= 16, four such vectors per wavefront,
// one per 16-lane row; else G = 64) streams a run of outputs.  Lane l < w
// holds Y[l]; before input x_i arrives, Y[l] = x_{i-w+1+l} (+) ... (+)
// x_{i-1} (lanes l >= w - 1 hold the identity).  Each input is broadcast to
// lanes 0 .. w-1 and added on the right (Y stays the left operand), lane 0
// then holds the window x_{i-w+1} .. x_i, and Y moves down one lane.  The first
// w - 1 inputs of the run only fill Y, which gives exactly the initial suffix
// sums of Alg. 1.  Inputs come in G at a time (one per lane); the outputs of
// G steps are collected by shifting them in at lane 0 and leave as one store.
// The moves are DPP lane shifts (row-wise for G = 16, wave-wide for G = 64).
// ---------------------------------------------------------------------------
constexpr uint32_t kScalarRun = 4096;  // outputs per vector

template <int G>
struct ScalarLanes;
template <>
struct ScalarLanes<16> {  // 16-lane rows
    static constexpr int kDown = 0x101, kUp = 0x111;  // row_shl:1, row_shr:1
    template <int K>
    static __device__ __forceinline__ uint32_t bcast(uint32_t v) {  // row_newbcast:K
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + K, 0xF, 0xF, false);
    }
};
template <>
struct ScalarLanes<64> {  // the whole wavefront
    static constexpr int kDown = 0x130, kUp = 0x138;  // wave_shl:1, wave_shr:1
    template <int K>
    static __device__ __forceinline__ uint32_t bcast(uint32_t v) {
        return (uint32_t)__builtin_amdgcn_readlane((int)v, K);
    }
};

// lane l takes lane l + 1 (DOWN) or l - 1 (UP) of its vector; the lane with
// no source keeps `keep`
template <int CTRL>
__device__ __forceinline__ uint32_t lane_move(uint32_t v, uint32_t keep) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)keep, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint2 lane_move(uint2 v, uint2 keep) {
    return make_uint2(lane_move<CTRL>(v.x, keep.x), lane_move<CTRL>(v.y, keep.y));
}
template <class L, int K>
__device__ __forceinline__ uint32_t lane_bcast(uint32_t v) { return L::template bcast<K>(v); }
template <class L, int K>
__device__ __forceinline__ uint2 lane_bcast(uint2 v) {
    return make_uint2(L::template bcast<K>(v.x), L::template bcast<K>(v.y));
}

template <class Op, int G, int K>
__device__ __forceinline__ void scalar_step(typename Op::T& Y, typename Op::T& ov,
                                            typename Op::T xv, bool in_window,
                                            typename Op::T ident) {
    using L = ScalarLanes<G>;
    const typename Op::T xi = lane_bcast<L, K>(xv);
    Y = in_window ? Op::combine(Y, xi) : ident;
    ov = lane_move<L::kUp>(ov, Y);     // lane 0 takes this step's window
    Y = lane_move<L::kDown>(Y, ident);
}

template <class Op, int G, int... K>
__device__ __forceinline__ void scalar_block(typename Op::T& Y, typename Op::T& ov,
                                             typename Op::T xv, bool in_window,
                                             typename Op::T ident,
                                             std::integer_sequence<int, K...>) {
    (scalar_step<Op, G, K>(Y, ov, xv, in_window, ident), ...);
}

template <class Op, int G>
__global__ __launch_bounds__(256) void sliding_scalar_kernel(const typename Op::T* __restrict__ x,
                                                             uint64_t n, uint32_t w,
                                                             typename Op::T* __restrict__ y,
                                                             uint64_t count) {
    using T = typename Op::T;
    constexpr int NV = kWave / G;  // vectors per wavefront
    const int lane = lane_id();
    const int j = lane % G;        // lane within the vector
    const uint64_t v = ((uint64_t)blockIdx.x * 4 + (uint64_t)wave_id()) * NV + (uint64_t)(lane / G);
    const uint64_t o0 = v * kScalarRun;
    // every vector of a wavefront takes the same number of steps; a vector
    // past the end computes nothing that is stored
    const uint64_t o0w = ((uint64_t)blockIdx.x * 4 + (uint64_t)wave_id()) * NV * kScalarRun;
    if (o0w >= count) return;
    const uint64_t o1 = o0 + kScalarRun < count ? o0 + kScalarRun : (o0 < count ? count : o0);
    const uint64_t iend = o1 + w - 1 <= n ? o1 + w - 1 : n;  // this vector's inputs o0 .. iend - 1
    const uint64_t steps = kScalarRun + w - 1;
    const T ident = Op::identity();
    const bool in_window = (uint32_t)j < w;
    T Y = ident, ov = ident;
    for (uint64_t t = 0; t < steps; t += G) {
        const uint64_t gi = o0 + t + (uint64_t)j;
        const T xv = gi < iend ? x[gi] : ident;
        scalar_block<Op, G>(Y, ov, xv, in_window, ident, std::make_integer_sequence<int, G>());
        // lane j holds the window that ended at input o0 + t + G - 1 - j
        const uint64_t last = o0 + t + (uint64_t)(G - 1 - j);  // its last input
        if (last + 1 >= o0 + w) {
            const uint64_t oi = last + 1 - w;                   // its output index
            if (oi < o1) y[oi] = ov;
        }
    }
}

template <class Op>
static int launch_scalar(const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                         hipStream_t s) {
    using T = typename Op::T;
    const uint64_t vecs = (count + kScalarRun - 1) / kScalarRun;
    if (w <= 16u) {
        const uint64_t blocks = (vecs + 15) / 16;  // 4 vectors per wave, 4 waves per block
        hipLaunchKernelGGL((sliding_scalar_kernel<Op, 16>), dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const T*>(x), n, w, static_cast<T*>(y), count);
    } else {
        const uint64_t blocks = (vecs + 3) / 4;
        hipLaunchKernelGGL((sliding_scalar_kernel<Op, 64>), dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const T*>(x), n, w, static_cast<T*>(y), count);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

uint32_t scalar_max_window() { return kWave; }

int launch_sliding_scalar(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                          hipStream_t s) {
    switch (op) {
    case kOpAdd: return launch_scalar<OpAdd>(x, n, w, y, count, s);
    case kOpMin: return launch_scalar<OpMin>(x, n, w, y, count, s);
    case kOpMax: return launch_scalar<OpMax>(x, n, w, y, count, s);
    case kOpAffine: return launch_scalar<OpAffine>(x, n, w, y, count, s);
    default: return -2;
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
constexpr uint64_t kDefaultSlidingWaves = 256ull * 128ull;  // 128 per compute unit
// Windows from this length load their halo early (EARLY_HALO).  At n = 2^28,
// timed per call (fraction of HBM peak): w = 1024, + (the prefix-difference
// form) 0.675 -> 0.74, min and max 0.67 -> 0.73; + at w = 768 0.69 -> 0.73;
// w = 128 and 256 0.71 -> 0.72, max at w = 384 0.70 -> 0.71; affine (8-pair
// runs) at w = 128 and 256 0.71 -> 0.73.  Four waves per workgroup (more
// neighbours sharing a CU) measured no better than two.  Affine above w = 512
// (241 VGPRs at R = 16) has no room for the halo's registers.
constexpr uint32_t kEarlyHaloMinW = 128;

template <class Op, int R, int WAVES, bool PFX = false, bool EARLY_HALO = false>
static int launch_generic(const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                          uint64_t target_waves, hipStream_t s) {
    using T = typename Op::T;
    constexpr uint64_t S = kWave * R;
    const uint64_t total_slabs = (count + S - 1) / S;
    const uint64_t tw = target_waves ? target_waves : kDefaultSlidingWaves;
    uint64_t spw = (total_slabs + tw - 1) / tw;
    if (spw < 1) spw = 1;
    const uint64_t waves = (total_slabs + spw - 1) / spw;
    const uint64_t blocks = (waves + WAVES - 1) / WAVES;
    const int vec = (((uintptr_t)x | (uintptr_t)y) & 15u) == 0 ? 1 : 0;
    const uint32_t rows = ring_rows<R>(w);
    const size_t lds = (size_t)WAVES * rows * (R + 1) * sizeof(T);
    hipLaunchKernelGGL((sliding_generic_kernel<Op, R, WAVES, PFX, EARLY_HALO>), dim3((unsigned)blocks),
                       dim3(WAVES * kWave), lds, s, static_cast<const T*>(x), n, w,
                       static_cast<T*>(y), count, total_slabs, spw, vec, rows);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class Op>
static int launch_log(const void* x, uint64_t n, uint32_t w, void* y, uint64_t count, hipStream_t s) {
    const int vec = (((uintptr_t)x | (uintptr_t)y) & 15u) == 0 ? 1 : 0;
    const uint32_t* xi = static_cast<const uint32_t*>(x);
    uint32_t* yo = static_cast<uint32_t*>(y);
    if (w <= kLogWaveSmall) return launch_log_wave<Op, 16>(xi, n, w, yo, count, vec, s);
    if (w <= kLogWaveMaxWindow) return launch_log_wave<Op, 32>(xi, n, w, yo, count, vec, s);
    constexpr int NT = 256;
    // two padded buffers of tile + w - 1 words within 64 KB
    const uint32_t tile = w <= 2048u ? 4096u : 2048u;
    const uint64_t L = tile + w - 1ull;
    const size_t lds = 2ull * (L + L / 16 + 1ull) * sizeof(uint32_t);
    const uint64_t blocks = (count + tile - 1) / tile;
    hipLaunchKernelGGL((sliding_log_kernel<Op, NT>), dim3((unsigned)blocks), dim3(NT), lds, s,
                       static_cast<const uint32_t*>(x), n, w, static_cast<uint32_t*>(y), count, tile,
                       vec);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Elements per lane and waves per workgroup: a window must fit in one slab of
// 64 * R elements; LDS per wave is the ring of two slab regions plus the
// repeated rows (the staging area lives in whichever region is free).
uint32_t generic_max_window() { return kWave * 32; }

// A tile of 2048 outputs plus a halo of w-1 in two padded LDS buffers stays
// within 64 KB.
uint32_t log_max_window() { return 4096; }

int launch_sliding_generic(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                           uint64_t tw, hipStream_t s) {
    // Default wave counts, measured at n = 2^28: 32768 for the 4-byte
    // operators (fewer, longer streams lose more to the last partial round of
    // waves than they save on halos); AFFINE with w <= 512 (8-element lane
    // runs, more waves resident) 65536: 0.72 of HBM peak at w = 4 .. 64 and
    // 0.71 at w = 256, against 0.68 and 0.67 with 32768.
    if (tw == 0) tw = (op == kOpAffine && w <= 512u) ? 2 * kDefaultSlidingWaves : kDefaultSlidingWaves;
    // <Op, R, waves per workgroup>
    const bool big = w > (uint32_t)(kWave * 16);
    const bool early = w >= kEarlyHaloMinW;
    switch (op) {
    case kOpAdd: return big ? launch_generic<OpAdd, 32, 1>(x, n, w, y, count, tw, s)
                     : early ? launch_generic<OpAdd, 16, 2, false, true>(x, n, w, y, count, tw, s)
                            : launch_generic<OpAdd, 16, 2>(x, n, w, y, count, tw, s);
    case kOpMin: return big ? launch_generic<OpMin, 32, 1>(x, n, w, y, count, tw, s)
                     : early ? launch_generic<OpMin, 16, 2, false, true>(x, n, w, y, count, tw, s)
                            : launch_generic<OpMin, 16, 2>(x, n, w, y, count, tw, s);
    case kOpMax: return big ? launch_generic<OpMax, 32, 1>(x, n, w, y, count, tw, s)
                     : early ? launch_generic<OpMax, 16, 2, false, true>(x, n, w, y, count, tw, s)
                            : launch_generic<OpMax, 16, 2>(x, n, w, y, count, tw, s);
    case kOpAffine:
        if (big) return launch_generic<OpAffine, 32, 1>(x, n, w, y, count, tw, s);
        if (w > (uint32_t)(kWave * 8)) return launch_generic<OpAffine, 16, 1>(x, n, w, y, count, tw, s);
        return early ? launch_generic<OpAffine, 8, 2, false, true>(x, n, w, y, count, tw, s)
                     : launch_generic<OpAffine, 8, 2>(x, n, w, y, count, tw, s);
    default: return -2;
    }
}

// The prefix-difference form, + only (the one invertible operator here).
int launch_sliding_prefix(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                          uint64_t tw, hipStream_t s) {
    if (op != kOpAdd) return -2;
    if (w <= kPrefixTileMaxWindow) {  // one-wave tiles
        const int vec = (((uintptr_t)x | (uintptr_t)y) & 15u) == 0 ? 1 : 0;
        const uint64_t tw = log_wave_outputs(kWave * kLogRun, w);
        const uint64_t ntiles = (count + tw - 1) / tw;
        hipLaunchKernelGGL(sliding_prefix_tile_kernel, dim3((unsigned)((ntiles + 3) / 4)),
                           dim3(256), 0, s, static_cast<const uint32_t*>(x), n, w,
                           static_cast<uint32_t*>(y), count, ntiles, vec);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    if (w > (uint32_t)(kWave * 16)) return launch_generic<OpAdd, 32, 1, true>(x, n, w, y, count, tw, s);
    if (w >= kEarlyHaloMinW) return launch_generic<OpAdd, 16, 2, true, true>(x, n, w, y, count, tw, s);
    return launch_generic<OpAdd, 16, 2, true>(x, n, w, y, count, tw, s);
}

// ---------------------------------------------------------------------------
// Wide windows (w above one slab, any length).  The segments of the generic
// path, [a w, (a+1) w), are now longer than a slab.  The window starting at
// offset o of segment A = a is A's suffix from o followed by the prefix of
// B = a + 1 up to offset o - 1:
//     y_{a w + o} = Sf_A(o) (+) Pf_B(o - 1),     Pf_B(-1) = the identity,
// so both operands sit at the same offset.  With chunks of T = 2048 offsets:
//   1. wide_chunk_sum: the sum of every chunk (a, c);
//   2. wide_chunk_scan: per segment, the sum of the chunks after c (for A's
//      suffixes) and before c (for B's prefixes);
//   3. wide_out: output chunk (a, c) = in-chunk suffixes of A's chunk c with
//      the later chunks' sum, in-chunk exclusive prefixes of B's chunk c after
//      the earlier chunks' sum.
// HBM: x read three times, y written once, plus 3 values per chunk.
// ---------------------------------------------------------------------------
constexpr int kWideNT = 256;
constexpr int kWidePer = 8;
constexpr uint32_t kWideChunk = kWideNT * kWidePer;  // offsets per chunk

struct WideGeom {
    uint64_t n, w, count;
    uint64_t nseg;  // segments holding input: ceil(n / w)
    uint64_t nch;   // chunks per segment: ceil(w / T)
};

// LDS slot of element e of a chunk: one pad word per eight elements, so that
// a thread's run of eight (read across lanes) hits distinct banks.
__device__ __forceinline__ uint32_t wide_slot(uint32_t e) { return e + e / kWidePer; }

// Chunk c of segment a into the thread's run of kWidePer consecutive
// elements (coalesced loads, turned around in LDS); elements outside the
// segment or past n read as the identity.
template <class Op>
__device__ __forceinline__ void wide_load(const typename Op::T* __restrict__ x, const WideGeom& g,
                                          uint64_t a, uint64_t c, typename Op::T* buf,
                                          typename Op::T (&v)[kWidePer]) {
    using T = typename Op::T;
    const uint64_t seg0 = a * g.w;
    const uint64_t off0 = c * kWideChunk;
#pragma unroll
    for (int k = 0; k < kWidePer; ++k) {
        const uint32_t e = (uint32_t)k * kWideNT + threadIdx.x;
        const uint64_t o = off0 + e;
        const uint64_t i = seg0 + o;
        buf[wide_slot(e)] = (o < g.w && i < g.n) ? x[i] : Op::identity();
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kWidePer; ++j) v[j] = buf[wide_slot(threadIdx.x * kWidePer + j)];
    __syncthreads();
    (void)sizeof(T);
}

// Workgroup-wide ordered scans of the threads' totals (thread order = element
// order).  excl: the sum of all earlier threads; after: of all later ones.
template <class Op>
__device__ __forceinline__ typename Op::T wide_excl_before(typename Op::T t, typename Op::T* part) {
    using T = typename Op::T;
    const int lane = lane_id(), wv = wave_id();
    T incl = t;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T o = shfl(incl, lane, -d);
        if (lane >= d) incl = Op::combine(o, incl);
    }
    T before = shfl(incl, lane, -1);
    if (lane == kWave - 1) part[wv] = incl;
    __syncthreads();
    T wpre = Op::identity();
    for (int q = 0; q < wv; ++q) wpre = Op::combine(wpre, part[q]);
    before = lane == 0 ? wpre : Op::combine(wpre, before);
    __syncthreads();
    return before;
}

template <class Op>
__device__ __forceinline__ typename Op::T wide_excl_after(typename Op::T t, typename Op::T* part) {
    using T = typename Op::T;
    const int lane = lane_id(), wv = wave_id();
    T incl = t;  // t (+) the later lanes of the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T o = shfl(incl, lane, d);
        if (lane + d < kWave) incl = Op::combine(incl, o);
    }
    T after = shfl(incl, lane, 1);
    if (lane == 0) part[wv] = incl;
    __syncthreads();
    T wsuf = Op::identity();
    for (int q = kWideNT / kWave - 1; q > wv; --q) wsuf = Op::combine(part[q], wsuf);
    after = lane == kWave - 1 ? wsuf : Op::combine(after, wsuf);
    __syncthreads();
    return after;
}

// 1. sums[a * nch + c] = the sum of chunk c of segment a
template <class Op>
__global__ __launch_bounds__(kWideNT) void wide_chunk_sum_kernel(const typename Op::T* __restrict__ x,
                                                                  WideGeom g,
                                                                  typename Op::T* __restrict__ sums) {
    using T = typename Op::T;
    __shared__ T buf[kWideChunk + kWideChunk / kWidePer];
    __shared__ T part[kWideNT / kWave];
    const uint64_t a = blockIdx.x / g.nch, c = blockIdx.x % g.nch;
    T v[kWidePer];
    wide_load<Op>(x, g, a, c, buf, v);
    T t = v[0];
#pragma unroll
    for (int j = 1; j < kWidePer; ++j) t = Op::combine(t, v[j]);
    const T before = wide_excl_before<Op>(t, part);
    if (threadIdx.x == kWideNT - 1) sums[blockIdx.x] = Op::combine(before, t);
}

// 2. per segment (one workgroup): pre[a][c] = sum of chunks 0 .. c-1,
//    post[a][c] = sum of chunks c+1 .. nch-1
template <class Op>
__global__ __launch_bounds__(kWideNT) void wide_chunk_scan_kernel(
    const typename Op::T* __restrict__ sums, WideGeom g, typename Op::T* __restrict__ pre,
    typename Op::T* __restrict__ post) {
    using T = typename Op::T;
    __shared__ T part[kWideNT / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * g.nch;
    T carry = Op::identity();
    for (uint64_t c0 = 0; c0 < g.nch; c0 += kWideNT) {
        const uint64_t c = c0 + threadIdx.x;
        const T t = c < g.nch ? sums[base + c] : Op::identity();
        const T before = wide_excl_before<Op>(t, part);
        if (c < g.nch) pre[base + c] = Op::combine(carry, before);
        // the block's total: before (+) t of its last thread
        __shared__ T total;
        if (threadIdx.x == kWideNT - 1) total = Op::combine(before, t);
        __syncthreads();
        carry = Op::combine(carry, total);
        __syncthreads();
    }
    carry = Op::identity();
    for (uint64_t e0 = 0; e0 < g.nch; e0 += kWideNT) {
        // blocks from the end: c = nch - 1 - e0 - (NT - 1 - tid) keeps thread order = chunk order
        const int64_t c = (int64_t)g.nch - 1 - (int64_t)e0 - (int64_t)(kWideNT - 1 - threadIdx.x);
        const T t = c >= 0 ? sums[base + (uint64_t)c] : Op::identity();
        const T after = wide_excl_after<Op>(t, part);
        if (c >= 0) post[base + (uint64_t)c] = Op::combine(after, carry);
        __shared__ T total;
        if (threadIdx.x == 0) total = Op::combine(t, after);
        __syncthreads();
        carry = Op::combine(total, carry);
        __syncthreads();
    }
}

// 3. outputs y_{a w + o} for the offsets o of chunk c
template <class Op>
__global__ __launch_bounds__(kWideNT) void wide_out_kernel(const typename Op::T* __restrict__ x,
                                                           WideGeom g,
                                                           const typename Op::T* __restrict__ pre,
                                                           const typename Op::T* __restrict__ post,
                                                           typename Op::T* __restrict__ y) {
    using T = typename Op::T;
    __shared__ T buf[kWideChunk + kWideChunk / kWidePer];
    __shared__ T part[kWideNT / kWave];
    const uint64_t a = blockIdx.x / g.nch, c = blockIdx.x % g.nch;
    const uint64_t out0 = a * g.w + c * kWideChunk;  // first output of the chunk
    if (out0 >= g.count) return;                        // uniform over the workgroup
    // A's chunk: inclusive suffixes inside the chunk, then the later chunks
    T va[kWidePer];
    wide_load<Op>(x, g, a, c, buf, va);
#pragma unroll
    for (int j = kWidePer - 2; j >= 0; --j) va[j] = Op::combine(va[j], va[j + 1]);
    const T after = wide_excl_after<Op>(va[0], part);
    const T tail = Op::combine(after, post[a * g.nch + c]);
#pragma unroll
    for (int j = 0; j < kWidePer; ++j) va[j] = Op::combine(va[j], tail);
    // B's chunk: exclusive prefixes inside the chunk after the earlier chunks
    T vb[kWidePer];
    const bool has_b = a + 1 < g.nseg;
    if (has_b) {
        wide_load<Op>(x, g, a + 1, c, buf, vb);
    } else {
#pragma unroll
        for (int j = 0; j < kWidePer; ++j) vb[j] = Op::identity();
    }
    T run = vb[0];
#pragma unroll
    for (int j = 1; j < kWidePer; ++j) {
        const T nx = Op::combine(run, vb[j]);
        vb[j] = run;  // exclusive inside the thread
        run = nx;
    }
    vb[0] = Op::identity();
    const T before = wide_excl_before<Op>(run, part);
    const T head = has_b ? Op::combine(pre[(a + 1) * g.nch + c], before) : Op::identity();
    // y = Sf_A (+) Pf_B, staged through LDS for coalesced stores
#pragma unroll
    for (int j = 0; j < kWidePer; ++j)
        buf[wide_slot(threadIdx.x * kWidePer + j)] = Op::combine(va[j], Op::combine(head, vb[j]));
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWidePer; ++k) {
        const uint32_t e = (uint32_t)k * kWideNT + threadIdx.x;
        const uint64_t o = c * kWideChunk + e;
        const uint64_t i = a * g.w + o;
        if (o < g.w && i < g.count) y[i] = buf[wide_slot(e)];
    }
}

uint64_t wide_workspace_bytes(int op, uint64_t n, uint64_t w) {
    const uint64_t esz = op == kOpAffine ? 8 : 4;
    const uint64_t nseg = (n + w - 1) / w, nch = (w + kWideChunk - 1) / kWideChunk;
    const uint64_t one = (nseg * nch * esz + 255) & ~255ull;
    return 3 * one;
}

template <class Op>
static int launch_wide_op(const void* x, uint64_t n, uint64_t w, void* y, uint64_t count,
                          void* workspace, hipStream_t s) {
    using T = typename Op::T;
    WideGeom g;
    g.n = n;
    g.w = w;
    g.count = count;
    g.nseg = (n + w - 1) / w;
    g.nch = (w + kWideChunk - 1) / kWideChunk;
    const uint64_t one = (g.nseg * g.nch * sizeof(T) + 255) & ~255ull;
    T* sums = static_cast<T*>(workspace);
    T* pre = reinterpret_cast<T*>(static_cast<uint8_t*>(workspace) + one);
    T* post = reinterpret_cast<T*>(static_cast<uint8_t*>(workspace) + 2 * one);
    const T* xt = static_cast<const T*>(x);
    const dim3 grid((unsigned)(g.nseg * g.nch)), block(kWideNT);
    hipLaunchKernelGGL((wide_chunk_sum_kernel<Op>), grid, block, 0, s, xt, g, sums);
    hipLaunchKernelGGL((wide_chunk_scan_kernel<Op>), dim3((unsigned)g.nseg), block, 0, s, sums, g,
                       pre, post);
    // output chunks: segments that hold an output (a w <= count - 1)
    const uint64_t nout = (count - 1) / w + 1;
    hipLaunchKernelGGL((wide_out_kernel<Op>), dim3((unsigned)(nout * g.nch)), block, 0, s, xt, g,
                       pre, post, static_cast<T*>(y));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sliding_wide(int op, const void* x, uint64_t n, uint64_t w, void* y, uint64_t count,
                        void* workspace, hipStream_t s) {
    switch (op) {
    case kOpAdd: return launch_wide_op<OpAdd>(x, n, w, y, count, workspace, s);
    case kOpMin: return launch_wide_op<OpMin>(x, n, w, y, count, workspace, s);
    case kOpMax: return launch_wide_op<OpMax>(x, n, w, y, count, workspace, s);
    case kOpAffine: return launch_wide_op<OpAffine>(x, n, w, y, count, workspace, s);
    default: return -2;
    }
}

int launch_sliding_log(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                       hipStream_t s) {
    switch (op) {
    case kOpMin: return launch_log<OpMin>(x, n, w, y, count, s);
    case kOpMax: return launch_log<OpMax>(x, n, w, y, count, s);
    default: return -2;
    }
}

}  // namespace sws
