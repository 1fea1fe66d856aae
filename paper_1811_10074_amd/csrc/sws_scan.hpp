// sws_scan.hpp -- per-wavefront segmented prefix/suffix scans and vector
// loads/stores of "runs" (R consecutive elements per lane), shared by the
// sliding-sum and minimizer kernels.
//
// Segments of length w start at every index that is a multiple of w.  A lane
// holds R consecutive elements; m0 is the first one's index mod w.  The scans
// are exact for any associative operator: combine(l, r) always receives the
// earlier operand on the left.
#pragma once

#include "sws_device.hpp"

#include <type_traits>

namespace sws {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class T, int R>
__device__ __forceinline__ void load_run(const T* __restrict__ x, uint64_t n, uint64_t p, bool vec,
                                         T identity, T (&v)[R]) {
    constexpr int kVec = (int)(R * sizeof(T) / 16);
    if (vec && p + R <= n) {
        const u32x4* src = reinterpret_cast<const u32x4*>(x + p);
        u32x4 q[kVec];
#pragma unroll
        for (int i = 0; i < kVec; ++i) q[i] = __builtin_nontemporal_load(src + i);
        const T* t = reinterpret_cast<const T*>(q);
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = t[e];
    } else {
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = (p + e < n) ? x[p + e] : identity;
    }
}

template <class T, int R>
__device__ __forceinline__ void store_run(T* __restrict__ y, uint64_t limit, uint64_t p, bool vec,
                                          const T (&v)[R]) {
    constexpr int kVec = (int)(R * sizeof(T) / 16);
    if (vec && p + R <= limit) {
        u32x4* dst = reinterpret_cast<u32x4*>(y + p);
        const u32x4* q = reinterpret_cast<const u32x4*>(v);
#pragma unroll
        for (int i = 0; i < kVec; ++i) __builtin_nontemporal_store(q[i], dst + i);
    } else {
#pragma unroll
        for (int e = 0; e < R; ++e)
            if (p + e < limit) y[p + e] = v[e];
    }
}

// Head bits of a lane's run of R elements: bit e (e < R) is set when element
// e starts a segment, bit R when the element after the run does (so the run's
// last element ends one).  Element e ends a segment exactly when bit e + 1 is
// set, so one mask serves both scans.  32 bits hold it for R < 32.
template <int R>
using HeadMask = typename std::conditional<(R < 32), uint32_t, uint64_t>::type;

template <int R>
__device__ __forceinline__ bool head_bit(HeadMask<R> h, int e) {
    return (h >> e) & 1u;
}

// Bits at every multiple of w in [0, R]: shifted by a lane's first head offset
// it gives the lane's head bits.
template <int R>
__device__ __forceinline__ HeadMask<R> head_pattern(uint32_t w) {
    HeadMask<R> p = 0;
    for (uint32_t j = 0; j <= (uint32_t)R; j += w) p |= (HeadMask<R>)1 << j;
    return p;
}

// Head bits of a lane whose first element has index m0 mod w.
template <int R>
__device__ __forceinline__ HeadMask<R> lane_heads(uint32_t m0, uint32_t w, HeadMask<R> pat) {
    const uint32_t f = m0 == 0u ? 0u : w - m0;  // offset of the first head
    const HeadMask<R> span = (HeadMask<R>)(((HeadMask<R>)2 << R) - 1u);  // bits 0..R
    return f <= (uint32_t)R ? (HeadMask<R>)((pat << f) & span) : (HeadMask<R>)0;
}

// In-segment prefix sums of one slab.  h: the lane's head bits.
// carry = prefix at the last element of the previous slab (identity if none).
template <class Op, int R>
__device__ __forceinline__ void slab_prefix(typename Op::T (&v)[R], HeadMask<R> h, uint32_t span,
                                            int lane, typename Op::T carry) {
    using T = typename Op::T;
#pragma unroll
    for (int e = 1; e < R; ++e)
        if (!head_bit<R>(h, e)) v[e] = Op::combine(v[e - 1], v[e]);
    // segmented inclusive scan of (has head, value) across lanes
    const HeadMask<R> inside = (HeadMask<R>)(((HeadMask<R>)1 << R) - 1u);
    uint32_t F = (h & inside) != 0u;
    T V = v[R - 1];
    for (uint32_t d = 1; d < span; d <<= 1) {
        const uint32_t Fo = shfl(F, lane, -(int)d);
        const T Vo = shfl(V, lane, -(int)d);
        if (lane >= (int)d && !F) {
            V = Op::combine(Vo, V);
            F = Fo;
        }
    }
    const uint32_t Fe = shfl(F, lane, -1);
    const T Ve = shfl(V, lane, -1);
    T c = carry;
    if (lane > 0) c = Fe ? Ve : Op::combine(carry, Ve);
    // the elements before the lane's first head extend the carried segment
    const int first = (int)(R < 32 ? __builtin_ctz((uint32_t)h | (1u << (R & 31)))
                                   : __builtin_ctzll((uint64_t)h | (1ull << (R & 63))));
#pragma unroll
    for (int e = 0; e < R; ++e)
        if (e < first) v[e] = Op::combine(c, v[e]);
}

// In-segment suffix sums of one slab, without the part of the last segment
// that lies in the next slab (patched by the caller).  h: the lane's head bits.
template <class Op, int R>
__device__ __forceinline__ void slab_suffix(typename Op::T (&v)[R], HeadMask<R> h, uint32_t span,
                                            int lane) {
    using T = typename Op::T;
#pragma unroll
    for (int e = R - 2; e >= 0; --e)
        if (!head_bit<R>(h, e + 1)) v[e] = Op::combine(v[e], v[e + 1]);
    const HeadMask<R> ends = h >> 1;  // bit e: element e ends a segment
    uint32_t G = ends != 0u;
    T U = v[0];
    for (uint32_t d = 1; d < span; d <<= 1) {
        const uint32_t Go = shfl(G, lane, (int)d);
        const T Uo = shfl(U, lane, (int)d);
        if (lane + (int)d < kWave && !G) {
            U = Op::combine(U, Uo);
            G = Go;
        }
    }
    const T Ue = shfl(U, lane, 1);
    if (lane < kWave - 1) {
        // elements after the lane's last segment end continue into lane+1
        const int after = ends == 0u ? 0
                          : (R < 32 ? 32 - __builtin_clz((uint32_t)ends)
                                    : 64 - __builtin_clzll((uint64_t)ends));
#pragma unroll
        for (int e = 0; e < R; ++e)
            if (e >= after) v[e] = Op::combine(v[e], Ue);
    }
}

}  // namespace sws
