// sws_device.hpp -- device-side building blocks shared by the libsws kernels:
// the associative operators of the sliding sum (Sec. 2.2 / Sec. 3.1) and
// 64-lane wavefront data movement.  gfx950 only: wave64, LDS, no MFMA.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sws {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Operators.  combine(l, r) always takes the earlier operand on the left, so
// non-commutative operators (AFFINE) keep the order of Eq. 2.
// ---------------------------------------------------------------------------
struct OpAdd {
    using T = uint32_t;
    static __device__ __forceinline__ T identity() { return 0u; }
    static __device__ __forceinline__ T combine(T l, T r) { return l + r; }
};
struct OpMin {
    using T = uint32_t;
    static __device__ __forceinline__ T identity() { return 0xFFFFFFFFu; }
    static __device__ __forceinline__ T combine(T l, T r) { return l < r ? l : r; }
};
struct OpMax {
    using T = uint32_t;
    static __device__ __forceinline__ T identity() { return 0u; }
    static __device__ __forceinline__ T combine(T l, T r) { return l > r ? l : r; }
};
// Affine maps z -> a*z + b mod 2^32; (a,b) (+) (c,d) = (a*c, a*d + b).
struct OpAffine {
    using T = uint2;
    static __device__ __forceinline__ T identity() { return make_uint2(1u, 0u); }
    static __device__ __forceinline__ T combine(T l, T r) {
        return make_uint2(l.x * r.x, l.x * r.y + l.y);
    }
};

// ---------------------------------------------------------------------------
// Lane shuffles over the whole wave (ds_bpermute).  Out-of-range sources are
// the caller's to mask.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t shfl_idx(uint32_t v, int src_lane) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}
__device__ __forceinline__ uint32_t shfl(uint32_t v, int lane, int delta) {
    return shfl_idx(v, (lane + delta) & (kWave - 1));
}
__device__ __forceinline__ uint2 shfl(uint2 v, int lane, int delta) {
    return make_uint2(shfl(v.x, lane, delta), shfl(v.y, lane, delta));
}

// Inclusive prefix sum over the wave's 64 lanes by DPP: four row shifts sum
// within each row of 16 lanes, then two row broadcasts carry row totals
// forward (lane 15 into row 1, lane 47 into row 3, then lane 31 into rows 2
// and 3).  Each step is one VALU add with a DPP source.  Every lane of the
// wave must be active.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// A minimizer key: 64-bit value (hash or k-mer) split in two words, and a tag
// holding the position inside the tile (bits 0..14) and an invalid flag
// (bit 15).
struct Key {
    uint32_t lo, hi, tag;
};
__device__ __forceinline__ Key shfl(Key v, int lane, int delta) {
    Key r;
    r.lo = shfl(v.lo, lane, delta);
    r.hi = shfl(v.hi, lane, delta);
    r.tag = shfl(v.tag, lane, delta);
    return r;
}

// Value of v in lane `src` (uniform result).
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ uint2 lane_value(uint2 v, int src) {
    return make_uint2(lane_value(v.x, src), lane_value(v.y, src));
}

__device__ __forceinline__ uint64_t lane_value_u64(uint64_t v, int src) {
    return ((uint64_t)lane_value((uint32_t)(v >> 32), src) << 32) | lane_value((uint32_t)v, src);
}

__device__ __forceinline__ Key lane_value(Key v, int src) {
    Key r;
    r.lo = lane_value(v.lo, src);
    r.hi = lane_value(v.hi, src);
    r.tag = lane_value(v.tag, src);
    return r;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Orders this wave's LDS accesses: the compiler may not move LDS operations
// across it, and the wave waits for its outstanding LDS operations.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of the calling wavefront in its workgroup, as a wave-uniform (scalar)
// value, so that loops and branches derived from it stay scalar.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

}  // namespace sws
