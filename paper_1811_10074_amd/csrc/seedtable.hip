// seedtable.hip -- seed pointer table and seed position table (Sec. 2.4,
// Fig. 1) over stored minimizers, on gfx950.
//
// Entries i = 0 .. count-1 are (hash[i], pos[i]) in input (position) order;
// key(h) = (h >> shift) mod 2^bits.  The position table lists the entries
// grouped by key, ascending, each group in input order; the pointer table
// holds ptr[j] = number of entries with key < j for j = 0 .. 2^bits, so the
// hits of key j are ptr[j] .. ptr[j+1] - 1 (the paper's table, whose entry
// for a seed closes that seed's list, is ptr[1 ..]).
//
// Method: a least-significant-digit radix sort of (key, input index) pairs
// with 8-bit digits, ceil(bits / 8) passes, each stable, so that equal keys
// keep input order; then a lower-bound search of the sorted keys fills the
// pointer table.  A pass is three launches:
//   1. digit histogram of each 4096-entry tile (LDS counters per wave);
//   2. per digit, an exclusive scan over the tiles (one workgroup per digit),
//      giving every (digit, tile) its offset inside the digit's range;
//   3. stable scatter: a tile's entries are ranked within their digit in
//      index order -- per wave, 64 consecutive entries at a time, with the
//      lanes of equal digit found by 8 ballots -- and written at
//      digit start + tile offset + rank.
// The first pass reads the keys straight from the hashes, the last one
// gathers the positions (and hashes) instead of writing index pairs.
#include "sws_device.hpp"
#include "sws_internal.hpp"

namespace sws {

namespace {

constexpr int kSeedNT = 256;                    // threads per workgroup
constexpr int kSeedWaves = kSeedNT / kWave;
constexpr int kSeedRounds = 16;                 // 64-entry rounds per wave
constexpr uint32_t kSeedTile = kSeedNT * kSeedRounds;  // entries per tile
constexpr int kDigits = 256;

__device__ __forceinline__ uint32_t seed_key(uint64_t h, uint32_t shift, uint32_t mask) {
    return (uint32_t)(h >> shift) & mask;
}

// Entry e of wave wv's share of tile b, round r: tile entries are taken in
// index order, 1024 per wave, 64 per round.
__device__ __forceinline__ uint64_t tile_entry(uint64_t b, int wv, int r, int lane) {
    return b * kSeedTile + (uint64_t)wv * (kSeedRounds * kWave) + (uint64_t)r * kWave + lane;
}

}  // namespace

// 1. digit histogram per tile: hist[d * ntiles + b]
template <bool FIRST>
__global__ __launch_bounds__(kSeedNT) void seed_hist_kernel(const uint64_t* __restrict__ hash,
                                                            const uint32_t* __restrict__ keys,
                                                            uint64_t count, uint32_t shift,
                                                            uint32_t mask, uint32_t dshift,
                                                            uint32_t* __restrict__ hist,
                                                            uint64_t ntiles) {
    __shared__ uint32_t cnt[kSeedWaves][kDigits];
    const int lane = lane_id();
    const int wv = wave_id();
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    wave_lds_sync();
    const uint64_t b = blockIdx.x;
#pragma unroll 4
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = tile_entry(b, wv, r, lane);
        if (i < count) {
            const uint32_t key = FIRST ? seed_key(hash[i], shift, mask) : keys[i];
            atomicAdd(&cnt[wv][(key >> dshift) & 0xFFu], 1u);
        }
    }
    __syncthreads();
    for (int d = (int)threadIdx.x; d < kDigits; d += kSeedNT) {
        uint32_t s = 0;
#pragma unroll
        for (int v = 0; v < kSeedWaves; ++v) s += cnt[v][d];
        hist[(uint64_t)d * ntiles + b] = s;
    }
}

// 2. per digit (one workgroup each): exclusive scan of hist[d * ntiles ..]
//    over the tiles, in place; totals[d] = the digit's count.
__global__ __launch_bounds__(kSeedNT) void seed_scan_kernel(uint32_t* __restrict__ hist,
                                                            uint64_t ntiles,
                                                            uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[kSeedWaves];
    const int lane = lane_id();
    const int wv = wave_id();
    uint32_t* row = hist + (uint64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (uint64_t base = 0; base < ntiles; base += kSeedNT) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < ntiles ? row[i] : 0u;
        uint32_t incl = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = shfl(incl, lane, -d);
            if (lane >= d) incl += o;
        }
        if (lane == kWave - 1) part[wv] = incl;
        __syncthreads();
        uint32_t before = carry;
        for (int v2 = 0; v2 < wv; ++v2) before += part[v2];
        uint32_t chunk = 0;
        for (int v2 = 0; v2 < kSeedWaves; ++v2) chunk += part[v2];
        if (i < ntiles) row[i] = before + incl - v;
        carry += chunk;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// 3. stable scatter of one tile
template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kSeedNT) void seed_scatter_kernel(
    const uint64_t* __restrict__ hash, const uint32_t* __restrict__ pos,
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ idx_in, uint64_t count,
    uint32_t shift, uint32_t mask, uint32_t dshift, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, uint64_t ntiles, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ idx_out, uint32_t* __restrict__ pos_out,
    uint64_t* __restrict__ hash_out) {
    __shared__ uint32_t cnt[kSeedWaves][kDigits];  // running counts, then wave offsets
    __shared__ uint32_t base[kDigits];             // digit start + this tile's offset
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t b = blockIdx.x;
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    // digit starts: exclusive scan of the 256 totals (wave 0), plus the tile's offset
    if (wv == 0) {
        uint32_t run = 0;
        for (int c = 0; c < kDigits; c += kWave) {
            const uint32_t v = totals[c + lane];
            uint32_t incl = v;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o = shfl(incl, lane, -d);
                if (lane >= d) incl += o;
            }
            base[c + lane] = run + incl - v + hist[(uint64_t)(c + lane) * ntiles + b];
            run += lane_value(incl, kWave - 1);
        }
    }
    wave_lds_sync();
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t key[kSeedRounds], src[kSeedRounds], rank[kSeedRounds];
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = tile_entry(b, wv, r, lane);
        const bool valid = i < count;
        key[r] = 0u;
        src[r] = 0u;
        if (valid) {
            key[r] = FIRST ? seed_key(hash[i], shift, mask) : keys_in[i];
            src[r] = FIRST ? (uint32_t)i : idx_in[i];
        }
        const uint32_t d = (key[r] >> dshift) & 0xFFu;
        // lanes holding the same digit (valid lanes only)
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bal = __ballot(on);
            same &= on ? bal : ~bal;
        }
        const uint32_t prior = valid ? cnt[wv][d] : 0u;
        rank[r] = prior + (uint32_t)__builtin_popcountll(same & below);
        // the highest lane of each group advances the group's count
        if (valid && (same >> lane) == 1ull)
            cnt[wv][d] = prior + (uint32_t)__builtin_popcountll(same);
        wave_lds_sync();
    }
    __syncthreads();
    // wave offsets within the tile: exclusive prefix over waves, per digit
    for (int d = (int)threadIdx.x; d < kDigits; d += kSeedNT) {
        uint32_t run = 0;
#pragma unroll
        for (int v = 0; v < kSeedWaves; ++v) {
            const uint32_t t = cnt[v][d];
            cnt[v][d] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = tile_entry(b, wv, r, lane);
        if (i >= count) continue;
        const uint32_t d = (key[r] >> dshift) & 0xFFu;
        const uint32_t dest = base[d] + cnt[wv][d] + rank[r];
        keys_out[dest] = key[r];
        if (LAST) {
            pos_out[dest] = pos[src[r]];
            if (hash_out) hash_out[dest] = hash[src[r]];
        } else {
            idx_out[dest] = src[r];
        }
    }
}

// 4. pointer table: ptr[j] = first index of keys (sorted) with key >= j, for
//    j = 0 .. nkeys; 16 consecutive j per thread, a binary search for the
//    first and a galloping search from there for the rest.
__global__ __launch_bounds__(kSeedNT) void seed_ptr_kernel(const uint32_t* __restrict__ keys,
                                                           uint64_t count, uint64_t nkeys,
                                                           uint32_t* __restrict__ ptr) {
    const uint64_t t = (uint64_t)blockIdx.x * kSeedNT + threadIdx.x;
    const uint64_t j0 = t * 16;
    if (j0 > nkeys) return;
    // lower bound of j0
    uint64_t lo = 0, hi = count;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)keys[mid] < j0) lo = mid + 1;
        else hi = mid;
    }
    uint64_t at = lo;
    for (uint64_t j = j0; j < j0 + 16 && j <= nkeys; ++j) {
        if (at < count && (uint64_t)keys[at] < j) {
            // keys[at] < j: gallop to a bound, then bisect
            uint64_t step = 1, prev = at;
            while (at + step < count && (uint64_t)keys[at + step] < j) {
                prev = at + step;
                step *= 2;
            }
            uint64_t l2 = prev + 1, h2 = at + step < count ? at + step : count;
            while (l2 < h2) {
                const uint64_t mid = l2 + (h2 - l2) / 2;
                if ((uint64_t)keys[mid] < j) l2 = mid + 1;
                else h2 = mid;
            }
            at = l2;
        }
        ptr[j] = (uint32_t)at;
    }
}

// ---------------------------------------------------------------------------
// Launcher.
// ---------------------------------------------------------------------------
namespace {

uint64_t seed_tiles(uint64_t count) { return (count + kSeedTile - 1) / kSeedTile; }

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

}  // namespace

uint64_t seed_table_workspace_bytes(uint64_t count) {
    const uint64_t nt = seed_tiles(count);
    return 4 * align256(4 * count) + align256(4ull * kDigits * nt) + align256(4ull * kDigits);
}

int launch_seed_table(const uint64_t* hash, const uint32_t* pos, uint64_t count, uint32_t bits,
                      uint32_t shift, uint32_t* ptr, uint32_t* pos_out, uint64_t* hash_out,
                      void* workspace, hipStream_t s) {
    const uint64_t nkeys = 1ull << bits;
    const uint32_t mask = (uint32_t)(nkeys - 1);
    const uint64_t nt = seed_tiles(count);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    uint32_t* keysA = reinterpret_cast<uint32_t*>(ws);
    uint32_t* idxA = reinterpret_cast<uint32_t*>(ws + align256(4 * count));
    uint32_t* keysB = reinterpret_cast<uint32_t*>(ws + 2 * align256(4 * count));
    uint32_t* idxB = reinterpret_cast<uint32_t*>(ws + 3 * align256(4 * count));
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + 4 * align256(4 * count));
    uint32_t* totals =
        reinterpret_cast<uint32_t*>(ws + 4 * align256(4 * count) + align256(4ull * kDigits * nt));
    const uint32_t* sorted = keysA;
    if (count > 0) {
        const int passes = (int)((bits + 7) / 8);
        const uint32_t* kin = nullptr;
        const uint32_t* iin = nullptr;
        uint32_t* kout = keysA;
        uint32_t* iout = idxA;
        for (int p = 0; p < passes; ++p) {
            const uint32_t dshift = 8u * (uint32_t)p;
            const bool first = p == 0, last = p == passes - 1;
            if (first)
                hipLaunchKernelGGL(seed_hist_kernel<true>, dim3((unsigned)nt), dim3(kSeedNT), 0, s,
                                   hash, kin, count, shift, mask, dshift, hist, nt);
            else
                hipLaunchKernelGGL(seed_hist_kernel<false>, dim3((unsigned)nt), dim3(kSeedNT), 0,
                                   s, hash, kin, count, shift, mask, dshift, hist, nt);
            hipLaunchKernelGGL(seed_scan_kernel, dim3(kDigits), dim3(kSeedNT), 0, s, hist, nt,
                               totals);
#define SWS_SEED_SCATTER(F, L)                                                                \
    hipLaunchKernelGGL((seed_scatter_kernel<F, L>), dim3((unsigned)nt), dim3(kSeedNT), 0, s,  \
                       hash, pos, kin, iin, count, shift, mask, dshift, hist, totals, nt, kout, \
                       iout, pos_out, hash_out)
            if (first && last) SWS_SEED_SCATTER(true, true);
            else if (first) SWS_SEED_SCATTER(true, false);
            else if (last) SWS_SEED_SCATTER(false, true);
            else SWS_SEED_SCATTER(false, false);
#undef SWS_SEED_SCATTER
            sorted = kout;
            kin = kout;
            iin = iout;
            kout = kout == keysA ? keysB : keysA;
            iout = iout == idxA ? idxB : idxA;
        }
    }
    const uint64_t threads = (nkeys + 1 + 15) / 16;
    hipLaunchKernelGGL(seed_ptr_kernel, dim3((unsigned)((threads + kSeedNT - 1) / kSeedNT)),
                       dim3(kSeedNT), 0, s, sorted, count, nkeys, ptr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sws
