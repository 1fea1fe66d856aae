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
// Method: a least-significant-digit radix sort with 8-bit digits,
// ceil(bits / 8) passes, each stable, so that equal keys keep input order.
// The entries travel through the passes as (hash, pos) when the hashes are
// wanted in the output (the key is recomputed from the hash), else as
// (key, pos).  A pass is four launches:
//   1. digit histogram of each 4096-entry tile, one 1 KB row per tile (LDS
//      counters per wave; with hashes, passes after the first read one
//      digit byte per entry that the previous scatter wrote, not the hash);
//   2. the tiles split into at most 512 ranges: per range, the exclusive
//      scan of its tiles' rows and the range's row of totals;
//   3. per digit, the exclusive scan over the ranges' totals and the
//      digit's total;
//   4. stable scatter: a tile's entries are ranked within their digit in
//      index order -- per wave, 64 consecutive entries at a time, with the
//      lanes of equal digit found by 8 ballots -- placed in LDS in digit
//      order, and written out as runs of consecutive addresses per digit.
//      A digit's run in a tile is ~16 entries long.  The tile's LDS staging
//      is 32 KB either way (with hashes, the positions pass through the
//      region after the hashes have left it), plus 10 KB of counters: 43,008
//      bytes per workgroup, three workgroups per CU.
// The last pass also writes the pointer table (see SeedPtrOut): its input is
// sorted by the key bits below its digit, which lets each tile own a range of
// pointer entries and fill it from the run of each digit in its LDS stage.
#include "sws_device.hpp"
#include "sws_internal.hpp"

namespace sws {

namespace {

constexpr int kSeedNT = 512;                           // threads per workgroup
constexpr int kSeedWaves = kSeedNT / kWave;
constexpr int kSeedRounds = 8;                         // 64-entry rounds per wave
constexpr uint32_t kSeedTile = kSeedNT * kSeedRounds;  // entries per tile
constexpr int kDigits = 256;
constexpr int kXcds = 8;                               // gfx950: 8 accelerator dies

__device__ __forceinline__ uint32_t seed_key(uint64_t h, uint32_t shift, uint32_t mask) {
    return (uint32_t)(h >> shift) & mask;
}

// Entry of wave wv's share of tile b, round r: tile entries are taken in
// index order, 512 per wave, 64 per round.
__device__ __forceinline__ uint32_t tile_slot(int wv, int r, int lane) {
    return (uint32_t)wv * (kSeedRounds * kWave) + (uint32_t)r * kWave + (uint32_t)lane;
}

// An entry on its way through the passes: the hash (HASH) or the key, and the
// position.
template <bool HASH>
struct SeedItem;
template <>
struct SeedItem<true> {
    uint64_t h;
    uint32_t p;
    __device__ uint32_t key(uint32_t shift, uint32_t mask) const { return seed_key(h, shift, mask); }
};
template <>
struct SeedItem<false> {
    uint32_t k;
    uint32_t p;
    __device__ uint32_t key(uint32_t, uint32_t) const { return k; }
};

// Where a pass reads its entries from and writes them to.
struct SeedBuffers {
    const uint64_t* hash_in;  // first pass: the caller's hashes; later: HASH carry
    const uint32_t* key_in;   // later passes without HASH
    const uint32_t* pos_in;
    uint64_t* hash_out;
    uint32_t* key_out;
    uint32_t* pos_out;
    // with hashes: the next pass's digit of every output entry, one byte
    // each, written by every scatter but the last and read by the next
    // pass's histogram (an eighth of the bytes of a hash; against a 4-byte
    // key the extra stores in the scatter cost what the histogram saves)
    const uint8_t* dig_in;
    uint8_t* dig_out;
};

template <bool FIRST, bool HASH>
__device__ __forceinline__ SeedItem<HASH> seed_load(const SeedBuffers& io, uint64_t i,
                                                    uint32_t shift, uint32_t mask) {
    SeedItem<HASH> it;
    if constexpr (HASH) {
        it.h = io.hash_in[i];
    } else {
        it.k = FIRST ? seed_key(io.hash_in[i], shift, mask) : io.key_in[i];
    }
    it.p = io.pos_in[i];
    return it;
}


}  // namespace

// 1. digit histogram per tile: hist[b * 256 + d], one coalesced 1 KB row per
//    tile.  The first pass, and every pass without hashes, takes the digits
//    from the keys; later passes with hashes from the digit bytes the
//    previous scatter wrote (8 per thread, their order within the tile does
//    not matter to a count).  One workgroup per tile:
//    four tiles per workgroup, their loads all issued first, measured slower
//    (too few workgroups to fill the chip).
template <bool FIRST, bool HASH>
__global__ __launch_bounds__(kSeedNT) void seed_hist_kernel(SeedBuffers io, uint64_t count,
                                                            uint32_t shift, uint32_t mask,
                                                            uint32_t dshift,
                                                            uint32_t* __restrict__ hist) {
    static_assert(kSeedTile == kSeedNT * 8, "eight digit bytes per thread");
    __shared__ uint32_t cnt[kSeedWaves][kDigits];
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t b = blockIdx.x;
    constexpr bool kBytes = HASH && !FIRST;
    uint32_t dig[kSeedRounds];
    if constexpr (!kBytes) {
#pragma unroll
        for (int r = 0; r < kSeedRounds; ++r) {
            const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
            const uint32_t k = i < count ? (FIRST ? seed_key(io.hash_in[i], shift, mask) : io.key_in[i]) : 0u;
            dig[r] = (k >> dshift) & 0xFFu;
        }
    } else {
        const uint64_t i0 = b * kSeedTile + 8ull * threadIdx.x;
        if (i0 + 8 <= count) {
            const uint2 v = *reinterpret_cast<const uint2*>(io.dig_in + i0);  // 8-byte aligned
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dig[r] = (v.x >> (8 * r)) & 0xFFu;
                dig[r + 4] = (v.y >> (8 * r)) & 0xFFu;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kSeedRounds; ++r) dig[r] = i0 + r < count ? io.dig_in[i0 + r] : 0u;
        }
    }
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = kBytes ? b * kSeedTile + 8ull * threadIdx.x + (uint64_t)r
                                  : b * kSeedTile + tile_slot(wv, r, lane);
        if (i < count) atomicAdd(&cnt[wv][dig[r]], 1u);
    }
    __syncthreads();
    for (int d = (int)threadIdx.x; d < kDigits; d += kSeedNT) {
        uint32_t c = 0;
#pragma unroll
        for (int v = 0; v < kSeedWaves; ++v) c += cnt[v][d];
        hist[b * kDigits + (uint64_t)d] = c;
    }
}

// 2a. per range of tiles [r * per, (r + 1) * per) (one 256-thread workgroup
//     each, thread d for digit d): hist[b * 256 + d] becomes the count of d in
//     the range's tiles before b, and rtot[r * 256 + d] the range's count of
//     d.  Every read and write is a coalesced 1 KB row.
__global__ __launch_bounds__(kDigits) void seed_range_scan_kernel(uint32_t* __restrict__ hist,
                                                                  uint64_t ntiles, uint64_t per,
                                                                  uint32_t* __restrict__ rtot) {
    const uint64_t d = threadIdx.x;
    const uint64_t b0 = blockIdx.x * per;
    const uint64_t b1 = b0 + per < ntiles ? b0 + per : ntiles;
    uint32_t run = 0;
    uint64_t b = b0;
    for (; b + 4 <= b1; b += 4) {  // four independent loads in flight
        uint32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = hist[(b + q) * kDigits + d];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            hist[(b + q) * kDigits + d] = run;
            run += v[q];
        }
    }
    for (; b < b1; ++b) {
        const uint32_t v = hist[b * kDigits + d];
        hist[b * kDigits + d] = run;
        run += v;
    }
    rtot[blockIdx.x * kDigits + d] = run;
}

// 2b. per digit d (one workgroup each, one range per thread, at most
//     kSeedNT ranges): rtot[r * 256 + d] becomes the count of d in the
//     ranges before r, and totals[d] the digit's count.
__global__ __launch_bounds__(kSeedNT) void seed_range_base_kernel(uint32_t* __restrict__ rtot,
                                                                  uint64_t nranges,
                                                                  uint32_t* __restrict__ totals) {
    __shared__ uint32_t part[kSeedWaves];
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t d = blockIdx.x;
    const uint64_t r = threadIdx.x;
    const uint32_t v = r < nranges ? rtot[r * kDigits + d] : 0u;
    const uint32_t incl = wave_inclusive_sum(v);
    if (lane == kWave - 1) part[wv] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w2 = 0; w2 < kSeedWaves; ++w2) {
        before += w2 < wv ? part[w2] : 0u;
        all += part[w2];
    }
    if (r < nranges) rtot[r * kDigits + d] = before + incl - v;
    if (threadIdx.x == 0) totals[d] = all;
}

// Exclusive scan of 256 values held one per lane-slot (v[c + lane], c in
// steps of 64) by one wave; returns the total.
__device__ __forceinline__ uint32_t wave_scan256(uint32_t* a, int lane) {
    uint32_t run = 0;
    for (int c = 0; c < kDigits; c += kWave) {
        const uint32_t v = a[c + lane];
        uint32_t incl = wave_inclusive_sum(v);
        a[c + lane] = run + incl - v;
        run += lane_value(incl, kWave - 1);
    }
    return run;
}

// The key of input entry i of a pass.
template <bool FIRST, bool HASH>
__device__ __forceinline__ uint32_t seed_in_key(const SeedBuffers& io, uint64_t i, uint32_t shift,
                                                uint32_t mask) {
    return (HASH || FIRST) ? seed_key(io.hash_in[i], shift, mask) : io.key_in[i];
}

// Where the pointer table comes from (the last pass, LAST).  That pass's input
// is sorted by the key's low part (the bits below the pass's digit), so tile b
// holds the low values (V_{b-1}, V_b], V_b being the low part of its last
// entry.  For such a v and any digit d,
//   ptr[(d, v)] = (entries of d in tiles before b) + (entries of d in tile b
//                 with low part < v),
// because every earlier tile's entries have low parts <= V_{b-1} < v and
// every later tile's have low parts >= V_b >= v.  Tile b writes exactly those
// entries (the first tile from v = 0, the last up to the largest low value),
// so every pointer entry is written once, by one tile, with no pass of its own.
struct SeedPtrOut {
    uint32_t* ptr;
    uint64_t nkeys;   // 2^bits; ptr[nkeys] = count
    uint32_t ndig;    // digit values of the last pass: 2^(bits - dshift)
};

// 3. stable scatter of one tile
template <bool FIRST, bool HASH, bool LAST>
__global__ __launch_bounds__(kSeedNT) void seed_scatter_kernel(
    SeedBuffers io, uint64_t count, uint32_t shift, uint32_t mask, uint32_t dshift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ rtot, uint64_t per,
    const uint32_t* __restrict__ totals, uint64_t ntiles, uint32_t per_xcd, SeedPtrOut po) {
    __shared__ uint32_t cnt[kSeedWaves][kDigits];  // running counts, then wave offsets
    __shared__ uint32_t gbase[kDigits];            // global start of the tile's run of d
    __shared__ uint32_t tstart[kDigits];           // start of d in the tile's digit order
    // the tile in digit order, field by field (no padding).  With hashes the
    // positions follow the hashes through the same 32 KB (42 KB per
    // workgroup instead of 58: three workgroups per CU instead of two).
    __shared__ uint64_t stage_h[HASH ? kSeedTile : 1];
    __shared__ uint32_t stage_k[HASH ? 1 : kSeedTile];
    __shared__ uint32_t stage_p_own[HASH ? 1 : kSeedTile];
    uint32_t* const stage_p = HASH ? reinterpret_cast<uint32_t*>(stage_h) : stage_p_own;
    // Workgroups are dealt to the dies round-robin; each die takes a
    // contiguous run of tiles, so that the line a tile's run of a digit (or of
    // pointer entries) leaves partly written is completed by the next tile in
    // the same L2.
    const uint64_t b = (uint64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
    if (b >= ntiles) return;  // uniform over the workgroup
    const int lane = lane_id();
    const int wv = wave_id();
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    wave_lds_sync();
    // Thread d < 256: digit d's total and the count of d in earlier tiles
    // (earlier ranges, then the range's tiles before b), loaded now into
    // registers and used only after the ranking rounds, so that no wave waits
    // on them before it ranks.
    const int tid = (int)threadIdx.x;
    uint32_t d_total = 0, d_range = 0, d_tile = 0;
    if (tid < kDigits) {
        d_total = totals[tid];
        d_range = rtot[(b / per) * kDigits + (uint64_t)tid];
        d_tile = hist[b * kDigits + (uint64_t)tid];
    }
    const uint64_t below = (1ull << lane) - 1ull;
    // LAST: the low parts of the previous tile's last entry and of this tile's
    // last entry bound this tile's pointer entries; loaded early
    const uint32_t lmask = LAST ? (1u << dshift) - 1u : 0u;  // dshift <= 24
    uint32_t vprev = 0, vlast = 0;
    if (LAST) {
        const uint64_t t_end = (b + 1) * kSeedTile < count ? (b + 1) * kSeedTile : count;
        if (b > 0) vprev = seed_in_key<FIRST, HASH>(io, b * kSeedTile - 1, shift, mask);
        vlast = seed_in_key<FIRST, HASH>(io, t_end - 1, shift, mask);
    }
    SeedItem<HASH> item[kSeedRounds];
    uint32_t rank[kSeedRounds];
    // every load of the tile first: the ranking rounds below are separated by
    // wave fences, which loads cannot be moved across
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        if (i < count) item[r] = seed_load<FIRST, HASH>(io, i, shift, mask);
        else item[r] = SeedItem<HASH>{};
    }
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        const bool valid = i < count;
        const uint32_t d = (item[r].key(shift, mask) >> dshift) & 0xFFu;
        // lanes holding the same digit (valid lanes only): a lane differs
        // from this one where some bit of the two digits differs, i.e. where
        // the bit's ballot differs from this lane's bit spread to a word
        // (0 or all ones; a signed 1-bit field extract), per 32-lane half
        uint32_t diff_lo = 0u, diff_hi = 0u;
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint32_t spread = (uint32_t)(((int32_t)(d << (31 - bit))) >> 31);
            const uint64_t bal = __ballot(spread != 0u);
            diff_lo |= (uint32_t)bal ^ spread;
            diff_hi |= (uint32_t)(bal >> 32) ^ spread;
        }
        const uint64_t same = ~(((uint64_t)diff_hi << 32) | diff_lo) & __ballot(valid);
        const uint32_t prior = valid ? cnt[wv][d] : 0u;
        rank[r] = prior + (uint32_t)__builtin_popcountll(same & below);
        // the highest lane of each group advances the group's count
        if (valid && (same >> lane) == 1ull)
            cnt[wv][d] = prior + (uint32_t)__builtin_popcountll(same);
        wave_lds_sync();
    }
    __syncthreads();
    // per digit: wave offsets (exclusive over waves), the tile's digit total
    // and the digit's total over all tiles
    if (tid < kDigits) {
        const int d = tid;
        uint32_t run = 0;
#pragma unroll
        for (int v = 0; v < kSeedWaves; ++v) {
            const uint32_t t = cnt[v][d];
            cnt[v][d] = run;
            run += t;
        }
        tstart[d] = run;
        gbase[d] = d_total;
    }
    __syncthreads();
    if (wv == 0) wave_scan256(tstart, lane);  // starts of the digits in the tile's order
    if (wv == 1) wave_scan256(gbase, lane);   // starts of the digits in the output
    __syncthreads();
    // global start of the tile's run of d (read only after the next barrier)
    if (tid < kDigits) gbase[tid] += d_range + d_tile;
    // place the tile in digit order (with hashes, the hashes only; the
    // slots are kept for the positions)
    uint32_t slot[kSeedRounds];
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        slot[r] = 0u;
        if (i >= count) continue;
        const uint32_t d = (item[r].key(shift, mask) >> dshift) & 0xFFu;
        slot[r] = tstart[d] + cnt[wv][d] + rank[r];
        if constexpr (HASH) {
            stage_h[slot[r]] = item[r].h;
        } else {
            stage_k[slot[r]] = item[r].k;
            stage_p[slot[r]] = item[r].p;
        }
    }
    __syncthreads();
    // write out: consecutive slots of one digit go to consecutive addresses
    const uint64_t t0 = b * kSeedTile;
    const uint32_t nb = count - t0 < kSeedTile ? (uint32_t)(count - t0) : kSeedTile;
    uint32_t dst_of[kSeedRounds];  // HASH: where slot threadIdx.x + j * kSeedNT goes
#pragma unroll
    for (int j = 0; j < kSeedRounds; ++j) {
        const uint32_t t = threadIdx.x + (uint32_t)j * kSeedNT;
        dst_of[j] = 0u;
        if (t >= nb) continue;
        const uint32_t k = HASH ? seed_key(stage_h[t], shift, mask) : stage_k[t];
        const uint32_t d = (k >> dshift) & 0xFFu;
        const uint32_t dst = gbase[d] + (t - tstart[d]);  // < count < 2^32
        if constexpr (HASH) {
            io.hash_out[dst] = stage_h[t];
            if constexpr (!LAST) io.dig_out[dst] = (uint8_t)((k >> (dshift + 8u)) & 0xFFu);
            dst_of[j] = dst;
        } else {
            io.key_out[dst] = k;
            io.pos_out[dst] = stage_p[t];
        }
    }
    if constexpr (LAST) {
        // this tile's pointer entries: low values vlo .. vhi of every digit
        const uint64_t vlo = b == 0 ? 0ull : (uint64_t)(vprev & lmask) + 1;
        const uint64_t vhi = b + 1 == ntiles ? lmask : vlast & lmask;
        if (vhi + 1 <= vlo + kWave) {
            // a short range (dense tables): entry j of d's run (low part l_j;
            // runs are in input order, so the low parts ascend) owns v in
            // (l_{j-1}, l_j], below which lie exactly j entries of the run;
            // the first entry's range starts at vlo
            for (uint32_t q = threadIdx.x; q < nb; q += kSeedNT) {
                const uint32_t k = HASH ? seed_key(stage_h[q], shift, mask) : stage_k[q];
                const uint32_t d = (k >> dshift) & 0xFFu;
                const uint32_t s0 = tstart[d];
                const uint64_t from =
                    q > s0 ? (uint64_t)((HASH ? seed_key(stage_h[q - 1], shift, mask) : stage_k[q - 1]) & lmask) + 1
                           : vlo;
                const uint64_t to = (uint64_t)(k & lmask);
                const uint32_t val = gbase[d] + (q - s0);
                for (uint64_t v = from > vlo ? from : vlo; v <= to; ++v)
                    po.ptr[((uint64_t)d << dshift) | v] = val;
            }
            // past a digit's last entry (or the whole range if the tile has
            // none of it) all of the run lies below: per digit, where that
            // starts and the value, then one sweep over (digit, v) so that
            // neighbouring lanes store to neighbouring entries
            uint32_t* tail_from = cnt[0];  // the rank counters are free by now
            uint32_t* tail_val = cnt[1];
            for (uint32_t d = threadIdx.x; d < po.ndig; d += kSeedNT) {
                const uint32_t s0 = tstart[d];
                const uint32_t s1 = d + 1 < (uint32_t)kDigits ? tstart[d + 1] : nb;
                tail_from[d] = s1 > s0 ? ((HASH ? seed_key(stage_h[s1 - 1], shift, mask) : stage_k[s1 - 1]) & lmask) + 1u
                                       : (uint32_t)vlo;
                tail_val[d] = gbase[d] + (s1 - s0);
            }
            __syncthreads();
            const uint32_t rng = (uint32_t)(vhi + 1 - vlo);  // 1 .. 64
            for (uint32_t idx = threadIdx.x; idx < po.ndig * rng; idx += kSeedNT) {
                const uint32_t d = idx / rng;
                const uint32_t v = (uint32_t)vlo + (idx - d * rng);
                if (v >= tail_from[d]) po.ptr[((uint64_t)d << dshift) | v] = tail_val[d];
            }
        } else {
            // a long range (sparse tables): lanes take consecutive v, each
            // counting the run's entries below v by a binary search
            for (uint32_t d = (uint32_t)wv; d < po.ndig; d += kSeedWaves) {
                const uint32_t s0 = tstart[d];
                const uint32_t s1 = d + 1 < (uint32_t)kDigits ? tstart[d + 1] : nb;
                for (uint64_t v = vlo + (uint64_t)lane; v <= vhi; v += kWave) {
                    uint32_t lo = s0, hi = s1;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        const uint32_t k = HASH ? seed_key(stage_h[mid], shift, mask) : stage_k[mid];
                        if ((k & lmask) < v) lo = mid + 1;
                        else hi = mid;
                    }
                    po.ptr[((uint64_t)d << dshift) | v] = gbase[d] + (lo - s0);
                }
            }
        }
        if (b + 1 == ntiles && threadIdx.x == 0) po.ptr[po.nkeys] = (uint32_t)count;
    }
    if constexpr (HASH) {
        // the positions, through the region the hashes have left
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSeedRounds; ++r) {
            const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
            if (i < count) stage_p[slot[r]] = item[r].p;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSeedRounds; ++j) {
            const uint32_t t = threadIdx.x + (uint32_t)j * kSeedNT;
            if (t < nb) io.pos_out[dst_of[j]] = stage_p[t];
        }
    }
}

__global__ void seed_fill_kernel(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Launcher.
// ---------------------------------------------------------------------------
namespace {

uint64_t seed_tiles(uint64_t count) { return (count + kSeedTile - 1) / kSeedTile; }

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

// Ranges of tiles of the offset scan: at most one per thread of the range
// base kernel.
uint64_t seed_ranges(uint64_t nt) { return nt < (uint64_t)kSeedNT ? nt : (uint64_t)kSeedNT; }

// The offset arrays of a pass.
struct SeedOffsets {
    uint32_t* hist;    // [tile * 256 + d]
    uint32_t* rtot;    // [range * 256 + d]
    uint32_t* totals;  // [d]
};

template <bool FIRST, bool HASH, bool LAST>
void seed_pass(const SeedBuffers& io, uint64_t count, uint32_t shift, uint32_t mask,
               uint32_t dshift, const SeedOffsets& off, uint64_t nt, const SeedPtrOut& po,
               hipStream_t s) {
    const uint64_t nr = seed_ranges(nt), per = (nt + nr - 1) / nr;
    hipLaunchKernelGGL((seed_hist_kernel<FIRST, HASH>), dim3((unsigned)nt), dim3(kSeedNT), 0, s,
                       io, count, shift, mask, dshift, off.hist);
    hipLaunchKernelGGL(seed_range_scan_kernel, dim3((unsigned)((nt + per - 1) / per)),
                       dim3(kDigits), 0, s, off.hist, nt, per, off.rtot);
    hipLaunchKernelGGL(seed_range_base_kernel, dim3(kDigits), dim3(kSeedNT), 0, s, off.rtot,
                       (nt + per - 1) / per, off.totals);
    const uint32_t per_xcd = (uint32_t)((nt + kXcds - 1) / kXcds);
    hipLaunchKernelGGL((seed_scatter_kernel<FIRST, HASH, LAST>), dim3(per_xcd * kXcds),
                       dim3(kSeedNT), 0, s, io, count, shift, mask, dshift, off.hist, off.rtot,
                       per, off.totals, nt, per_xcd, po);
}

template <bool HASH>
void seed_pass_any(bool first, bool last, const SeedBuffers& io, uint64_t count, uint32_t shift,
                   uint32_t mask, uint32_t dshift, const SeedOffsets& off, uint64_t nt,
                   const SeedPtrOut& po, hipStream_t s) {
    if (first && last) seed_pass<true, HASH, true>(io, count, shift, mask, dshift, off, nt, po, s);
    else if (first) seed_pass<true, HASH, false>(io, count, shift, mask, dshift, off, nt, po, s);
    else if (last) seed_pass<false, HASH, true>(io, count, shift, mask, dshift, off, nt, po, s);
    else seed_pass<false, HASH, false>(io, count, shift, mask, dshift, off, nt, po, s);
}

}  // namespace

// Workspace: two carries of (8-byte hash or 4-byte key, 4-byte position),
// the tile histogram rows, the range counts, the 256 digit totals and the
// digit bytes.
uint64_t seed_table_workspace_bytes(uint64_t count, uint32_t bits) {
    (void)bits;
    const uint64_t nt = seed_tiles(count);
    return 2 * align256(8 * count) + 2 * align256(4 * count) + align256(4ull * kDigits * nt) +
           align256(4ull * kDigits * seed_ranges(nt)) + align256(4ull * kDigits) +
           align256(count);
}

int launch_seed_table(const uint64_t* hash, const uint32_t* pos, uint64_t count, uint32_t bits,
                      uint32_t shift, uint32_t* ptr, uint32_t* pos_out, uint64_t* hash_out,
                      void* workspace, hipStream_t s) {
    const uint64_t nkeys = 1ull << bits;
    const uint32_t mask = (uint32_t)(nkeys - 1);
    const uint64_t nt = seed_tiles(count);
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    uint64_t* carryH[2] = {reinterpret_cast<uint64_t*>(ws),
                           reinterpret_cast<uint64_t*>(ws + align256(8 * count))};
    uint8_t* wp = ws + 2 * align256(8 * count);
    uint32_t* carryP[2] = {reinterpret_cast<uint32_t*>(wp),
                           reinterpret_cast<uint32_t*>(wp + align256(4 * count))};
    SeedOffsets off;
    off.hist = reinterpret_cast<uint32_t*>(wp + 2 * align256(4 * count));
    off.rtot = off.hist + align256(4ull * kDigits * nt) / 4;
    off.totals = off.rtot + align256(4ull * kDigits * seed_ranges(nt)) / 4;
    uint8_t* digits = reinterpret_cast<uint8_t*>(off.totals) + align256(4ull * kDigits);
    const bool with_hash = hash_out != nullptr;
    if (count == 0) {
        // no entries: every pointer is 0
        const uint64_t blocks = (nkeys + 1 + 255) / 256;
        hipLaunchKernelGGL(seed_fill_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)),
                           dim3(256), 0, s, ptr, nkeys + 1, 0u);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    const int passes = (int)((bits + 7) / 8);
    SeedPtrOut po;
    po.ptr = ptr;
    po.nkeys = nkeys;
    po.ndig = 1u << (bits - 8u * (uint32_t)(passes - 1));
    SeedBuffers io{};
    io.hash_in = hash;
    io.pos_in = pos;
    // one digit buffer serves every pass: a pass's histogram has read it
    // before its scatter writes the next pass's digits
    io.dig_in = digits;
    io.dig_out = digits;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        const int o = p & 1;
        // outputs: the caller's arrays on the last pass, else a carry buffer
        io.pos_out = last ? pos_out : carryP[o];
        if (with_hash) io.hash_out = last ? hash_out : carryH[o];
        else io.key_out = reinterpret_cast<uint32_t*>(carryH[o]);  // keys in the hash slots
        const uint32_t dshift = 8u * (uint32_t)p;
        if (with_hash)
            seed_pass_any<true>(p == 0, last, io, count, shift, mask, dshift, off, nt, po, s);
        else
            seed_pass_any<false>(p == 0, last, io, count, shift, mask, dshift, off, nt, po, s);
        // this pass's outputs are the next pass's inputs
        io.pos_in = io.pos_out;
        if (with_hash) io.hash_in = io.hash_out;
        else io.key_in = io.key_out;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sws
