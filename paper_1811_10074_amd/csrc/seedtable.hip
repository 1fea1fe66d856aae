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
// (key, pos).  A pass is three launches:
//   1. digit histogram of each 4096-entry tile (LDS counters per wave; a
//      digit's run in the scatter is ~16 entries long, and the tile's 54 KB of
//      LDS staging lets two workgroups share a CU: 0.478 against 0.494 ms for
//      8192-entry tiles, one workgroup per CU);
//   2. per digit, an exclusive scan over the tiles (one workgroup per digit),
//      giving every (digit, tile) its offset inside the digit's range;
//   3. stable scatter: a tile's entries are ranked within their digit in
//      index order -- per wave, 64 consecutive entries at a time, with the
//      lanes of equal digit found by 8 ballots -- placed in LDS in digit
//      order, and written out as runs of consecutive addresses per digit.
// The pointer table is then the merge of the keys 0 .. 2^bits with the sorted
// keys (every key's lower bound), cut by merge path into equal shares.
#include "sws_device.hpp"
#include "sws_internal.hpp"

namespace sws {

namespace {

constexpr int kSeedNT = 512;                           // threads per workgroup
constexpr int kSeedWaves = kSeedNT / kWave;
constexpr int kSeedRounds = 8;                         // 64-entry rounds per wave
constexpr uint32_t kSeedTile = kSeedNT * kSeedRounds;  // entries per tile
constexpr int kDigits = 256;
constexpr uint32_t kPtrChunk = 4096;                   // pointer entries per workgroup

__device__ __forceinline__ uint32_t seed_key(uint64_t h, uint32_t shift, uint32_t mask) {
    return (uint32_t)(h >> shift) & mask;
}

// Entry of wave wv's share of tile b, round r: tile entries are taken in
// index order, 1024 per wave, 64 per round.
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

template <bool HASH>
__device__ __forceinline__ void seed_store(const SeedBuffers& io, uint64_t d,
                                           const SeedItem<HASH>& it) {
    if constexpr (HASH) io.hash_out[d] = it.h;
    else io.key_out[d] = it.k;
    io.pos_out[d] = it.p;
}

}  // namespace

// 1. digit histogram per tile: hist[d * ntiles + b]
template <bool FIRST, bool HASH>
__global__ __launch_bounds__(kSeedNT) void seed_hist_kernel(SeedBuffers io, uint64_t count,
                                                            uint32_t shift, uint32_t mask,
                                                            uint32_t dshift,
                                                            uint32_t* __restrict__ hist,
                                                            uint64_t ntiles) {
    __shared__ uint32_t cnt[kSeedWaves][kDigits];
    const int lane = lane_id();
    const int wv = wave_id();
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    wave_lds_sync();
    const uint64_t b = blockIdx.x;
    // every load of the tile first, so that their latencies overlap
    uint32_t key[kSeedRounds];
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        key[r] = 0u;
        if (i < count) key[r] = (HASH || FIRST) ? seed_key(io.hash_in[i], shift, mask) : io.key_in[i];
    }
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        if (i < count) atomicAdd(&cnt[wv][(key[r] >> dshift) & 0xFFu], 1u);
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

// Exclusive scan of 256 values held one per lane-slot (v[c + lane], c in
// steps of 64) by one wave; returns the total.
__device__ __forceinline__ uint32_t wave_scan256(uint32_t* a, int lane) {
    uint32_t run = 0;
    for (int c = 0; c < kDigits; c += kWave) {
        const uint32_t v = a[c + lane];
        uint32_t incl = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = shfl(incl, lane, -d);
            if (lane >= d) incl += o;
        }
        a[c + lane] = run + incl - v;
        run += lane_value(incl, kWave - 1);
    }
    return run;
}

// 3. stable scatter of one tile
template <bool FIRST, bool HASH>
__global__ __launch_bounds__(kSeedNT) void seed_scatter_kernel(
    SeedBuffers io, uint64_t count, uint32_t shift, uint32_t mask, uint32_t dshift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, uint64_t ntiles) {
    __shared__ uint32_t cnt[kSeedWaves][kDigits];  // running counts, then wave offsets
    __shared__ uint32_t gbase[kDigits];            // global start of the tile's run of d
    __shared__ uint32_t tstart[kDigits];           // start of d in the tile's digit order
    // the tile in digit order, field by field (no padding)
    __shared__ uint64_t stage_h[HASH ? kSeedTile : 1];
    __shared__ uint32_t stage_k[HASH ? 1 : kSeedTile];
    __shared__ uint32_t stage_p[kSeedTile];
    const int lane = lane_id();
    const int wv = wave_id();
    const uint64_t b = blockIdx.x;
    for (int d = lane; d < kDigits; d += kWave) cnt[wv][d] = 0u;
    if (wv == 0) {
        for (int d = lane; d < kDigits; d += kWave) gbase[d] = totals[d];
        wave_lds_sync();
        wave_scan256(gbase, lane);  // digit starts
        for (int d = lane; d < kDigits; d += kWave) gbase[d] += hist[(uint64_t)d * ntiles + b];
    }
    wave_lds_sync();
    const uint64_t below = (1ull << lane) - 1ull;
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
    // per digit: wave offsets (exclusive over waves) and the tile's digit total
    for (int d = (int)threadIdx.x; d < kDigits; d += kSeedNT) {
        uint32_t run = 0;
#pragma unroll
        for (int v = 0; v < kSeedWaves; ++v) {
            const uint32_t t = cnt[v][d];
            cnt[v][d] = run;
            run += t;
        }
        tstart[d] = run;
    }
    __syncthreads();
    if (wv == 0) wave_scan256(tstart, lane);
    __syncthreads();
    // place the tile in digit order
#pragma unroll
    for (int r = 0; r < kSeedRounds; ++r) {
        const uint64_t i = b * kSeedTile + tile_slot(wv, r, lane);
        if (i >= count) continue;
        const uint32_t d = (item[r].key(shift, mask) >> dshift) & 0xFFu;
        const uint32_t slot = tstart[d] + cnt[wv][d] + rank[r];
        if constexpr (HASH) stage_h[slot] = item[r].h;
        else stage_k[slot] = item[r].k;
        stage_p[slot] = item[r].p;
    }
    __syncthreads();
    // write out: consecutive slots of one digit go to consecutive addresses
    const uint64_t t0 = b * kSeedTile;
    const uint32_t nb = count - t0 < kSeedTile ? (uint32_t)(count - t0) : kSeedTile;
    for (uint32_t t = threadIdx.x; t < nb; t += kSeedNT) {
        SeedItem<HASH> it;
        if constexpr (HASH) it.h = stage_h[t];
        else it.k = stage_k[t];
        it.p = stage_p[t];
        const uint32_t d = (it.key(shift, mask) >> dshift) & 0xFFu;
        seed_store<HASH>(io, (uint64_t)gbase[d] + (t - tstart[d]), it);
    }
}

// 4. pointer table: ptr[j] = number of sorted entries with key < j, for
//    j = 0 .. nkeys: a merge of the implicit sequence 0 .. nkeys (A) with the
//    sorted keys (B), A first on ties; when A's j is merged, the B entries
//    merged before it are exactly those with key < j.  The merge path is cut
//    into diagonals of kMergeTile steps (one workgroup each); a first kernel
//    finds where each diagonal crosses A, so that every workgroup does the
//    same amount of work however the keys are spread.

// A's index at merge diagonal d: the number of A elements among the first d.
template <bool HASH>
__device__ __forceinline__ uint64_t merge_split(const uint64_t* hash, const uint32_t* keys,
                                                uint32_t shift, uint32_t mask, uint64_t nA,
                                                uint64_t nB, uint64_t d) {
    uint64_t lo = d > nB ? d - nB : 0, hi = d < nA ? d : nA;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        const uint64_t j = d - mid - 1;
        const uint64_t bk = HASH ? seed_key(hash[j], shift, mask) : keys[j];
        if (mid <= bk) lo = mid + 1;  // A[mid] = mid goes before B[j]
        else hi = mid;
    }
    return lo;
}

template <bool HASH>
__global__ void seed_ptr_split_kernel(const uint64_t* __restrict__ hash,
                                      const uint32_t* __restrict__ keys, uint64_t count,
                                      uint32_t shift, uint32_t mask, uint64_t nkeys,
                                      uint64_t nblocks, uint32_t* __restrict__ splits) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nblocks) return;
    const uint64_t nA = nkeys + 1, total = nA + count;
    const uint64_t d = t * kPtrChunk < total ? t * kPtrChunk : total;
    splits[t] = (uint32_t)merge_split<HASH>(hash, keys, shift, mask, nA, count, d);
}

template <bool HASH>
__global__ __launch_bounds__(kSeedNT) void seed_ptr_merge_kernel(
    const uint64_t* __restrict__ hash, const uint32_t* __restrict__ keys, uint64_t count,
    uint32_t shift, uint32_t mask, uint64_t nkeys, const uint32_t* __restrict__ splits,
    uint32_t* __restrict__ ptr) {
    constexpr int per = kPtrChunk / kSeedNT;  // merge steps per thread
    __shared__ uint32_t sB[kPtrChunk];        // this diagonal's B keys
    __shared__ uint32_t sOut[kPtrChunk];      // ptr of this diagonal's A elements
    const uint64_t nA = nkeys + 1, total = nA + count;
    const uint64_t d0 = (uint64_t)blockIdx.x * kPtrChunk;
    const uint64_t d1 = d0 + kPtrChunk < total ? d0 + kPtrChunk : total;
    const uint64_t i0 = splits[blockIdx.x], i1 = splits[blockIdx.x + 1];
    const uint64_t j0 = d0 - i0, j1 = d1 - i1;
    const uint32_t na = (uint32_t)(i1 - i0), nb = (uint32_t)(j1 - j0);
    for (uint32_t j = threadIdx.x; j < nb; j += kSeedNT)
        sB[j] = HASH ? seed_key(hash[j0 + j], shift, mask) : keys[j0 + j];
    __syncthreads();
    // this thread's sub-diagonal [dt, dt + per) of the window
    const uint32_t dt = threadIdx.x * per;
    if (dt < na + nb) {
        uint32_t lo = dt > nb ? dt - nb : 0, hi = dt < na ? dt : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) / 2;
            if (i0 + mid <= (uint64_t)sB[dt - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        uint32_t i = lo, j = dt - lo;
        for (int step = 0; step < per && i + j < na + nb; ++step) {
            if (i < na && (j >= nb || i0 + i <= (uint64_t)sB[j])) {
                sOut[i] = (uint32_t)(j0 + j);
                ++i;
            } else {
                ++j;
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < na; i += kSeedNT) ptr[i0 + i] = sOut[i];
}

// ---------------------------------------------------------------------------
// Launcher.
// ---------------------------------------------------------------------------
namespace {

uint64_t seed_tiles(uint64_t count) { return (count + kSeedTile - 1) / kSeedTile; }

uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

template <bool FIRST, bool HASH>
void seed_pass(const SeedBuffers& io, uint64_t count, uint32_t shift, uint32_t mask,
               uint32_t dshift, uint32_t* hist, uint32_t* totals, uint64_t nt, hipStream_t s) {
    hipLaunchKernelGGL((seed_hist_kernel<FIRST, HASH>), dim3((unsigned)nt), dim3(kSeedNT), 0, s,
                       io, count, shift, mask, dshift, hist, nt);
    hipLaunchKernelGGL(seed_scan_kernel, dim3(kDigits), dim3(kSeedNT), 0, s, hist, nt, totals);
    hipLaunchKernelGGL((seed_scatter_kernel<FIRST, HASH>), dim3((unsigned)nt), dim3(kSeedNT), 0,
                       s, io, count, shift, mask, dshift, hist, totals, nt);
}

}  // namespace

// Workspace: two carries of (8-byte hash or 4-byte key, 4-byte position),
// the digit-major tile histogram, the 256 digit totals and the merge-path
// splits of the pointer fill.
uint64_t merge_blocks(uint64_t count, uint32_t bits) {
    return ((1ull << bits) + 1 + count + kPtrChunk - 1) / kPtrChunk;
}

uint64_t seed_table_workspace_bytes(uint64_t count, uint32_t bits) {
    const uint64_t nt = seed_tiles(count);
    return 2 * align256(8 * count) + 2 * align256(4 * count) + align256(4ull * kDigits * nt) +
           align256(4ull * kDigits) + align256(4 * (merge_blocks(count, bits) + 1));
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
    uint32_t* hist = reinterpret_cast<uint32_t*>(wp + 2 * align256(4 * count));
    uint32_t* totals = reinterpret_cast<uint32_t*>(wp + 2 * align256(4 * count) +
                                                   align256(4ull * kDigits * nt));
    const bool with_hash = hash_out != nullptr;
    // the sorted keys (or hashes) the pointer fill reads
    const uint64_t* sorted_h = hash;
    const uint32_t* sorted_k = nullptr;
    if (count > 0) {
        const int passes = (int)((bits + 7) / 8);
        SeedBuffers io{};
        io.hash_in = hash;
        io.pos_in = pos;
        for (int p = 0; p < passes; ++p) {
            const bool last = p == passes - 1;
            const int o = p & 1;
            // outputs: the caller's arrays on the last pass, else a carry buffer
            io.pos_out = last ? pos_out : carryP[o];
            if (with_hash) io.hash_out = last ? hash_out : carryH[o];
            else io.key_out = reinterpret_cast<uint32_t*>(carryH[o]);  // keys in the hash slots
            const uint32_t dshift = 8u * (uint32_t)p;
            if (p == 0) {
                if (with_hash) seed_pass<true, true>(io, count, shift, mask, dshift, hist, totals, nt, s);
                else seed_pass<true, false>(io, count, shift, mask, dshift, hist, totals, nt, s);
            } else {
                if (with_hash) seed_pass<false, true>(io, count, shift, mask, dshift, hist, totals, nt, s);
                else seed_pass<false, false>(io, count, shift, mask, dshift, hist, totals, nt, s);
            }
            // this pass's outputs are the next pass's inputs
            io.pos_in = io.pos_out;
            if (with_hash) io.hash_in = io.hash_out;
            else io.key_in = io.key_out;
        }
        if (with_hash) sorted_h = hash_out;
        else sorted_k = io.key_in;
    }
    uint32_t* splits = reinterpret_cast<uint32_t*>(wp + 2 * align256(4 * count) +
                                                   align256(4ull * kDigits * nt) +
                                                   align256(4ull * kDigits));
    const uint64_t nblocks = merge_blocks(count, bits);
    const unsigned gs = (unsigned)((nblocks + 1 + kSeedNT - 1) / kSeedNT);
    if (count > 0 && !with_hash) {
        hipLaunchKernelGGL((seed_ptr_split_kernel<false>), dim3(gs), dim3(kSeedNT), 0, s, sorted_h,
                           sorted_k, count, shift, mask, nkeys, nblocks, splits);
        hipLaunchKernelGGL((seed_ptr_merge_kernel<false>), dim3((unsigned)nblocks), dim3(kSeedNT),
                           0, s, sorted_h, sorted_k, count, shift, mask, nkeys, splits, ptr);
    } else {
        hipLaunchKernelGGL((seed_ptr_split_kernel<true>), dim3(gs), dim3(kSeedNT), 0, s, sorted_h,
                           sorted_k, count, shift, mask, nkeys, nblocks, splits);
        hipLaunchKernelGGL((seed_ptr_merge_kernel<true>), dim3((unsigned)nblocks), dim3(kSeedNT),
                           0, s, sorted_h, sorted_k, count, shift, mask, nkeys, splits, ptr);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sws
