// api.cpp -- the extern "C" entry points of libsws (declared in sws.h): host-side
// validation, path choice and launch.  Nothing here touches device memory
// before every argument has been checked; nothing here allocates or waits.
#include "sws.h"

#include <stdint.h>
#include <string.h>

#include "sws_internal.hpp"

namespace {

bool known_flags(uint32_t flags, bool windows = true, bool kept = false) {
    const uint32_t ok = SWS_KMER_FORWARD | SWS_HASH_IDENTITY |
                        (windows ? SWS_SPLIT_AT_INVALID : 0u) | (kept ? SWS_WORKSPACE_KEPT : 0u);
    return (flags & ~ok) == 0u;
}

// Wavefronts a generic sliding-sum launch aims for, per calling thread
// (0: the default, which depends on w).  Thread-local, so calls from
// different threads never see each other's setting.
thread_local uint64_t t_sliding_waves = 0;

// Threads per workgroup of the single-sequence block kernel (32 < w <= 1024).
constexpr uint32_t kBlockThreads = 256;
// Threads per workgroup of the batched kernel unless the caller picks one.
constexpr uint32_t kBatchDefaultThreads = 256;

// Tiles of a single-sequence call: the same tile width the launch uses.
uint64_t max_tiles(uint64_t nwin, uint32_t k, uint32_t w) {
    const uint32_t tw = sws::minimizer_windows_per_tile(kBlockThreads, k, w);
    if (tw == 0) return 0;
    return (nwin + tw - 1) / tw;
}

constexpr uint32_t kMaxMinimizerWindow = 1024;  // keys per wavefront
constexpr uint64_t kMaxPositions = 0xFFFFFFFEull;

int check_minimizer_args(uint64_t n, uint32_t k, uint32_t w, uint32_t flags) {
    if (k < 1 || k > 31 || w < 1 || !known_flags(flags, true, true)) return SWS_ERR_INVALID;
    if (w > kMaxMinimizerWindow) return SWS_ERR_UNSUPPORTED;
    // the split semantics is built into the w <= 32 (wave-tile) kernels
    if ((flags & SWS_SPLIT_AT_INVALID) && w > sws::minimizer_wave_max_window())
        return SWS_ERR_UNSUPPORTED;
    if (n >= kMaxPositions) return SWS_ERR_UNSUPPORTED;
    return SWS_OK;
}

uint64_t window_count(uint64_t n, uint32_t k, uint32_t w) {
    const uint64_t need = (uint64_t)k + w - 1;
    return n >= need ? n - need + 1 : 0;
}

// Everything a minimizer call checks before it looks at its workspace.
int check_minimizer_call(uint64_t n, uint32_t k, uint32_t w, uint32_t flags,
                         const uint64_t* out_hash, const uint32_t* out_pos, uint64_t capacity,
                         const uint64_t* d_count) {
    const int st = check_minimizer_args(n, k, w, flags);
    if (st != SWS_OK) return st;
    if (d_count == nullptr) return SWS_ERR_INVALID;
    const uint64_t nwin = window_count(n, k, w);
    if (nwin > 0 && (out_hash == nullptr || out_pos == nullptr)) return SWS_ERR_INVALID;
    if (capacity < nwin) return SWS_ERR_CAPACITY;
    return SWS_OK;
}

int minimizers_common(const sws::GenomeInput& in, uint64_t n, uint32_t k, uint32_t w,
                      uint32_t flags, uint64_t* out_hash, uint32_t* out_pos, uint64_t capacity,
                      uint64_t* d_count, void* workspace, uint64_t ws_bytes, hipStream_t s) {
    const int st = check_minimizer_call(n, k, w, flags, out_hash, out_pos, capacity, d_count);
    if (st != SWS_OK) return st;
    const uint64_t nwin = window_count(n, k, w);
    const uint32_t tw = sws::minimizer_windows_per_tile(kBlockThreads, k, w);
    if (tw == 0) return SWS_ERR_UNSUPPORTED;  // unreachable for k <= 31, w <= 1024
    const uint64_t ntiles = nwin ? (nwin + tw - 1) / tw : 0;
    const uint64_t need = sws::minimizer_workspace_bytes(ntiles);
    if (workspace == nullptr || ws_bytes < need || ((uintptr_t)workspace & 7u)) return SWS_ERR_WORKSPACE;
    if (nwin == 0) {
        // nothing to compute; the count is still written on the stream
        return sws::launch_zero(d_count, 1, s) == 0 ? SWS_OK : SWS_ERR_DEVICE;
    }
    sws::MinimizerArgs a;
    memset(&a, 0, sizeof(a));
    a.k = k;
    a.w = w;
    a.flags = flags & ~(uint32_t)SWS_WORKSPACE_KEPT;  // the kernels see the k-mer flags only
    a.tw = tw;
    a.nwin = nwin;
    a.ntiles = ntiles;
    a.out_hash = out_hash;
    a.out_pos = out_pos;
    a.capacity = capacity;
    a.d_count = d_count;
    return sws::launch_minimizers(in, a, kBlockThreads, workspace, s,
                                  (flags & SWS_WORKSPACE_KEPT) != 0u) == 0
               ? SWS_OK
               : SWS_ERR_DEVICE;
}

}  // namespace

extern "C" {

uint32_t sws_abi_version(void) { return SWS_ABI_VERSION; }

const char* sws_status_str(int status) {
    switch (status) {
    case SWS_OK: return "SWS_OK";
    case SWS_ERR_INVALID: return "SWS_ERR_INVALID: invalid argument";
    case SWS_ERR_CAPACITY: return "SWS_ERR_CAPACITY: output capacity too small";
    case SWS_ERR_WORKSPACE: return "SWS_ERR_WORKSPACE: workspace missing, misaligned or too small";
    case SWS_ERR_DEVICE: return "SWS_ERR_DEVICE: kernel launch failed";
    case SWS_ERR_UNSUPPORTED: return "SWS_ERR_UNSUPPORTED: request not served by this build";
    default: return "unknown sws status";
    }
}

int sws_sliding_sum_ex(int op, uint64_t w, const void* x, uint64_t n, void* y, int path,
                       hipStream_t s) {
    if (op < SWS_OP_ADD_U32 || op > SWS_OP_AFFINE_U32) return SWS_ERR_INVALID;
    if (path < SWS_PATH_AUTO || path > SWS_PATH_SCALAR) return SWS_ERR_INVALID;
    if (w == 0) return SWS_ERR_INVALID;
    const bool idem = op == SWS_OP_MIN_U32 || op == SWS_OP_MAX_U32;
    if (path == SWS_PATH_LOG && !idem) return SWS_ERR_UNSUPPORTED;
    if (path == SWS_PATH_PREFIX && op != SWS_OP_ADD_U32) return SWS_ERR_UNSUPPORTED;
    if (n < w) return SWS_OK;
    if (x == nullptr || y == nullptr) return SWS_ERR_INVALID;
    const uintptr_t align = op == SWS_OP_AFFINE_U32 ? 8u : 4u;
    if (((uintptr_t)x | (uintptr_t)y) & (align - 1u)) return SWS_ERR_INVALID;
    const uint64_t count = n - w + 1;
    int use = path;
    // measured at n = 2^28: for w <= 64 the one-wave tiles of the prefix
    // difference (+) and of the doubling (min, max) beat the streaming generic
    // kernel by 2-7%; the prefix difference matches it up to w = 256 and is
    // 9-33% faster from w = 1024 on (its work does not grow with w)
    if (use == SWS_PATH_AUTO) {
        if (op == SWS_OP_ADD_U32) use = w <= 64 || w > 512 ? SWS_PATH_PREFIX : SWS_PATH_GENERIC;
        else if (idem) use = w <= 64 ? SWS_PATH_LOG : SWS_PATH_GENERIC;
        else use = SWS_PATH_GENERIC;
    }
    if (use == SWS_PATH_LOG) {
        if (w > sws::log_max_window()) return SWS_ERR_UNSUPPORTED;
        return sws::launch_sliding_log(op, x, n, (uint32_t)w, y, count, s) == 0 ? SWS_OK
                                                                               : SWS_ERR_DEVICE;
    }
    if (use == SWS_PATH_SCALAR) {
        if (w > sws::scalar_max_window()) return SWS_ERR_UNSUPPORTED;
        return sws::launch_sliding_scalar(op, x, n, (uint32_t)w, y, count, s) == 0
                   ? SWS_OK
                   : SWS_ERR_DEVICE;
    }
    if (w > sws::generic_max_window()) return SWS_ERR_UNSUPPORTED;
    const uint64_t waves = t_sliding_waves;  // 0: the launcher's default for (n, w)
    const int rc = use == SWS_PATH_PREFIX
                       ? sws::launch_sliding_prefix(op, x, n, (uint32_t)w, y, count, waves, s)
                       : sws::launch_sliding_generic(op, x, n, (uint32_t)w, y, count, waves, s);
    return rc == 0 ? SWS_OK : SWS_ERR_DEVICE;
}

int sws_sliding_sum(int op, uint64_t w, const void* x, uint64_t n, void* y, hipStream_t s) {
    return sws_sliding_sum_ex(op, w, x, n, y, SWS_PATH_AUTO, s);
}

}  // extern "C"

namespace {

// Windows above one slab go to the wide path on AUTO and GENERIC; LOG keeps
// its own limit, PREFIX and SCALAR do not serve them.
bool takes_wide_path(uint64_t w, int path) {
    return w > sws::generic_max_window() && (path == SWS_PATH_AUTO || path == SWS_PATH_GENERIC);
}

int check_sliding_args(int op, uint64_t w, int path) {
    if (op < SWS_OP_ADD_U32 || op > SWS_OP_AFFINE_U32) return SWS_ERR_INVALID;
    if (path < SWS_PATH_AUTO || path > SWS_PATH_SCALAR) return SWS_ERR_INVALID;
    if (w == 0) return SWS_ERR_INVALID;
    return SWS_OK;
}

}  // namespace

extern "C" {

int sws_sliding_sum_workspace(int op, uint64_t w, uint64_t n, int path, uint64_t* bytes) {
    if (bytes == nullptr) return SWS_ERR_INVALID;
    const int st = check_sliding_args(op, w, path);
    if (st != SWS_OK) return st;
    *bytes = (n >= w && takes_wide_path(w, path)) ? sws::wide_workspace_bytes(op, n, w) : 0;
    return SWS_OK;
}

int sws_sliding_sum_ws(int op, uint64_t w, const void* x, uint64_t n, void* y, int path,
                       void* workspace, uint64_t ws_bytes, hipStream_t s) {
    const int st = check_sliding_args(op, w, path);
    if (st != SWS_OK) return st;
    if (!takes_wide_path(w, path)) return sws_sliding_sum_ex(op, w, x, n, y, path, s);
    if (n < w) return SWS_OK;
    if (x == nullptr || y == nullptr) return SWS_ERR_INVALID;
    const uintptr_t align = op == SWS_OP_AFFINE_U32 ? 8u : 4u;
    if (((uintptr_t)x | (uintptr_t)y) & (align - 1u)) return SWS_ERR_INVALID;
    if (n >= (1ull << 40)) return SWS_ERR_UNSUPPORTED;  // grid of n / 2048 chunk workgroups
    if (workspace == nullptr || ws_bytes < sws::wide_workspace_bytes(op, n, w) ||
        ((uintptr_t)workspace & 7u))
        return SWS_ERR_WORKSPACE;
    return sws::launch_sliding_wide(op, x, n, w, y, n - w + 1, workspace, s) == 0 ? SWS_OK
                                                                                 : SWS_ERR_DEVICE;
}

int sws_pack2bit(const uint8_t* seq, uint64_t n, uint32_t* packed, uint32_t* invalid,
                 hipStream_t s) {
    if (n == 0) return SWS_OK;
    if (seq == nullptr || packed == nullptr) return SWS_ERR_INVALID;
    return sws::launch_pack2bit(seq, n, packed, invalid, s) == 0 ? SWS_OK : SWS_ERR_DEVICE;
}

int sws_kmers(const uint8_t* seq, uint64_t n, uint32_t k, uint32_t flags, uint64_t* out,
              hipStream_t s) {
    if (k < 1 || k > 31 || !known_flags(flags, false)) return SWS_ERR_INVALID;
    if (k >= 30 && (flags & SWS_HASH_IDENTITY) == 0u) return SWS_ERR_UNSUPPORTED;
    if (n < k) return SWS_OK;
    if (seq == nullptr || out == nullptr) return SWS_ERR_INVALID;
    if ((uintptr_t)out & 7u) return SWS_ERR_INVALID;
    sws::GenomeInput in;
    memset(&in, 0, sizeof(in));
    in.kind = sws::kInAscii;
    in.aligned = ((uintptr_t)seq & 15u) == 0;
    in.seq = seq;
    in.n = n;
    return sws::launch_kmers(in, k, flags, out, s) == 0 ? SWS_OK : SWS_ERR_DEVICE;
}

int sws_minimizers_workspace(uint64_t n, uint32_t k, uint32_t w, uint64_t* bytes) {
    if (bytes == nullptr) return SWS_ERR_INVALID;
    const int st = check_minimizer_args(n, k, w, 0);
    if (st != SWS_OK) return st;
    *bytes = sws::minimizer_workspace_bytes(max_tiles(window_count(n, k, w), k, w));
    return SWS_OK;
}

int sws_minimizers(const uint8_t* seq, uint64_t n, uint32_t k, uint32_t w, uint32_t flags,
                   uint64_t* out_hash, uint32_t* out_pos, uint64_t capacity, uint64_t* d_count,
                   void* workspace, uint64_t ws_bytes, hipStream_t s) {
    if (n > 0 && seq == nullptr) return SWS_ERR_INVALID;
    sws::GenomeInput in;
    memset(&in, 0, sizeof(in));
    in.kind = sws::kInAscii;
    in.aligned = ((uintptr_t)seq & 15u) == 0;
    in.seq = seq;
    in.n = n;
    return minimizers_common(in, n, k, w, flags, out_hash, out_pos, capacity, d_count, workspace,
                             ws_bytes, s);
}

int sws_minimizers_2bit(const uint32_t* packed, const uint32_t* invalid, uint64_t n, uint32_t k,
                        uint32_t w, uint32_t flags, uint64_t* out_hash, uint32_t* out_pos,
                        uint64_t capacity, uint64_t* d_count, void* workspace, uint64_t ws_bytes,
                        hipStream_t s) {
    if (n > 0 && packed == nullptr) return SWS_ERR_INVALID;
    if (((uintptr_t)packed | (uintptr_t)invalid) & 3u) return SWS_ERR_INVALID;
    sws::GenomeInput in;
    memset(&in, 0, sizeof(in));
    in.kind = sws::kIn2bit;
    in.packed = packed;
    in.invalid = invalid;
    in.n = n;
    return minimizers_common(in, n, k, w, flags, out_hash, out_pos, capacity, d_count, workspace,
                             ws_bytes, s);
}

int sws_minimizers_noalloc(const uint8_t* seq, uint64_t n, uint32_t k, uint32_t w, uint32_t flags,
                           uint64_t* out_hash, uint32_t* out_pos, uint64_t capacity,
                           uint64_t* d_count, hipStream_t s) {
    if (n > 0 && seq == nullptr) return SWS_ERR_INVALID;
    // the scratch is always cleared: whatever another call left there is no
    // state this call may rely on
    if (flags & SWS_WORKSPACE_KEPT) return SWS_ERR_INVALID;
    const int st = check_minimizer_call(n, k, w, flags, out_hash, out_pos, capacity, d_count);
    if (st != SWS_OK) return st;
    static_assert(sws::kNoAllocScratchBytes == SWS_NOALLOC_SCRATCH_BYTES, "scratch size");
    if (sws::minimizer_workspace_bytes(max_tiles(window_count(n, k, w), k, w)) >
        sws::kNoAllocScratchBytes)
        return SWS_ERR_WORKSPACE;
    // the scratch address belongs to one device: the stream's must be current
    int cur = -1;
    hipDevice_t sdev = -1;
    if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(s, &sdev) != hipSuccess) {
        (void)hipGetLastError();
        return SWS_ERR_DEVICE;
    }
    if ((int)sdev != cur) return SWS_ERR_INVALID;
    void* scratch = sws::noalloc_scratch(cur);
    if (scratch == nullptr) return SWS_ERR_DEVICE;
    sws::GenomeInput in;
    memset(&in, 0, sizeof(in));
    in.kind = sws::kInAscii;
    in.aligned = ((uintptr_t)seq & 15u) == 0;
    in.seq = seq;
    in.n = n;
    return minimizers_common(in, n, k, w, flags, out_hash, out_pos, capacity, d_count, scratch,
                             sws::kNoAllocScratchBytes, s);
}

// Batched calls need w <= 32 (one wavefront's tile) and k + w <= 49 (the
// boundary bits a lane tests fit in 64).
int check_batch_args(uint64_t total, uint32_t k, uint32_t w, uint32_t flags) {
    if (k < 1 || k > 31 || w < 1 || !known_flags(flags, true, true)) return SWS_ERR_INVALID;
    if (w > 32 || k + w > 49) return SWS_ERR_UNSUPPORTED;
    if (total >= kMaxPositions) return SWS_ERR_UNSUPPORTED;
    return SWS_OK;
}

uint64_t batch_tiles(uint64_t total, uint32_t k, uint32_t w) {
    const uint32_t tw = sws::batch_tile_windows(k, w);
    return total ? (total + tw - 1) / tw : 0;
}

int sws_minimizers_batch_workspace(uint64_t total_bases, uint32_t nreads, uint32_t k, uint32_t w,
                                   uint64_t* bytes) {
    (void)nreads;
    if (bytes == nullptr) return SWS_ERR_INVALID;
    const int st = check_batch_args(total_bases, k, w, 0);
    if (st != SWS_OK) return st;
    *bytes = sws::batch_workspace_bytes(batch_tiles(total_bases, k, w));
    return SWS_OK;
}

int sws_minimizers_batch_ex(const uint8_t* seqs, const uint64_t* d_offsets, uint32_t nreads,
                            uint64_t total_bases, uint32_t k, uint32_t w, uint32_t flags,
                            uint64_t* out_hash, uint32_t* out_pos, uint32_t* out_read,
                            uint64_t capacity, uint64_t* d_read_out_offsets, void* workspace,
                            uint64_t ws_bytes, uint32_t threads, hipStream_t s) {
    const int st = check_batch_args(total_bases, k, w, flags);
    if (st != SWS_OK) return st;
    if (threads == 0) threads = kBatchDefaultThreads;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512) return SWS_ERR_INVALID;
    if (d_offsets == nullptr || d_read_out_offsets == nullptr) return SWS_ERR_INVALID;
    if (total_bases > 0 && seqs == nullptr) return SWS_ERR_INVALID;
    if (capacity > 0 && (out_hash == nullptr || out_pos == nullptr || out_read == nullptr))
        return SWS_ERR_INVALID;
    const uint64_t ntiles = batch_tiles(total_bases, k, w);
    const uint64_t need = sws::batch_workspace_bytes(ntiles);
    if (workspace == nullptr || ws_bytes < need || ((uintptr_t)workspace & 7u)) return SWS_ERR_WORKSPACE;
    if (ntiles == 0) {
        // every read is empty: all offsets are 0
        return sws::launch_zero(d_read_out_offsets, (uint64_t)nreads + 1, s) == 0 ? SWS_OK
                                                                                 : SWS_ERR_DEVICE;
    }
    sws::GenomeInput in;
    memset(&in, 0, sizeof(in));
    in.kind = sws::kInAscii;
    in.aligned = ((uintptr_t)seqs & 15u) == 0;
    in.seq = seqs;
    in.n = total_bases;
    sws::BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.offsets = d_offsets;
    a.nreads = nreads;
    a.total = total_bases;
    a.k = k;
    a.w = w;
    a.flags = flags & ~(uint32_t)SWS_WORKSPACE_KEPT;  // the kernels see the k-mer flags only
    a.tw = sws::batch_tile_windows(k, w);
    a.ntiles = ntiles;
    a.out_hash = out_hash;
    a.out_pos = out_pos;
    a.out_read = out_read;
    a.capacity = capacity;
    a.read_out = d_read_out_offsets;
    return sws::launch_minimizers_batch(in, a, threads, workspace, s,
                                        (flags & SWS_WORKSPACE_KEPT) != 0u) == 0
               ? SWS_OK
               : SWS_ERR_DEVICE;
}

int sws_minimizers_batch(const uint8_t* seqs, const uint64_t* d_offsets, uint32_t nreads,
                         uint64_t total_bases, uint32_t k, uint32_t w, uint32_t flags,
                         uint64_t* out_hash, uint32_t* out_pos, uint32_t* out_read,
                         uint64_t capacity, uint64_t* d_read_out_offsets, void* workspace,
                         uint64_t ws_bytes, hipStream_t s) {
    return sws_minimizers_batch_ex(seqs, d_offsets, nreads, total_bases, k, w, flags, out_hash,
                                   out_pos, out_read, capacity, d_read_out_offsets, workspace,
                                   ws_bytes, 0, s);
}

int sws_seed_table_workspace(uint64_t count, uint32_t bits, uint64_t* bytes) {
    if (bytes == nullptr || bits < 1 || bits > 30) return SWS_ERR_INVALID;
    if (count > 0xFFFFFFFFull) return SWS_ERR_UNSUPPORTED;
    *bytes = sws::seed_table_workspace_bytes(count, bits);
    return SWS_OK;
}

int sws_seed_table(const uint64_t* hash, const uint32_t* pos, uint64_t count, uint32_t bits,
                   uint32_t shift, uint32_t* ptr, uint32_t* pos_out, uint64_t* hash_out,
                   void* workspace, uint64_t ws_bytes, hipStream_t s) {
    if (bits < 1 || bits > 30 || shift > 64u - bits || ptr == nullptr) return SWS_ERR_INVALID;
    if (count > 0xFFFFFFFFull) return SWS_ERR_UNSUPPORTED;
    if (count > 0 && (hash == nullptr || pos == nullptr || pos_out == nullptr))
        return SWS_ERR_INVALID;
    if (workspace == nullptr || ws_bytes < sws::seed_table_workspace_bytes(count, bits) ||
        ((uintptr_t)workspace & 15u))
        return SWS_ERR_WORKSPACE;
    return sws::launch_seed_table(hash, pos, count, bits, shift, ptr, pos_out, hash_out,
                                  workspace, s) == 0
               ? SWS_OK
               : SWS_ERR_DEVICE;
}

int sws_set_sliding_waves(uint64_t waves) {
    if (waves > (1ull << 24)) return SWS_ERR_INVALID;
    t_sliding_waves = waves;
    return SWS_OK;
}

}  // extern "C"
