// sws_internal.hpp -- declarations shared by the libsws host entry points and
// the kernel translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sws {

enum { kOpAdd = 0, kOpMin = 1, kOpMax = 2, kOpAffine = 3 };

// sliding.hip
uint32_t generic_max_window();
uint32_t log_max_window();
// target_waves: wavefronts the launch aims for; each streams
// ceil(slabs / target_waves) consecutive slabs (0: the default, 32768).
int launch_sliding_generic(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                           uint64_t target_waves, hipStream_t s);
uint32_t scalar_max_window();
int launch_sliding_scalar(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                          hipStream_t s);
int launch_sliding_prefix(int op, const void* x, uint64_t n, uint32_t w, void* y,
                          uint64_t count, uint64_t target_waves, hipStream_t s);
int launch_sliding_log(int op, const void* x, uint64_t n, uint32_t w, void* y, uint64_t count,
                       hipStream_t s);
// Windows longer than a slab (any w): chunked segment sums in a workspace.
uint64_t wide_workspace_bytes(int op, uint64_t n, uint64_t w);
int launch_sliding_wide(int op, const void* x, uint64_t n, uint64_t w, void* y, uint64_t count,
                        void* workspace, hipStream_t s);

// genome.hip
enum { kInAscii = 0, kIn2bit = 1 };
constexpr uint64_t kWsStatusOffset = 256;  // workspace: counter, error flag, then tile status
constexpr uint32_t kStatusStride = 8;      // status words one per 64-byte line
constexpr uint32_t kWaveTileGroup = 4;     // wave tiles per workgroup on the w <= 32 path
constexpr uint32_t kSplitFlag = 4;         // minimizer flag: invalid bases split the sequence

struct GenomeInput {
    int kind;                 // kInAscii or kIn2bit
    int aligned;              // seq is 16-byte aligned
    const uint8_t* seq;       // ASCII bases
    const uint32_t* packed;   // 2-bit words
    const uint32_t* invalid;  // invalid bits, may be null
    uint64_t n;
};

struct MinimizerArgs {
    uint32_t k, w, flags, tw;       // tw: windows stored per tile
    uint64_t nwin;                  // windows in the sequence
    uint64_t ntiles;
    uint64_t* out_hash;
    uint32_t* out_pos;
    uint64_t capacity;
    uint64_t* d_count;
    // workspace: a 256-byte header (error word at byte 8, the last call's
    // epoch at byte 16), then the look-back status words
    uint32_t* err;
    uint64_t* status;
    uint64_t* epoch;
};

struct BatchArgs {
    const uint64_t* offsets;  // nreads + 1
    uint32_t nreads;
    uint64_t total;           // bases in the batch
    uint32_t k, w, flags, tw;
    uint64_t ntiles;
    uint64_t* out_hash;
    uint32_t* out_pos;
    uint32_t* out_read;
    uint64_t capacity;
    uint64_t* read_out;       // nreads + 1
    uint32_t* first_read;     // workspace: per tile
    uint64_t* status;         // workspace
    uint32_t* err;            // workspace
    uint64_t* epoch;          // workspace header: epoch of the last call
};

int launch_zero(uint64_t* p, uint64_t words, hipStream_t s);
int launch_minimizers_batch(const GenomeInput& in, BatchArgs a, uint32_t nt, void* workspace,
                            hipStream_t s, bool kept);
uint64_t batch_workspace_bytes(uint64_t ntiles);
uint32_t batch_tile_windows(uint32_t k, uint32_t w);
int launch_pack2bit(const uint8_t* seq, uint64_t n, uint32_t* packed, uint32_t* invalid,
                    hipStream_t s);
int launch_kmers(const GenomeInput& in, uint32_t k, uint32_t flags, uint64_t* out, hipStream_t s);
uint32_t minimizer_tile_windows(uint32_t nt, uint32_t w);
uint32_t minimizer_wave_max_window();  // largest w of the wave-tile kernels
uint32_t minimizer_windows_per_tile(uint32_t nt, uint32_t k, uint32_t w);
uint64_t minimizer_workspace_bytes(uint64_t ntiles);
// The allocation-free minimizer call's scratch: a static device array of this
// many bytes.  noalloc_scratch(device) is its address on `device`, which must
// be the calling thread's current device (nullptr otherwise or on failure).
constexpr uint64_t kNoAllocScratchBytes = 4ull << 20;
void* noalloc_scratch(int device);

// Seed pointer/position tables (seedtable.hip).
uint64_t seed_table_workspace_bytes(uint64_t count, uint32_t bits);
int launch_seed_table(const uint64_t* hash, const uint32_t* pos, uint64_t count, uint32_t bits,
                      uint32_t shift, uint32_t* ptr, uint32_t* pos_out, uint64_t* hash_out,
                      void* workspace, hipStream_t s);
int launch_minimizers(const GenomeInput& in, MinimizerArgs a, uint32_t nt, void* workspace,
                      hipStream_t s, bool kept);

}  // namespace sws
