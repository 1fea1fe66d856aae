/*
 * sws.h -- C ABI of libsws: sliding window sums and minimizer seed tables on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Snytsar & Turakhia, "Parallel approach to
 * sliding window sums" (arXiv:1811.10074):
 *   - the sliding window sum of Sec. 2.2, Eq. 2:
 *       y_i = x_i (+) x_{i+1} (+) ... (+) x_{i+w-1},  i = 0 .. n-w,
 *     exactly w addends per output, for an associative operator (+);
 *   - k-mers of a DNA sequence as a sliding sum of bases under concatenation
 *     (Sec. 2.4), their canonical form and hash (Sec. 4 hashes the k-mers);
 *   - minimizer seeds (Sec. 2.4, Fig. 2): for each window of w consecutive
 *     k-mers, the smallest (hash, position) pair; adjacent windows that share
 *     the pair store it once.
 *
 * Conventions for every entry point:
 *   - Data pointers are device pointers owned by the caller.  The library
 *     never allocates, frees or synchronizes; every byte of scratch comes from
 *     the caller's workspace (sws_minimizers_noalloc alone uses a static
 *     device array instead); all work is enqueued on the given stream, so the
 *     calls may be captured into a HIP graph.
 *   - Arguments are validated on the host before anything is enqueued.  On
 *     any error status nothing is enqueued and nothing is written.
 *   - SWS_ERR_DEVICE means the launch itself failed (hipGetLastError).
 *     Faults during execution surface at the caller's next synchronization.
 *   - Calls are re-entrant and keep no process-wide state (except
 *     sws_minimizers_noalloc's scratch array); calls on different streams may
 *     overlap as long as they do not share a workspace or an output buffer.
 *   - Every integer result is exact; there is no floating point anywhere.
 */
#ifndef SWS_H
#define SWS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2: seed tables, the prefix-difference and scalar-input paths, SWS_SPLIT_AT_INVALID,
 *    SWS_WORKSPACE_KEPT (all additions; no call changed its meaning).
 * 3: sws_minimizers_batch_ex takes the workgroup size per call; the process-wide
 *    sws_set_minimizer_block is gone; sws_set_sliding_waves is per thread.
 * 4: sws_sliding_sum_workspace / sws_sliding_sum_ws (windows of any length) and
 *    sws_minimizers_noalloc (additions; no call changed its meaning).
 * 5: the batched calls accept SWS_WORKSPACE_KEPT (an addition). */
#define SWS_ABI_VERSION 5u

typedef enum {
    SWS_OK = 0,
    SWS_ERR_INVALID = -1,     /* bad argument: unknown op/flag/path, w = 0, k outside [1, 31], null pointer with n > 0 */
    SWS_ERR_CAPACITY = -2,    /* output capacity below the bound stated for the call */
    SWS_ERR_WORKSPACE = -3,   /* workspace null or smaller than the size the *_workspace query returns */
    SWS_ERR_DEVICE = -4,      /* a kernel launch failed */
    SWS_ERR_UNSUPPORTED = -5  /* a valid request this build does not serve (see each call) */
} sws_status;

/* Operators of the sliding sum.  Elements and results share one type. */
typedef enum {
    SWS_OP_ADD_U32 = 0,    /* uint32, (a + b) mod 2^32, identity 0                                     */
    SWS_OP_MIN_U32 = 1,    /* uint32, unsigned min, identity 2^32 - 1                                 */
    SWS_OP_MAX_U32 = 2,    /* uint32, unsigned max, identity 0                                        */
    SWS_OP_AFFINE_U32 = 3  /* pairs (a, b) of uint32, interleaved a0 b0 a1 b1 ...: the map z -> a z + b;
                              (a,b) (+) (c,d) = (a c, a d + b) mod 2^32, the composition f_ab(f_cd(z));
                              associative, not commutative, identity (1, 0)                            */
} sws_op;

/* How the sliding sum is computed.  All paths give identical bits. */
typedef enum {
    SWS_PATH_AUTO = 0,    /* the library picks per (op, w): ADD: PREFIX for w <= 64 or w > 512; MIN and
                             MAX: LOG for w <= 64; else GENERIC (the fastest measured at n = 2^28)       */
    SWS_PATH_GENERIC = 1, /* block prefix/suffix scans: Alg. 2 of Sec. 3.1 with block length w, any
                             associative op, O(1) operator applications per output                    */
    SWS_PATH_LOG = 2,     /* doubling of overlapping windows, O(log w) per output; only for MIN and MAX,
                             whose idempotence lets two overlapping halves cover a window (Sec. 3.1,
                             the commutative case); SWS_ERR_UNSUPPORTED for ADD and AFFINE            */
    SWS_PATH_PREFIX = 3,  /* difference of running prefixes, y_i = P_{i+w-1} - P_{i-1} (the invertible
                             case named in the conclusion): one scan, cost independent of w; only for
                             ADD; SWS_ERR_UNSUPPORTED for the others                                  */
    SWS_PATH_SCALAR = 4   /* Alg. 1 of Sec. 3.1 (scalar input): one wavefront keeps the w-1 running
                             suffix sums in its lanes and takes the input one element at a time; any
                             op, w <= 64 (SWS_ERR_UNSUPPORTED above)                                  */
} sws_path;

/* k-mer / minimizer flags (bitwise or). */
enum {
    SWS_KMER_CANONICAL = 0u, /* min(forward, reverse complement)                          */
    SWS_KMER_FORWARD = 1u,   /* forward strand only (the lexicographic seeds of Fig. 2)   */
    SWS_HASH_MIX64 = 0u,     /* hash each k-mer with mix64 (below)                        */
    SWS_HASH_IDENTITY = 2u,  /* use the k-mer value itself                                */
    SWS_SPLIT_AT_INVALID = 4u, /* minimizers only: invalid bases split the sequence into
                                  segments and a window holding an invalid k-mer stores
                                  nothing (each segment as its own sequence, positions
                                  kept); w <= 32, else SWS_ERR_UNSUPPORTED            */
    SWS_WORKSPACE_KEPT = 8u    /* sws_minimizers / sws_minimizers_2bit and the batched
                                  calls (sws_minimizers_batch / _ex) only: the workspace
                                  holds what the previous call with this flag left, or
                                  was zero-filled, and nothing else wrote it since; the
                                  call then skips clearing it (one kernel launch fewer).
                                  Call without the flag (or zero-fill) at least once
                                  every 2^30 calls.  Not a k-mer option: no effect on
                                  the results                                        */
};

/*
 * Base coding (Sec. 2.4 sorts seeds lexicographically): A/a = 0, C/c = 1,
 * G/g = 2, T/t = 3; every other byte (N, IUPAC codes, ...) is invalid.  The
 * k-mer starting at i has the value sum_j code(s_{i+j}) * 4^(k-1-j) (forward)
 * and sum_j (3 - code(s_{i+j})) * 4^j (reverse complement), so numeric order is
 * lexicographic order.  A k-mer that covers an invalid base is invalid.
 *
 * mix64 (the paper names no hash; this one is fixed by the library and is
 * invertible): all arithmetic mod 2^64,
 *   x ^= x >> 32; x *= 0x9E3779B97F4A7C15; x ^= x >> 29;
 *   x *= 0x243F6A8885A308D3; x ^= x >> 32.
 */

/* ------------------------------------------------------------------------ */
/* Sliding window sum, Sec. 2.2 Eq. 2.                                        */
/* ------------------------------------------------------------------------ */

/*
 * y[i] = x[i] (+) ... (+) x[i+w-1] for i = 0 .. n-w.
 *   op  : sws_op.
 *   w   : window length, >= 1.  n < w is not an error: no outputs, nothing
 *         enqueued.
 *   x   : device array of n elements (uint32, or uint32 pairs for AFFINE),
 *         4-byte aligned (8-byte for AFFINE).  The fast path wants 16-byte
 *         alignment of x and y; other alignments are served by a slower path
 *         with identical results.
 *   y   : device array receiving n - w + 1 elements of the same type; must not
 *         overlap x.
 *   s   : stream (0 = the null stream).
 * Errors: SWS_ERR_INVALID (op unknown, w = 0, x or y null with n >= w,
 * misaligned element pointer), SWS_ERR_DEVICE.
 */
int sws_sliding_sum(int op, uint64_t w, const void *x, uint64_t n, void *y, hipStream_t s);

/* As sws_sliding_sum with an explicit path (sws_path).  SWS_PATH_LOG with ADD
 * or AFFINE, and SWS_PATH_PREFIX with anything but ADD, return
 * SWS_ERR_UNSUPPORTED. */
int sws_sliding_sum_ex(int op, uint64_t w, const void *x, uint64_t n, void *y, int path,
                       hipStream_t s);

/*
 * Windows of any length.  sws_sliding_sum and sws_sliding_sum_ex serve
 * w <= 2048 (the log path to 4096, the scalar path to 64) and return
 * SWS_ERR_UNSUPPORTED above.  These two serve every w >= 1 (Eq. 2 has no
 * bound on w): on SWS_PATH_AUTO and SWS_PATH_GENERIC, a window longer than
 * 2048 is computed by the same segment identity as the generic path with
 * segments of w elements cut into chunks of 2048: the window at offset o of a
 * segment is the segment's suffix from o followed by the next segment's prefix
 * up to o - 1, and per-chunk sums (in the workspace) carry both across chunks.
 * Any associative op; x is read three times.  SWS_PATH_LOG keeps its limit
 * (4096), SWS_PATH_PREFIX its limit (2048), SWS_PATH_SCALAR its limit (64).
 */

/* Workspace bytes sws_sliding_sum_ws needs for (op, w, n, path): 0 when the
 * request takes a path without scratch (w <= 2048, or a path other than AUTO
 * and GENERIC), else 3 values per chunk of 2048 offsets per segment of w.
 * Errors: SWS_ERR_INVALID (op, path, w = 0, bytes null). */
int sws_sliding_sum_workspace(int op, uint64_t w, uint64_t n, int path, uint64_t *bytes);

/* As sws_sliding_sum_ex, for any w.  workspace: ws_bytes bytes of device
 * scratch, 8-byte aligned, at least sws_sliding_sum_workspace(op, w, n, path)
 * (may be NULL when that is 0); contents on entry do not matter.
 * Errors: as sws_sliding_sum_ex, plus SWS_ERR_WORKSPACE. */
int sws_sliding_sum_ws(int op, uint64_t w, const void *x, uint64_t n, void *y, int path,
                       void *workspace, uint64_t ws_bytes, hipStream_t s);

/* ------------------------------------------------------------------------ */
/* 2-bit packing, k-mers.                                                     */
/* ------------------------------------------------------------------------ */

/*
 * Packs n ASCII bases into 2-bit codes.
 *   packed  : ceil(n/16) uint32 words; base i occupies bits [31-2(i%16) .. 30-2(i%16)]
 *             of word i/16 (first base in the most significant bits).  Invalid
 *             bases are stored as code 0.  Bits past n are zero.
 *   invalid : ceil(n/32) uint32 words, or NULL; bit (i%32) of word i/32 is set iff
 *             base i is invalid.  Bits past n are zero.
 * Errors: SWS_ERR_INVALID (null pointer with n > 0), SWS_ERR_DEVICE.
 */
int sws_pack2bit(const uint8_t *seq, uint64_t n, uint32_t *packed, uint32_t *invalid,
                 hipStream_t s);

/*
 * out[i] for i = 0 .. n-k: the canonical (or forward, SWS_KMER_FORWARD) k-mer
 * value at i, hashed with mix64 unless SWS_HASH_IDENTITY; UINT64_MAX when the
 * k-mer covers an invalid base.  n < k: no outputs.
 *   k     : 1 .. 31.  With hashing, k must be <= 29: for k = 30, 31 one valid
 *           k-mer hashes to UINT64_MAX and could not be told from an invalid
 *           one, so those requests return SWS_ERR_UNSUPPORTED.
 * Errors: SWS_ERR_INVALID, SWS_ERR_UNSUPPORTED, SWS_ERR_DEVICE.
 */
int sws_kmers(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t flags, uint64_t *out,
              hipStream_t s);

/* ------------------------------------------------------------------------ */
/* Minimizers, Sec. 2.4 / Fig. 2.                                             */
/* ------------------------------------------------------------------------ */

/*
 * Window p (p = 0 .. n-k-w+1) holds the k-mers starting at p .. p+w-1.  Its
 * minimizer is the smallest (value, position) pair among its valid k-mers
 * (value = hash or k-mer value as flagged; ties go to the leftmost position).
 * A window without a valid k-mer has no minimizer.  The minimizer of window p
 * is stored iff it exists and differs from that of window p-1 (p = 0 always
 * stores).  Outputs are in ascending position.
 *
 * Output bound: at most max(0, n-k-w+2) minimizers; capacity below that bound
 * is SWS_ERR_CAPACITY.  Positions are uint32, so n must be < 2^32 - 1
 * (SWS_ERR_UNSUPPORTED otherwise).
 */

/* Workspace bytes sws_minimizers / sws_minimizers_2bit need for n bases. */
int sws_minimizers_workspace(uint64_t n, uint32_t k, uint32_t w, uint64_t *bytes);

/*
 *   seq       : n ASCII bases (device).
 *   k, w      : 1 <= k <= 31, w >= 1.
 *   flags     : SWS_KMER_* | SWS_HASH_*.
 *   out_hash  : capacity uint64 (device): value of each stored minimizer.
 *   out_pos   : capacity uint32 (device): its k-mer start position.
 *   d_count   : one uint64 (device): receives the number stored, or UINT64_MAX
 *               if the kernel detected an internal error (a tile that waited
 *               too long for its predecessors' counts; outputs are then
 *               unusable).
 *   workspace : ws_bytes bytes of device scratch, 8-byte aligned, at least
 *               sws_minimizers_workspace(n, k, w); its contents on entry do
 *               not matter (the call clears what it uses), unless flags holds
 *               SWS_WORKSPACE_KEPT (see there).  The call leaves it valid for
 *               a later call with that flag, of any size it is large enough for.
 */
int sws_minimizers(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t w, uint32_t flags,
                   uint64_t *out_hash, uint32_t *out_pos, uint64_t capacity, uint64_t *d_count,
                   void *workspace, uint64_t ws_bytes, hipStream_t s);

/* As sws_minimizers, from the 2-bit layout of sws_pack2bit: packed
 * (ceil(n/16) words, 4-byte aligned) and invalid (ceil(n/32) words, or NULL when
 * every base is valid). */
int sws_minimizers_2bit(const uint32_t *packed, const uint32_t *invalid, uint64_t n, uint32_t k,
                        uint32_t w, uint32_t flags, uint64_t *out_hash, uint32_t *out_pos,
                        uint64_t capacity, uint64_t *d_count, void *workspace, uint64_t ws_bytes,
                        hipStream_t s);

/*
 * sws_minimizers without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The call allocates nothing and calls no
 * allocating routine; its look-back scratch is a static device array of
 * SWS_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU, held from
 * the first call on that GPU until the process ends.
 *   Arguments and results: as sws_minimizers (ASCII input).
 *   flags     : SWS_KMER_* | SWS_HASH_* | SWS_SPLIT_AT_INVALID; the scratch is
 *               cleared on every call (one small kernel), so SWS_WORKSPACE_KEPT
 *               is SWS_ERR_INVALID.
 *   s         : a stream of the calling thread's current device (the null
 *               stream included); a stream of another device is
 *               SWS_ERR_INVALID.
 * Limit: the request must fit the array, i.e. sws_minimizers_workspace(n, k, w)
 * <= SWS_NOALLOC_SCRATCH_BYTES (256 bytes plus 64 per look-back participant:
 * about 2.6e8 bases at w <= 32, about 2.6e8 windows above); a larger request
 * is SWS_ERR_WORKSPACE and enqueues nothing.
 * Concurrency: every call on one GPU uses that GPU's one array, so calls that
 * overlap on one GPU (other streams, other threads) race and their results
 * are undefined; serialize them, or use sws_minimizers with a workspace each.
 * Errors: as sws_minimizers, plus SWS_ERR_DEVICE when the array's address
 * cannot be obtained.
 */
#define SWS_NOALLOC_SCRATCH_BYTES (4u << 20)
int sws_minimizers_noalloc(const uint8_t *seq, uint64_t n, uint32_t k, uint32_t w, uint32_t flags,
                           uint64_t *out_hash, uint32_t *out_pos, uint64_t capacity,
                           uint64_t *d_count, hipStream_t s);

/* ------------------------------------------------------------------------ */
/* Batched minimizers over many reads in one launch.                          */
/* ------------------------------------------------------------------------ */

/* Workspace bytes sws_minimizers_batch needs. */
int sws_minimizers_batch_workspace(uint64_t total_bases, uint32_t nreads, uint32_t k, uint32_t w,
                                   uint64_t *bytes);

/*
 * Reads r = 0 .. nreads-1 are seqs[d_offsets[r] .. d_offsets[r+1]) (ASCII,
 * device), with d_offsets non-decreasing, d_offsets[0] = 0 and
 * d_offsets[nreads] = total_bases.  Each read is treated as its own sequence
 * (as sws_minimizers): no k-mer or window spans two reads and positions are
 * relative to the read start.  Outputs are read-major in input order:
 *   out_hash, out_pos, out_read : capacity entries each (device);
 *   d_read_out_offsets          : nreads + 1 uint64 (device): read r's
 *                                 minimizers are entries [off[r], off[r+1]);
 *                                 off[nreads] is the total.
 * The offsets live on the device, so the exact bound
 * sum_r max(0, len_r - k - w + 2) is the caller's to compute; the kernels never
 * write an entry at or past capacity, and off[nreads] reports the full total,
 * so a total above capacity means the outputs were truncated.
 * total_bases must be < 2^32 - 1 (SWS_ERR_UNSUPPORTED otherwise).
 * flags: SWS_KMER_* | SWS_HASH_* | SWS_SPLIT_AT_INVALID | SWS_WORKSPACE_KEPT.
 * workspace: ws_bytes bytes of device scratch, 8-byte aligned, at least
 * sws_minimizers_batch_workspace(total_bases, nreads, k, w); its contents on
 * entry do not matter (the call clears what it uses), unless flags holds
 * SWS_WORKSPACE_KEPT (see there); the call leaves it valid for a later
 * batched call with that flag, of any size it is large enough for.
 */
int sws_minimizers_batch(const uint8_t *seqs, const uint64_t *d_offsets, uint32_t nreads,
                         uint64_t total_bases, uint32_t k, uint32_t w, uint32_t flags,
                         uint64_t *out_hash, uint32_t *out_pos, uint32_t *out_read,
                         uint64_t capacity, uint64_t *d_read_out_offsets, void *workspace,
                         uint64_t ws_bytes, hipStream_t s);

/*
 * As sws_minimizers_batch with the threads per workgroup of the launch chosen
 * by the caller (the autotuner's knob): 64, 128, 256 or 512 (1, 2, 4 or 8
 * wavefront tiles of 1024 k-mer positions per workgroup), or 0 for the
 * default (256).  Results do not depend on it.  Any other value:
 * SWS_ERR_INVALID.
 */
int sws_minimizers_batch_ex(const uint8_t *seqs, const uint64_t *d_offsets, uint32_t nreads,
                            uint64_t total_bases, uint32_t k, uint32_t w, uint32_t flags,
                            uint64_t *out_hash, uint32_t *out_pos, uint32_t *out_read,
                            uint64_t capacity, uint64_t *d_read_out_offsets, void *workspace,
                            uint64_t ws_bytes, uint32_t threads, hipStream_t s);

/* ------------------------------------------------------------------------ */
/* Seed pointer table and seed position table, Sec. 2.4 and Fig. 1.           */
/* ------------------------------------------------------------------------ */

/* Workspace bytes sws_seed_table needs for `count` entries. */
int sws_seed_table_workspace(uint64_t count, uint32_t bits, uint64_t *bytes);

/*
 * Builds the seed table of Fig. 1 over count entries (hash[i], pos[i]), taken
 * in input order (the output of sws_minimizers is in position order).  The
 * table is keyed by key(h) = (h >> shift) mod 2^bits: with the k-mer value as
 * the hash (SWS_HASH_IDENTITY), shift = 0 and bits = 2k it is the paper's
 * table over all 4^k seeds in lexicographic order; with mix64 hashes, the top
 * bits (shift = 64 - bits) give a hash-bucketed table.
 *   hash, pos : device arrays of count entries (u64, u32); not modified.
 *   count     : < 2^32.
 *   bits      : 1 .. 30; shift + bits <= 64.
 *   ptr       : device u32[2^bits + 1]: ptr[j] = number of entries with
 *               key < j, so the hits of key j are pos_out[ptr[j] .. ptr[j+1]).
 *               The paper's table, whose entry for a seed closes that seed's
 *               list, is ptr + 1.
 *   pos_out   : device u32[count]: the positions grouped by key, ascending,
 *               each group in input order.
 *   hash_out  : device u64[count] receiving the hashes in the same order, or
 *               NULL.
 *   workspace : ws_bytes bytes of device scratch, 16-byte aligned, at least
 *               sws_seed_table_workspace(count, bits); contents on entry do
 *               not matter.
 * Outputs must not overlap the inputs or each other.
 * Errors: SWS_ERR_INVALID (bits or shift out of range, null array with
 * count > 0, null ptr), SWS_ERR_UNSUPPORTED (count >= 2^32),
 * SWS_ERR_WORKSPACE, SWS_ERR_DEVICE.
 */
int sws_seed_table(const uint64_t *hash, const uint32_t *pos, uint64_t count, uint32_t bits,
                   uint32_t shift, uint32_t *ptr, uint32_t *pos_out, uint64_t *hash_out,
                   void *workspace, uint64_t ws_bytes, hipStream_t s);

/* ------------------------------------------------------------------------ */
/* Launch configuration (used by the autotuner).                              */
/* ------------------------------------------------------------------------ */

/*
 * Sets how many wavefronts a generic-path (or streaming prefix-path)
 * sliding-sum launch aims for.  The input is cut into slabs of 64*R elements
 * (R = 8, 16 or 32 by window and operator) and each wavefront streams
 * ceil(slabs / waves) consecutive slabs, so fewer waves means longer streams
 * per wave.  0 restores the default (32768, 128 per compute unit; 65536 for
 * AFFINE with w <= 512).  Results
 * do not depend on it.  The setting belongs to the
 * calling thread: it applies to that thread's later calls only.
 * Errors: SWS_ERR_INVALID (waves > 2^24).
 */
int sws_set_sliding_waves(uint64_t waves);

/* Human-readable name of a status code (static storage). */
const char *sws_status_str(int status);

/* SWS_ABI_VERSION of the loaded library. */
uint32_t sws_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SWS_H */
