/*
 * rs.h -- C ABI of librs, an MI355X (gfx950) integer-sorting library for the
 * hot path of Gerbessiotis, "Integer sorting on multicores: some (experiments
 * and) observations" (arXiv 1708.09495).
 *
 * The paper states the problem as sorting n integer keys with radix-r
 * count-sort rounds (Section 3, Eq. Ts and Eq. Tp) or with the block
 * networks BTN and OET on p sorted runs (Section 2, Section 3 Eq. To and
 * Eq. Tb).  This library sorts unsigned 32- or 64-bit keys ascending.
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller.  The
 *     library never allocates, frees or retains them.  Scratch memory comes
 *     only from the caller's workspace `ws` of `ws_bytes` bytes, which must be
 *     at least rs_workspace_bytes(...) for the same arguments and 256-byte
 *     aligned.  The workspace must not be shared by calls that may overlap.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *     on it and the call returns without waiting: results are valid once the
 *     stream has been synchronised.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and returned synchronously; nothing is written in that case.  A HIP
 *     launch failure returns RS_ERR_HIP.  Device faults surface at the
 *     caller's next synchronisation, as for any HIP work.
 *   - `in == out` (and vals_in == vals_out) is allowed: the sort is then in
 *     place.  A key-value sort is in place for both arrays or for neither
 *     (keys_in == keys_out exactly when vals_in == vals_out), else
 *     RS_ERR_INVALID.  Other overlaps are not allowed.
 *   - n = 0 is valid and enqueues nothing.
 *   - The library never aborts the process.
 *   - The radix rounds take their tiles in an XCD-aware order (chunks of 16
 *     neighbouring tiles per XCD, so that the cache lines neighbouring
 *     tiles' outputs share meet in one L2) on devices of 256 compute units
 *     in 8 XCDs, where the hardware hands workgroup b to XCD b mod 8, for
 *     sorts of at least 1,024 tiles (about 15 million uint32 keys); the
 *     environment variable RS_XCD_ORDER=0 (read once per device and
 *     process) keeps the order in which workgroups reach one counter.
 *     Results are the same either way.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RS_OK = 0,
    RS_ERR_INVALID = 1,      /* bad argument (NULL pointer, bad width, ...)   */
    RS_ERR_UNSUPPORTED = 2,  /* valid request the library does not serve     */
    RS_ERR_WORKSPACE = 3,    /* workspace NULL, too small or misaligned       */
    RS_ERR_HIP = 4           /* a HIP runtime call failed                     */
} rs_status;

typedef enum {
    RS_ALGO_AUTO = 0,       /* tuned choice for the size                     */
    RS_ALGO_LSD = 1,        /* radix-2^b count-sort rounds (Section 3)       */
    RS_ALGO_BTN = 2,        /* block bitonic on p runs (Section 2, Eq. Tb)   */
    RS_ALGO_OET = 3,        /* block odd-even transposition (Sec. 2, Eq. To) */
    RS_ALGO_LEARNED = 4,    /* learned-CDF buckets, LSD fallback             */
    RS_ALGO_LDS_RADIX = 5   /* one workgroup's LDS radix sort (small n)      */
} rs_algo;

typedef enum {
    RS_OP_SORT = 0,       /* rs_sort_u32 / rs_sort_u64                 */
    RS_OP_SORT_KV = 1,    /* rs_sort_kv                                */
    RS_OP_BATCH = 2,      /* rs_sort_batch_u32                         */
    RS_OP_SEGMENTED = 3,  /* rs_sort_segmented                         */
    RS_OP_TUNE = 4,       /* rs_tune_run (n = instances)               */
    RS_OP_BLOCKS = 5      /* rs_sort_blocks_u32 (num_segments = p)     */
} rs_op;

/* Facts about the most recent call made on the calling host thread. */
typedef struct {
    int32_t algo;               /* rs_algo actually run                        */
    int32_t radix_bits;         /* b of the count-sort rounds (0 if none)      */
    int32_t passes;             /* count-sort rounds run: ceil(w/b)            */
    int32_t runs_p;             /* p of BTN/OET (runs per instance)            */
    int64_t network_stages;     /* BTN: lg p (lg p+1)/2; OET: p                */
    int32_t tile_keys;          /* keys per workgroup tile of the LSD rounds   */
    int32_t fallback;           /* learned path: 1 if plain LSD was used       */
    int64_t buckets_overflowed; /* learned path: buckets over LDS capacity     */
    int64_t keys_overflowed;    /* learned path: keys in those buckets         */
    double  train_loss;         /* learned path: final training loss           */
    uint32_t device_error;      /* bit 0: a bounded wait gave up; bit 1: a computed
                                   destination was out of range (not written)    */
    int32_t hip_error;          /* hipError_t of the failing call when RS_ERR_HIP */
    int32_t passes_skipped;     /* RS_ALGO_AUTO: rounds of `passes` not run because
                                   every key has the same digit there           */
} rs_stats;

/* Sort n uint32 keys ascending.  Follows Section 3: ceil(32/b) stable
 * count-sort rounds at radix 2^b from the least significant digit, each a
 * per-tile digit histogram, a device-wide exclusive scan and a stable
 * rank-and-scatter.  radix_bits in [1, 16]; 0 = default (8).  algo: LSD runs
 * every round; AUTO (radix_bits <= 11) skips the rounds whose digit is the
 * same for every key -- such a stable round is the identity; the all-round
 * histogram shows them, and the choice is made on the device --; LDS_RADIX
 * for n <= rs_small_capacity(4) (one workgroup); BTN/OET: one workgroup up
 * to that size, above it rs_sort_blocks_u32 with p = 0.
 * Layout: `in` and `out` are dense arrays of n keys.  n < 2^32 (digit
 * counts and prefixes are 32-bit words); larger n returns
 * RS_ERR_UNSUPPORTED. */
rs_status rs_sort_u32(const uint32_t* in, uint32_t* out, size_t n, int radix_bits,
                      rs_algo algo, void* ws, size_t ws_bytes, void* stream);

/* As rs_sort_u32 for uint64 keys: ceil(64/b) rounds.  algo LEARNED sorts
 * with learned-CDF buckets (keys only). */
rs_status rs_sort_u64(const uint64_t* in, uint64_t* out, size_t n, int radix_bits,
                      rs_algo algo, void* ws, size_t ws_bytes, void* stream);

/* Stable key-value sort: keys of key_bytes (4 or 8), values of val_bytes
 * (4 or 8) move with their key; equal keys keep their input order.
 * algo: AUTO, LSD or LEARNED (LEARNED needs key_bytes = 8). */
rs_status rs_sort_kv(const void* keys_in, const void* vals_in, void* keys_out, void* vals_out,
                     size_t n, int key_bytes, int val_bytes, int radix_bits, rs_algo algo,
                     void* ws, size_t ws_bytes, void* stream);

/* Sort `count` independent uint32 arrays of n keys each, stored back to back
 * (array i at in + i*n), one workgroup per array, in one launch.  algo BTN
 * or OET: the block networks of Section 2 on p runs of n_pad/p keys, where
 * n_pad is the next power of two >= n and the tail is padded with
 * UINT32_MAX; p = 0 picks the tuned p.  algo LDS_RADIX: radix-2^8 rounds in
 * LDS.  AUTO: the tuned fastest.  Requires n <= rs_small_capacity(4). */
rs_status rs_sort_batch_u32(const uint32_t* in, uint32_t* out, size_t n, size_t count,
                            rs_algo algo, int p, void* ws, size_t ws_bytes, void* stream);

/* Batched segmented sort: segment s is [offsets[s], offsets[s+1]) of `in`
 * (offsets: DEVICE array of num_segments+1 non-decreasing int64,
 * offsets[0] = 0, offsets[num_segments] = total_n; empty segments allowed;
 * no segment may exceed 2^32 - 1 keys).  Each segment is sorted
 * independently (Section 3's radix-2^8 count-sort rounds, or a network of
 * Section 2 in LDS).  The segments of 10,241 .. 14,336 keys (one tile of
 * those rounds, at least 71% full) and of 16,385 .. 2^30 - 1 keys are
 * sorted together by four device-wide radix-2^8 rounds over all their
 * tiles of 14,336 keys, each tile's prefix taken inside its own segment.
 * One persistent launch sorts the others, each by one workgroup: in its
 * LDS up to 16,384 keys (BTN/OET/LDS radix per the tuning table), by its
 * own radix-2^8 rounds from 2^30 keys.
 * algo: AUTO (tuned); BTN, OET or LDS_RADIX force the small-segment
 * algorithm; LSD keeps the tuned small-segment algorithm and sorts every
 * longer segment by one workgroup's rounds, never by the shared rounds
 * (the schedule of the paper's model, one processor per segment; its
 * workspace is smaller).  Invalid offsets (decreasing, negative, past
 * total_n, or overlapping segments) raise the range error in the status
 * word and leave the segments concerned unsorted; nothing outside `in`,
 * `out` and the workspace is touched.  `in == out` is allowed. */
rs_status rs_sort_segmented(const uint32_t* in, uint32_t* out, const int64_t* offsets,
                            size_t num_segments, int64_t total_n, rs_algo algo, void* ws,
                            size_t ws_bytes, void* stream);

/* The block networks at device scale (Section 2; Section 3, Eqs. Tb and
 * To): the n keys are cut into p runs of N = ceil(n/p) keys (the tail padded
 * with UINT32_MAX), every run is sorted by one workgroup, then BTN runs
 * Batcher's bitonic sorter on p wires, lg p (lg p + 1)/2 stages, or OET runs
 * p rounds of neighbour pairs (round t pairs runs i, i+1 with i = t mod 2),
 * each comparator a merge-split of two runs (the N smallest keys to one run,
 * ties taken from the lower-indexed run) and each stage one pass over all
 * keys in device memory.  The first n keys of the result are written to
 * `out`.  algo RS_ALGO_BTN (p a power of two) or RS_ALGO_OET; p in
 * [2, 4096] with p * N < 2^32, 0 = rs_blocks_default_p(n, algo).
 * Layout: dense arrays of n keys; `in == out` is allowed.  Workspace:
 * rs_workspace_bytes(RS_OP_BLOCKS, n, 4, 0, 0, algo, p) (two padded copies
 * of the keys).  rs_get_stats reports p and the stage count. */
rs_status rs_sort_blocks_u32(const uint32_t* in, uint32_t* out, size_t n, rs_algo algo, int p,
                             void* ws, size_t ws_bytes, void* stream);

/* The MBSP cost model that picks p for the block networks at device scale
 * (Section 3, Eqs. TbG and ToG, with a processor read as a workgroup).  For
 * n keys on p runs of N = ceil(n/p) keys, in nanoseconds:
 *   T(p) = local_ns_per_key * N * ceil(p / resident_runs)
 *        + stages(p) * (stage_ps_per_key * 1e-3 * p * N + stage_fixed_us * 1e3)
 * with stages(p) = lg p (lg p + 1)/2 (BTN) or p (OET).  local_ns_per_key is
 * the paper's 68 G, one workgroup's radix sort of its run; unlike the
 * paper's 4 (n/p) g, a merge-split stage runs on every compute unit, so it
 * costs per key of the whole array.  The defaults are one MI355X's
 * calibration (local 3.74 ns, stage 1.67 ps per key + 17.2 us, 512 resident
 * workgroups); `bench.py --workload blocks --mbsp` measures G and g. */
typedef struct {
    double local_ns_per_key;   /* > 0                                        */
    double stage_ps_per_key;   /* >= 0                                       */
    double stage_fixed_us;     /* >= 0                                       */
    int32_t resident_runs;     /* >= 1: runs sorted at once                  */
} rs_block_model;

/* Replaces the model (host, process-wide, not thread-safe against
 * concurrent sorts); RS_ERR_INVALID for NULL or values out of range. */
rs_status rs_blocks_set_model(const rs_block_model* m);

/* Copies the current model to `out` (host); RS_ERR_INVALID for NULL. */
rs_status rs_blocks_get_model(rs_block_model* out);

/* The p that p = 0 selects for n keys: the p minimising T(p) among
 * 2 <= p <= min(4096, n/64) (p = 2 when n < 128), powers of two only for
 * BTN, the smaller on a tie.  0 for n = 0 or an algo other than BTN/OET. */
int32_t rs_blocks_default_p(size_t n, rs_algo algo);

/* Bytes of workspace the call (op, n, ...) needs.  For RS_OP_BATCH, n is
 * the array length and num_segments the count; for RS_OP_SEGMENTED, n is
 * total_n; for RS_OP_BLOCKS, num_segments is p (0 = default).  Returns 0 for
 * arguments no call would accept. */
size_t rs_workspace_bytes(int op, size_t n, int key_bytes, int val_bytes, int radix_bits,
                          rs_algo algo, size_t num_segments);

/* Largest n one workgroup can sort in LDS for keys of key_bytes bytes. */
size_t rs_small_capacity(int key_bytes);

/* Static description of a status code. */
const char* rs_status_string(rs_status s);

/* Copies the calling thread's stats of its most recent call.  If that call
 * enqueued device work whose outcome the stats report (device_error, the
 * learned path's overflow counts), this synchronises that call's stream and
 * reads them from that call's workspace, which must therefore still be
 * allocated and not reused by other work. */
rs_status rs_get_stats(rs_stats* out);

/* ---- sorting without allocation ------------------------------------------ */

#define RS_NOALLOC_SCRATCH_BYTES (40u << 20) /* static scratch per device        */
#define RS_NOALLOC_MAX_KEYS (1u << 22)       /* largest n of rs_sort_u32_noalloc */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as rs_sort_u32 with algo LSD or AUTO, taking no workspace.  Its
 * scratch is a static device array of RS_NOALLOC_SCRATCH_BYTES inside the
 * library, one copy on every device the library runs on, held until the
 * process ends; the call makes no hipMalloc, hipFree or other allocating
 * call (and records no kernel timing events).
 *   in, out     DEVICE arrays of n uint32 keys (in == out: in place);
 *   n           <= RS_NOALLOC_MAX_KEYS (4,194,304), else RS_ERR_UNSUPPORTED;
 *   radix_bits  0 (= 8) or 1..11; 12..16 return RS_ERR_UNSUPPORTED;
 *   algo        RS_ALGO_LSD or RS_ALGO_AUTO, else RS_ERR_UNSUPPORTED;
 *   stream      a hipStream_t of the CURRENT device (NULL: the default
 *               stream), else RS_ERR_INVALID; the current device's scratch
 *               is used.
 * Every call on one device shares that device's scratch, which keeps the
 * last call's contents (each call clears what must start at zero itself):
 * calls that may overlap on one device -- on different streams, or from
 * different host threads -- race, and the caller must order them.
 * Argument errors return before anything is enqueued, as for rs_sort_u32;
 * rs_get_stats reports the call. */
rs_status rs_sort_u32_noalloc(const uint32_t* in, uint32_t* out, size_t n, int radix_bits,
                              rs_algo algo, void* stream);

/* ---- tuning table --------------------------------------------------------- */

/* The tuned choices for length class size_log2 = k (arrays of length in
 * (2^(k-1), 2^k], k = 0..32):
 *   algo, p         k <= 14 only (0 above): the small-array algorithm,
 *                   RS_ALGO_BTN, RS_ALGO_OET or RS_ALGO_LDS_RADIX, and p the
 *                   runs of BTN/OET.  Used by RS_ALGO_AUTO for small single
 *                   arrays and batches, and for the small segments of
 *                   rs_sort_segmented;
 *   radix_bits      the radix of LSD sorts of single uint32 arrays (keys
 *                   only) of the class called with radix_bits = 0 (0: 8);
 *   tile_items      keys per thread of the tiles of uint32 keys-only LSD
 *                   rounds at radix <= 2^8: 8, 16 or 28 (0: by size, 16
 *                   below 2^23 keys);
 *   seg_tile_items  keys per thread of the tiles with which one workgroup
 *                   sorts a segment of the class longer than its LDS
 *                   capacity (RS_ALGO_LSD segments, the block networks'
 *                   runs, segments of 2^30 keys and more): 8 or 16 (0: 16).
 * The choices change the workspace a call needs: rs_workspace_bytes reads
 * the same table, so size the workspace after the table is set. */
typedef struct {
    int32_t size_log2;
    int32_t algo;
    int32_t p;
    int32_t radix_bits;
    int32_t tile_items;
    int32_t seg_tile_items;
} rs_tune_entry;

/* Replaces the entries for the classes listed (process-wide, not
 * thread-safe against concurrent sorts).  RS_ERR_INVALID for a bad class,
 * algorithm, p (a power of two with 2^k / p <= 64), radix (0..16) or tile. */
rs_status rs_tune_set(const rs_tune_entry* entries, int count);

/* Copies the current table (classes 0..32) to `out` (host); returns the
 * number of entries written. */
int rs_tune_get(rs_tune_entry* out, int max);

/* Writes the current table to the file `path` as JSON, keyed by the current
 * device's gfx architecture name and compute unit count:
 *   {"format": "rs-tuning-1", "arch": "...", "cus": N,
 *    "classes": [{"size_log2": k, "algo": a, "p": p, "radix_bits": b,
 *                 "tile_items": t, "seg_tile_items": s}, ...]}
 * RS_ERR_INVALID if the file cannot be written, RS_ERR_HIP without a device. */
rs_status rs_tune_save(const char* path);

/* Replaces the table with the one in `path` (as rs_tune_save writes it).
 * RS_ERR_INVALID for a file that cannot be read or parsed or holds a bad
 * entry; RS_ERR_UNSUPPORTED when it was written for another architecture or
 * compute unit count; RS_ERR_HIP without a device.  The table is unchanged
 * unless RS_OK.  The environment variable RS_TUNING_FILE names a file loaded
 * the same way when the table is first used (silently skipped when it does
 * not load). */
rs_status rs_tune_load(const char* path);

/* One timing of the autotuner. */
typedef struct {
    int32_t size_log2;      /* arrays (or segments) of 2^size_log2 keys         */
    int32_t algo;           /* RS_ALGO_BTN / _OET / _LDS_RADIX: one workgroup   */
                            /* per array; RS_ALGO_LSD: the device-wide radix    */
                            /* sort of one array; RS_ALGO_AUTO: the segmented   */
                            /* sort of segments of that length                  */
    int32_t p;              /* runs of BTN/OET                                   */
    int32_t radix_bits;     /* LSD: radix bits                                   */
    int32_t tile_items;     /* LSD: keys per thread of its tiles (0: by size)    */
    int32_t seg_tile_items; /* segmented: keys per thread of a large segment's   */
                            /* tiles                                             */
    int32_t chosen;         /* 1 if installed in the tuning table                */
    double us_per_array;    /* per array (segment), `instances` in one launch;  */
                            /* LSD: one array per call                           */
    double us_single;       /* one array alone: launch latency included          */
    double us_model;        /* rs_tune_run_model: the cost model's prediction   */
                            /* per array (NaN where not modelled; 0 from        */
                            /* rs_tune_run); us_per_array is NaN for a          */
                            /* candidate it predicted but did not time          */
} rs_tune_result;

/* Autotuner, on the current device:
 *   - every class k = 1..14: BTN and OET at every valid p and the LDS radix
 *     sort on `instances` arrays of 2^k keys in one launch (and one array
 *     alone); the fastest is installed; the device-wide LSD sort of one
 *     array is timed beside them (the small-n crossover);
 *   - every class k = 15 .. min(24, lg(instances * 16384)): the LSD sort of
 *     one array of 2^k uint32 keys at radix 2^8 with 8-, 16- and 28-key
 *     tiles and at radix 2^11; the fastest is installed as the class's radix and
 *     tile if it beats the default (radix 2^8, 16-key tiles below 2^23
 *     keys, 28 above) by at least 3%, else the default;
 *   - every class k = 15 .. 20 with at least 512 segments of 2^k keys in
 *     instances * 16384 keys: those segments sorted one workgroup each (as
 *     RS_ALGO_LSD sorts them) with 8- and 16-key-per-thread tiles; 8 is
 *     installed if at least 3% faster, else 16 (classes with fewer segments
 *     keep their entry).  The shared device-wide rounds, which sort such
 *     segments under RS_ALGO_AUTO, have no tile choice.
 * Each candidate is timed twice, interleaved with the others, and keeps its
 * faster time.
 * Writes at most `max` results to `out` (host) and returns how many, or
 * minus an rs_status.  Synchronises `stream`.  The workspace (device, at
 * least rs_workspace_bytes(RS_OP_TUNE, instances, ...)) holds the inputs. */
int rs_tune_run(void* ws, size_t ws_bytes, int instances, void* stream, rs_tune_result* out,
                int max);

/* The same tuning with the small classes (k = 1..14) guided by a cost model
 * of the form of the paper's T_b and T_o (Section 3; Section 4, Eqs. for
 * BTN and OET with p processors): per array,
 *   t(p) = c0 npad lg N (lg N + 1) / 4 + c1 S npad (lg N + 1) + c2 S p + c3,
 * N = npad / p keys per processor, S = lg p (lg p + 1) / 2 merge-split
 * stages for BTN and p rounds for OET.  The three constants are fitted per
 * network (c3: a share of the launch), by least squares on relative error,
 * to timings of the smallest,
 * middle and largest valid p in classes 4, 7, 10 and 13; then each class
 * times only the p the model predicts fastest and its two neighbours for
 * each network, and the LDS radix sort, and installs the fastest timed.
 * Candidates predicted but not timed are reported with us_per_array = NaN
 * and their prediction in us_model.  The larger classes are tuned as by
 * rs_tune_run.  Same arguments, workspace and return value. */
int rs_tune_run_model(void* ws, size_t ws_bytes, int instances, void* stream, rs_tune_result* out,
                      int max);

/* ---- kernel timing (benchmarks) ---------------------------------------- */

typedef struct {
    char name[32];     /* kernel name                                          */
    int64_t launches;  /* launches recorded since the last read                */
    double total_ms;   /* summed duration between the bracketing HIP events    */
} rs_kernel_time;

/* Copies `bytes` bytes of device memory from `in` to `out` (not
 * overlapping) with a plain streaming kernel, 16-byte words when both are
 * 16-byte aligned: the read + write bandwidth ceiling the sorts are measured
 * against (timed as "stream_copy").  RS_ERR_INVALID for NULL or
 * overlapping buffers. */
rs_status rs_stream_copy(const void* in, void* out, size_t bytes, void* stream);

/* on = 1: from now on every kernel launch of this library is bracketed by a
 * pair of HIP events recorded on the launch's own stream (process-wide).
 * on = 0 stops recording.  Recording adds two event records per launch. */
rs_status rs_profile_enable(int on);

/* Waits for every recorded event, writes at most `max` per-kernel totals to
 * `out` (host array) and clears the record.  Returns the number of entries
 * written, or -1 on a HIP error. */
int rs_profile_read(rs_kernel_time* out, int max);

#ifdef __cplusplus
}
#endif
#endif
