// rs_internal.hpp -- host-side plans and launchers shared by the librs
// translation units.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rs.h"

namespace rs {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Bounded waits: a look-back that polls this many times without progress
// records an error in the workspace status word and gives up, so every
// kernel always terminates.
constexpr uint32_t SPIN_LIMIT = 1u << 20;
constexpr uint32_t STATUS_SPIN = 1u;   // a bounded wait gave up
constexpr uint32_t STATUS_RANGE = 2u;  // a computed destination was out of range (not written)

// ---- kernel timing: every launch site brackets its launch with
//      prof(st, id, 0) ... prof(st, id, 1); a no-op unless enabled.
enum KernelId {
    KID_FILL = 0,
    KID_HIST,
    KID_ONESWEEP,
    KID_COPY,
    KID_BATCH,
    KID_SEG_PLAN,
    KID_SEG,
    KID_LEARN_SAMPLE,
    KID_LEARN_TRAIN,
    KID_LEARN_SPLIT,
    KID_LEARN_ASSIGN,
    KID_LEARN_BUCKET,
    KID_LEARN_CHECK,
    KID_WIDE_COUNT,
    KID_WIDE_SCATTER,
    KID_LEARN_PASS,
    KID_LEARN_MID,
    KID_BLOCK_MERGE,
    KID_STREAM_COPY,
    KID_SEG_ROUND,
    KID_COUNT_
};
extern bool g_prof_on;
// set on the calling thread while an entry point that must not create HIP
// events (the no-allocation sort) runs
extern thread_local bool g_prof_muted;
void prof_record(hipStream_t st, int kid, int phase);
inline void prof(hipStream_t st, int kid, int phase) {
    if (g_prof_on && !g_prof_muted) prof_record(st, kid, phase);
}

// ---- LSD radix sort (count-sort rounds, Section 3) -----------------------
// Tile order across XCDs (see LsdPlan::nx): consecutive tiles per XCD, and
// the per-round counters (one per XCD) kept CTR_STRIDE words apart.
constexpr uint32_t XCD_CHUNK = 16;
constexpr uint32_t CTR_STRIDE = 8;
// The XCD count the tile order uses on the current device (0: one counter).
uint32_t xcd_order_count();
struct LsdPlan {
    size_t n = 0;
    int kb = 4, vb = 0;      // key / value bytes (kb = 2: 16-bit digit keys)
    int vb2 = 0;             // bytes of a second payload (16-bit keys only)
    int bits = 8;            // radix bits b
    int passes = 0;          // ceil(8*kb / b)
    int R = 256;             // 2^b
    int tile = 0;            // keys per workgroup tile
    size_t tiles = 0;
    // Tile order across XCDs: nx = 0, tiles in the order workgroups arrive
    // at one counter; nx > 0, chunks of XCD_CHUNK consecutive tiles per XCD
    // (chunk k on XCD k mod nx), each XCD's workgroups taking its chunks'
    // tiles in order from a counter of its own.  grid: workgroups launched
    // (tiles, or nx > 0: padded to whole rounds of nx chunks).
    uint32_t nx = 0;
    size_t grid = 0;
    bool lb64 = false;       // 64-bit look-back words (n >= 2^30)
    size_t lb_words = 0;     // look-back words per pass (tiles * R)
    // workspace layout (byte offsets)
    size_t off_status = 0, off_ctr = 0, off_hist = 0, off_lb = 0, off_tk = 0, off_tv = 0, off_tv2 = 0;
    size_t zero_bytes = 0;   // bytes from off_status that must be zeroed (status, ctr, hist)
    size_t total = 0;
    int kid_hist = KID_HIST;          // timing labels of the plan's launches
    int kid_scatter = KID_ONESWEEP;
    bool skip = false;       // skip the rounds whose digit is the same for every key
};
// Byte offset, inside the status block, of the route of a sort that skips
// rounds (its first word: the mask of skipped rounds).
constexpr size_t ROUTE_OFFSET = 16;

// Largest key count + 1 of the LSD rounds: digit counts and prefixes are
// 32-bit words.
constexpr uint64_t LSD_MAX_N = 1ull << 32;

// Plans an LSD sort; returns false when (kb, vb, bits, vb2) is not supported
// or n >= LSD_MAX_N.  items: keys per thread of the tiles, 0 = by size; 8, 16
// or 28 for uint32 keys without values at radix <= 2^8 (other shapes: 0 only).
bool lsd_plan(size_t n, int kb, int vb, int bits, LsdPlan* p, int vb2 = 0, int items = 0);

// Radix bits and tile items of an LSD sort of n keys asked for with
// radix_bits (0: the tuned radix of n's length class for uint32 keys without
// values, else 8), from the tuning table (items 0: by size).
void lsd_tuned(size_t n, int kb, int vb, int radix_bits, int* bits, int* items);

// Enqueues the whole LSD sort on `st`.  `ws` holds at least p.total bytes.
rs_status lsd_run(const LsdPlan& p, const void* kin, void* kout, const void* vin, void* vout,
                  void* ws, hipStream_t st, const void* vin2 = nullptr, void* vout2 = nullptr);

// ---- wide-digit count-sort rounds (b = 12..16, reduce-then-scan) ----------
struct WidePlan {
    size_t n = 0;
    int kb = 4, vb = 0;
    int bits = 16;
    int passes = 0;           // ceil(8*kb / b)
    uint32_t R = 0;           // 2^b
    uint64_t tile_keys = 0;   // keys per tile (whole 4096-key sub-tiles)
    uint32_t tiles = 0;
    size_t off_status = 0, off_table = 0, off_base = 0, off_tk = 0, off_tv = 0;
    size_t total = 0;
};
// Plans a wide-digit sort; false unless 12 <= bits <= 16 and n < 2^32.
bool wide_plan(size_t n, int kb, int vb, int bits, WidePlan* p);
rs_status wide_run(const WidePlan& p, const void* kin, void* kout, const void* vin, void* vout, void* ws,
                   hipStream_t st);

// Records the HIP error of a failed launch or runtime call for rs_get_stats
// and returns RS_ERR_HIP.
rs_status hip_fail(hipError_t e);
// hipGetLastError after a launch, mapped to a status.
inline rs_status launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RS_OK : hip_fail(e);
}

// ---- one workgroup per small array (BTN, OET, LDS radix) -----------------
constexpr uint32_t SMALL_CAP_U32 = 16384;          // keys one workgroup holds
uint32_t small_npad(uint32_t n);                   // next power of two >= n
bool small_valid_p(uint32_t n, int p);             // p a power of two, n_pad/p <= 64
int small_default_p(int algo, uint32_t n);
// `count` arrays of n keys back to back, one workgroup each.
rs_status small_run(int algo, const uint32_t* in, uint32_t* out, uint32_t n, size_t count, int p,
                    hipStream_t st);

// ---- segmented sort ---------------------------------------------------------
constexpr uint32_t SEG_SMALL_MAX = 16384;        // longest segment sorted in LDS
// Tuned choices per length class c (length in (2^(c-1), 2^c]).
struct SegTable {
    int8_t algo[64];      // small arrays: RS_ALGO_BTN, RS_ALGO_OET or RS_ALGO_LDS_RADIX
    int16_t p[64];        // runs for BTN/OET
    int8_t radix[64];     // single uint32 arrays, radix_bits = 0: LSD radix bits (0: 8)
    int8_t items[64];     // their radix-2^8 tiles: keys per thread (0: by size)
    int8_t seg_items[64]; // large segments: keys per thread of a tile, 8 or 16 (0: 16)
};
constexpr int TUNE_CLASSES = 33;  // classes 0 .. 32 in rs_tune_get / rs_tune_set
// Segments that fill their tiles well are sorted by onesweep rounds whose
// tiles every workgroup takes from one counter per round (the device-wide
// round's kernel, with the look-back inside each segment): every segment
// too long for one workgroup's LDS, up to SEG_OS_MAX - 1 keys, and those
// that fill one tile at least 71% (SEG_OS_MIN .. SEG_OS_TILE keys; a tile
// costs about the same whatever it holds, and below that fill, or with a
// second tile at most 2,048 keys long, one workgroup's LDS sort is faster).
// The others are sorted by one workgroup each.
constexpr uint64_t SEG_OS_MIN = 10241;
constexpr uint64_t SEG_OS_MAX = 1ull << 30;
constexpr uint64_t SEG_OS_TILE = 512 * 28;  // keys per tile of those rounds
constexpr bool seg_shared_len(uint64_t L) {
    return (L >= SEG_OS_MIN && L <= SEG_OS_TILE) || (L > SEG_SMALL_MAX && L < SEG_OS_MAX);
}
static_assert(SEG_OS_MIN <= SEG_OS_TILE && SEG_OS_TILE <= SEG_SMALL_MAX, "one tile, then the LDS capacity");
static_assert(!seg_shared_len(10240) && seg_shared_len(10241) && seg_shared_len(14336) && !seg_shared_len(14337) &&
                  !seg_shared_len(16384) && seg_shared_len(16385) && seg_shared_len((1ull << 30) - 1) &&
                  !seg_shared_len(1ull << 30),
              "the lengths the shared rounds take");
struct SegTile {          // one tile of the large segments' rounds (32 bytes)
    int64_t lo;           // first position of its segment
    int64_t len;          // keys of its segment (0: no tile, the workgroup leaves)
    uint32_t tl;          // tile within the segment
    uint32_t rank;        // the segment among the large ones (its histograms)
    uint32_t bb;          // look-back block of the segment's first tile
    uint32_t pad;
};
struct SegOs {
    const SegTile* td = nullptr;         // per tile of the round's numbering (max_tiles)
    const uint32_t* used = nullptr;      // tiles in use (the surplus workgroups leave at once)
    uint32_t max_tiles = 0;              // tiles the look-back words are laid out for (the block sums follow)
    const uint32_t* hist = nullptr;      // per large segment: 4 rounds x 256 digit counts
};
struct SegPlan {
    size_t off_status = 0, off_cnt = 0, off_order = 0, off_tmp = 0;
    // onesweep rounds of the large segments: tile map, per-segment
    // histograms, round counters, look-back words (4 rounds x max_tiles x 256)
    size_t off_ttile = 0, off_lrank = 0, off_tdesc = 0, off_shist = 0, off_osctr = 0, off_oslb = 0;
    uint64_t max_tiles = 0;   // bound on the tiles of the large segments (grid of a round)
    uint64_t max_blocks = 0;  // bound on their look-back blocks of 16 tiles
    uint64_t max_large = 0;   // bound on their number (histograms held)
    size_t off_bbase = 0;
    size_t zero_bytes = 0, total = 0;
    bool shared = true;       // segments of the lengths seg_shared_len takes share device-wide rounds
};
// shared = false: every segment is sorted by one workgroup (the tables of
// the shared rounds are not allocated)
bool seg_plan(uint64_t S, int64_t total, SegPlan* p, bool shared = true);
rs_status seg_run(const SegPlan& p, const uint32_t* in, uint32_t* out, const int64_t* offsets,
                  uint64_t S, int64_t total, const SegTable& table, void* ws, hipStream_t st);

// the four onesweep rounds of the segments seg_shared_len takes (in -> tmp
// -> out -> tmp -> out), after their plan kernels
rs_status segos_run(const SegPlan& p, const uint32_t* in, uint32_t* out, uint32_t* tmp, const int64_t* off,
                    uint64_t S, int64_t total, unsigned char* ws, hipStream_t st);

size_t tune_ws_bytes(int instances);

// ---- BTN / OET at device scale: p runs in HBM, merge-split stages -----------
struct BlockPlan {
    uint32_t p = 0;     // runs
    uint64_t N = 0;     // keys per run (the tail padded with the largest key)
    uint32_t nch = 0;   // merge chunks per pair
    SegPlan seg;        // the runs' local sorts
    size_t off_seg = 0, off_off = 0, off_x = 0, off_y = 0, off_cr = 0, total = 0;
};
// p for p = 0: the minimum of the MBSP cost model over the valid p
uint32_t block_default_p(size_t n, int algo);
const rs_block_model& block_model();
void block_model_set(const rs_block_model& m);
double block_model_ns(const rs_block_model& m, size_t n, int algo, uint32_t p);
bool block_plan(size_t n, int algo, uint32_t p, BlockPlan* bp);
int64_t block_stages(int algo, uint32_t p);
rs_status block_run(const BlockPlan& bp, int algo, const uint32_t* in, uint32_t* out, size_t n,
                    const SegTable& table, void* ws, hipStream_t st);

// The process-wide tuning table (defaults until rs_tune_set / rs_tune_run).
SegTable& tune_table();

// ---- learned-CDF buckets -------------------------------------------------------
struct LearnOpts {
    int32_t train_steps;          // Adam steps
    float lr;                     // Adam learning rate
    int32_t use_network;          // 0: bucket by the feature alone (no network)
    int32_t bucket_cap;           // LDS capacity of a bucket (<= 6144 pairs)
    int32_t feature_mode;         // -1 automatic (2), 0 linear, 1 log-scaled, 2 sample quantiles
    double fallback_frac;         // overflowed-key share that sends the whole array to LSD
    int32_t train_blocks;         // workgroups of the training launch
    int32_t max_fallback_buckets; // more overflowed buckets than this: whole-array LSD
};
struct LearnReport {
    int32_t fallback;
    int64_t buckets_overflowed, keys_overflowed;
    double train_loss;
    uint32_t device_error, unsorted;
    int32_t feature_mode;
    // device word holding the path's own errors and every inner LSD sort's
    // status word, complete once the stream reaches the end of the call
    const uint32_t* err_word;
};
LearnOpts& learn_opts();
size_t learned_ws_bytes(size_t n, int vb);
// Synchronises `st` (it reads the overflow counts back).
rs_status learned_run(const void* kin, void* kout, const void* vin, void* vout, size_t n, int vb, void* ws,
                      size_t ws_bytes, hipStream_t st, LearnReport* rep);
rs_status mlp_forward(const float* params, const float* x, float* y, size_t m, hipStream_t st);
rs_status mlp_adam_step(float* params, float* m1, float* m2, const float* grad, int step, float lr,
                        float beta1, float beta2, float eps, hipStream_t st);
// Test hooks of the learned path: parameters used instead of training
// (NULL: back to training); a planted fault (RS_LEARNED_FAULT_*).
rs_status learned_inject_weights(const float* params, size_t count);
rs_status learned_inject_fault(int kind, const uint64_t* spl, size_t count);
rs_status learned_debug_ids(uint16_t* direct, uint16_t* assigned);
rs_status mlp_loss_grad(const float* params, const float* x, const float* t, size_t m, float* grad,
                        hipStream_t st);
constexpr int MLP_NPARAM = 1153;

// Device-to-device copy by a streaming kernel (16-byte words when both
// pointers are 16-byte aligned).
rs_status stream_copy(const void* in, void* out, size_t bytes, hipStream_t st);

// Zero-fill of device memory by a kernel (no hipMemsetAsync, so callers may
// capture the stream into a graph).
rs_status fill_u32(void* p, size_t words, uint32_t v, hipStream_t st);

}  // namespace rs
