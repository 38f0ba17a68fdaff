// rs_lsd.hip -- the count-sort rounds of LSD radix sort on gfx950.
//
// Section 3 of the paper prices one count-sort round as a first read of the
// keys to count digits, a prefix over the count array, and a second read plus
// a write that places every key in input order (3Ng + 2NG), and the parallel
// form adds the exchange of the p count arrays (2prg).  On one MI355X the
// rounds are organised as:
//
//   k_fill      zero the status word, tile counters and global histograms;
//   k_hist      ONE read of the keys that counts the digits of every round at
//               once (the global digit histogram does not depend on the order
//               of the keys, so all rounds' counts come from the input) and
//               zeroes the look-back words;
//   k_onesweep  one launch per round: each workgroup takes the next tile id,
//               ranks its keys stably by digit (an LDS match per group of
//               16 lanes, the group's running count beside its mask; whole
//               waves with ballots above 8 bits), publishes its per-digit
//               counts, reorders the tile by digit in LDS, looks back over
//               earlier tiles for their exclusive prefix (decoupled
//               look-back, Merrill and Garland 2016, with flag and count
//               packed in one word) and writes each digit's run to HBM
//               contiguously.
//
// The paper's count exchange (2prg) is the look-back table: R words per
// tile.  Per round HBM traffic is one read and one write of the keys (and
// values); the histogram read is paid once for all rounds.
#include <atomic>
#include <cstdlib>
#include <type_traits>

#include "rs_dev.h"
#include "rs_internal.hpp"

namespace rs {
namespace {

constexpr int NT = 512;          // threads per onesweep workgroup
constexpr int NW = NT / WAVE;    // waves per workgroup
constexpr int HIST_NT = 256;
constexpr uint32_t HIST_HOT = 8;  // lanes on lane 0's digit worth one aggregated add
constexpr uint32_t FLAG_AGG = 1, FLAG_PRE = 2;
constexpr int LBWIN = 4;         // predecessors read per look-back step
constexpr int LBB = 16;          // tiles per look-back block
constexpr int LBWIN_B = 4;       // blocks read per look-back step
constexpr int BW_SH = 26;        // block word: tiles counted above bit 26, their digit count below
static_assert(LBB < (1 << (32 - BW_SH)) && (size_t)LBB * 65536 < (1u << BW_SH),
              "a block word holds the tile count and the block's digit count");
constexpr int RANK_GL = 16;      // lanes per ranking group at radix <= 2^8 (16 or 32)

template <typename LB> struct LBW;
template <> struct LBW<uint32_t> {
    static constexpr int SH = 30;
    static constexpr uint32_t MASK = (1u << 30) - 1;
};
template <> struct LBW<uint64_t> {
    static constexpr int SH = 62;
    static constexpr uint64_t MASK = (1ull << 62) - 1;
};

// keys per thread of a onesweep tile, by key and value bytes and the digit
// width the LDS arrays are sized for (measured at 2^28 keys; radix 2^11
// tiles stay smaller so that two workgroups still share a compute unit)
constexpr int lsd_items(int kb, int vb, int maxb) {
    if (maxb > 8) return kb == 4 ? (vb == 0 ? 24 : 16) : 8;
    if (kb == 4) return vb == 0 ? 28 : (vb == 4 ? 22 : 16);
    return vb == 0 ? 18 : (vb == 8 ? 12 : 8);
}
// below this many uint32 keys (keys only) the radix-2^8 rounds take smaller
// tiles, so that the tiles still outnumber the workgroups the chip holds at
// once (measured: at 2^20 keys 0.120 ms per sort against 0.142)
constexpr size_t LSD_SMALL_N = size_t(1) << 23;
constexpr int LSD_ITEMS_SMALL = 16;
constexpr int LSD_ITEMS_TINY = 8;  // a tuning choice for small arrays: twice the tiles
// 16-bit digit keys carry up to two 8-byte payloads (the learned path moves
// bucket ids with their keys and values)

template <int VB> struct ValT { using type = uint32_t; };
template <> struct ValT<8> { using type = uint64_t; };

// Buffers of a sort that skips the rounds whose digit is the same for every
// key (in the workspace's status block, written on the device once the
// histograms are known).
struct Route {
    uint32_t mask;              // bit j: round j is skipped
    uint32_t passes, inplace;
    uint32_t pad_;
    const void* in;
    void* out;
    void* tmp;
    const void* vin;
    void* vout;
    void* vtmp;
};
static_assert(ROUTE_OFFSET + sizeof(Route) <= ALIGN, "the route lives in the status block");

// One workgroup: the rounds whose global histogram has a single non-empty
// bin (a count of n) are the identity and are skipped; thread 0 writes the
// route the rounds follow.
__global__ void k_route(const uint32_t* __restrict__ ghist, int passes, int R, uint64_t n, Route* __restrict__ rt,
                        const void* in, void* out, void* tmp, const void* vin, void* vout, void* vtmp) {
    __shared__ uint32_t m;
    if (threadIdx.x == 0) m = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < passes * R; i += blockDim.x)
        if ((uint64_t)ghist[i] == n) atomicOr(&m, 1u << (i / R));
    __syncthreads();
    if (threadIdx.x == 0) {
        Route r;
        r.mask = m;
        r.passes = (uint32_t)passes;
        r.inplace = in == out;
        r.pad_ = 0;
        r.in = in;
        r.out = out;
        r.tmp = tmp;
        r.vin = vin;
        r.vout = vout;
        r.vtmp = vtmp;
        *rt = r;
    }
}

// After the rounds: the sorted keys (and values) are still in the input when
// no round ran, or in the workspace copy after an odd number of rounds of an
// in-place sort; then they are copied to `out`.
__global__ void k_route_copy(const Route* __restrict__ rt, uint64_t kwords, uint64_t vwords) {
    const uint32_t m = rt->mask;
    const int E = __popc(~m & (rt->passes >= 32 ? ~0u : (1u << rt->passes) - 1u));
    const uint32_t* ks;
    const uint32_t* vs;
    if (rt->inplace) {
        if (!(E & 1)) return;
        ks = static_cast<const uint32_t*>(rt->tmp);
        vs = static_cast<const uint32_t*>(rt->vtmp);
    } else {
        if (E != 0) return;
        ks = static_cast<const uint32_t*>(rt->in);
        vs = static_cast<const uint32_t*>(rt->vin);
    }
    uint32_t* kd = static_cast<uint32_t*>(rt->out);
    uint32_t* vd = static_cast<uint32_t*>(rt->vout);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kwords; i += stride) kd[i] = ks[i];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < vwords; i += stride) vd[i] = vs[i];
}

// Plain streaming copy of n16 16-byte words: one contiguous chunk of 1,024
// words (16 KiB) per workgroup, four loads in flight per thread (the read +
// write ceiling the sorts are compared with; contiguous chunks per
// workgroup measured faster than a grid-wide stride).
constexpr uint64_t COPY_CHUNK16 = 1024;
__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                    uint64_t n16) {
    const uint64_t b = (uint64_t)blockIdx.x * COPY_CHUNK16 + threadIdx.x;
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (b + q * 256 < n16) v[q] = in[b + q * 256];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (b + q * 256 < n16) out[b + q * 256] = v[q];
}

__global__ void k_copy_bytes(const unsigned char* __restrict__ in, unsigned char* __restrict__ out, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

__global__ void k_fill(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Digit histograms of every round in one read of the keys.  LDS holds
// passes * 2^bits counters; the zeroing of the look-back words (`zp`,
// `zwords` 32-bit words) rides along on the same grid.
template <typename K>
__global__ __launch_bounds__(HIST_NT) void k_hist(const K* __restrict__ keys, uint64_t n, int bits,
                                                   int passes, uint32_t* __restrict__ ghist,
                                                   uint32_t* __restrict__ zp, uint64_t zwords) {
    extern __shared__ uint32_t h[];
    const int R = 1 << bits;
    const uint32_t mask = (uint32_t)R - 1;
    const int tot = passes * R;
    for (int i = threadIdx.x; i < tot; i += HIST_NT) h[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * HIST_NT;
    uint64_t i = (uint64_t)blockIdx.x * HIST_NT + threadIdx.x;
    // Counting: the lanes whose digit equals lane 0's are added by one lane
    // when there are at least HIST_HOT of them (skewed keys put most of a
    // wave on one digit in the high rounds, and their atomics would
    // serialise on one counter); the other lanes add one by one.  The test
    // costs instructions, so a round that misses before it has hit in the
    // current 16-step window drops out of the test until the window ends.
    // The counts are exact either way.  (Wave-uniform masks, one bit per
    // round: up to 64 rounds.)
    const uint64_t all = passes >= 64 ? ~0ull : (1ull << passes) - 1;
    uint64_t test = all, hit = 0;
    auto count = [&](uint32_t slot, int p) {
        const uint64_t bit = 1ull << p;
        if (test & bit) {
            const uint32_t first = __builtin_amdgcn_readfirstlane(slot);
            const uint32_t c = (uint32_t)__popcll(ballot(slot == first));
            if (c >= HIST_HOT) {
                hit |= bit;
                if ((threadIdx.x & 63) == 0) atomicAdd(&h[first], c);
                if (slot != first) atomicAdd(&h[slot], 1u);
                return;
            }
            if (!(hit & bit)) test &= ~bit;
        }
        atomicAdd(&h[slot], 1u);
    };
    // four independent loads in flight per thread; whole waves only, so
    // lane 0 is active and the hot-digit test sees 64 keys
    const uint64_t nfull = n - n % ((uint64_t)HIST_NT * gridDim.x);
    for (uint32_t step = 1; i + 3 * stride < nfull; i += 4 * stride, ++step) {
        K k0 = keys[i], k1 = keys[i + stride], k2 = keys[i + 2 * stride], k3 = keys[i + 3 * stride];
        for (int p = 0; p < passes; ++p) {
            const int s = p * bits;
            count(p * R + ((uint32_t)(k0 >> s) & mask), p);
            count(p * R + ((uint32_t)(k1 >> s) & mask), p);
            count(p * R + ((uint32_t)(k2 >> s) & mask), p);
            count(p * R + ((uint32_t)(k3 >> s) & mask), p);
        }
        if ((step & 15) == 0) {
            test = all;
            hit = 0;
        }
    }
    for (; i < nfull; i += stride) {
        K k0 = keys[i];
        for (int p = 0; p < passes; ++p) count(p * R + ((uint32_t)(k0 >> (p * bits)) & mask), p);
    }
    for (; i < n; i += stride) {
        K k0 = keys[i];
        for (int p = 0; p < passes; ++p)
            atomicAdd(&h[p * R + ((uint32_t)(k0 >> (p * bits)) & mask)], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < tot; j += HIST_NT)
        if (h[j]) atomicAdd(&ghist[j], h[j]);
    const uint64_t gstride = (uint64_t)gridDim.x * HIST_NT;
    for (uint64_t j = (uint64_t)blockIdx.x * HIST_NT + threadIdx.x; j < zwords; j += gstride) zp[j] = 0u;
}

// The same histograms for the common shapes, with the digit arithmetic
// fixed at compile time and the LDS counters laid out by lane: counter word
// (pass, digit, column), column = lane mod COLS.  At radix 2^8 with 16
// columns the 32 lanes that one LDS cycle serves fall in at most two words
// per bank whatever the digits (skewed keys included); the columns are
// summed once at the end.  One key and pass costs a bit-field extract, one
// address operation and one LDS add; the LDS adds set the pace.
constexpr int HC_NT = 1024;
constexpr uint64_t HC_GRID = 1024;  // workgroups (fewer for small n)

template <typename K, int BITS, int PASSES, int COLS>
__global__ __launch_bounds__(HC_NT) __attribute__((amdgpu_waves_per_eu(8))) void k_hist_fixed(
    const K* __restrict__ keys, uint64_t n, uint32_t* __restrict__ ghist, uint32_t* __restrict__ zp,
    uint64_t zwords) {
    static_assert(COLS >= 1 && COLS <= 32 && (COLS & (COLS - 1)) == 0, "a power-of-two column count");
    constexpr int R = 1 << BITS;
    constexpr int ROWS = PASSES * R;
    extern __shared__ uint32_t h[];
    for (int i = threadIdx.x; i < ROWS * COLS; i += HC_NT) h[i] = 0;
    __syncthreads();
    const uint32_t col = threadIdx.x & (COLS - 1);
    auto count = [&](K key) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const uint32_t d = (uint32_t)(key >> (p * BITS)) & (uint32_t)(R - 1);
            atomicAdd(&h[(p * R + d) * COLS + col], 1u);
        }
    };
    // 16-byte loads over the aligned body, four in flight per thread; the
    // keys before the first 16-byte boundary and after the last whole
    // vector are counted one per thread by workgroup 0
    constexpr int VK = 16 / sizeof(K);
    const uint64_t mis = (reinterpret_cast<uintptr_t>(keys) & 15) / sizeof(K);
    uint64_t head = mis ? VK - mis : 0;
    if (head > n) head = n;
    const uint64_t nv = (n - head) / VK;
    const uint64_t tail0 = head + nv * VK;
    const uint4* __restrict__ kv = reinterpret_cast<const uint4*>(keys + head);
    auto count_vec = [&](const uint4 v) {
        if constexpr (sizeof(K) == 8) {
            count((K)(((uint64_t)v.y << 32) | v.x));
            count((K)(((uint64_t)v.w << 32) | v.z));
        } else {
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (sizeof(K) == 4) {
                    count((K)w[j]);
                } else {
                    count((K)(w[j] & 0xffffu));
                    count((K)(w[j] >> 16));
                }
            }
        }
    };
    const uint64_t stride = (uint64_t)gridDim.x * HC_NT;
    uint64_t i = (uint64_t)blockIdx.x * HC_NT + threadIdx.x;
    for (; i + 3 * stride < nv; i += 4 * stride) {
        const uint4 v0 = kv[i], v1 = kv[i + stride], v2 = kv[i + 2 * stride], v3 = kv[i + 3 * stride];
        count_vec(v0); count_vec(v1); count_vec(v2); count_vec(v3);
    }
    for (; i < nv; i += stride) count_vec(kv[i]);
    if (blockIdx.x == 0) {
        if (threadIdx.x < head) count(keys[threadIdx.x]);
        if (tail0 + threadIdx.x < n) count(keys[tail0 + threadIdx.x]);
    }
    __syncthreads();
    // sum the columns of each row, each lane starting at its own column so
    // that a wave's reads spread over the banks
    for (int r = threadIdx.x; r < ROWS; r += HC_NT) {
        uint32_t c_sum = 0;
#pragma unroll
        for (int c = 0; c < COLS; ++c) c_sum += h[r * COLS + ((c + r) & (COLS - 1))];
        if (c_sum) atomicAdd(&ghist[r], c_sum);
    }
    const uint64_t gstride = (uint64_t)gridDim.x * HC_NT;
    for (uint64_t j = (uint64_t)blockIdx.x * HC_NT + threadIdx.x; j < zwords; j += gstride) zp[j] = 0u;
}

// launch k_hist_fixed<K, BITS, PASSES, COLS> over n keys
template <typename K, int BITS, int PASSES, int COLS>
void launch_hist_fixed(const void* kin, uint64_t n, uint32_t* gh, uint32_t* zp, uint64_t zwords,
                       hipStream_t st) {
    const size_t shm = sizeof(uint32_t) * (size_t)PASSES * (1u << BITS) * COLS;
    static_assert(sizeof(uint32_t) * (size_t)PASSES * (1u << BITS) * COLS <= 65536, "LDS per workgroup");
    uint64_t g = (n + HC_NT * 16 - 1) / (HC_NT * 16);
    if (g > HC_GRID) g = HC_GRID;
    const uint64_t gz = (zwords + HC_NT * 16 - 1) / (HC_NT * 16);
    if (g < gz) g = gz;
    if (g < 1) g = 1;
    hipLaunchKernelGGL((k_hist_fixed<K, BITS, PASSES, COLS>), dim3((unsigned)g), dim3(HC_NT), shm, st,
                       static_cast<const K*>(kin), n, gh, zp, zwords);
}

// One stable count-sort round over tiles of NT*ITEMS keys.
//   MAXB  : largest radix bits the LDS arrays are sized for (bits <= MAXB)
//   VB    : value bytes (0 = keys only)
//   VB2   : bytes of a second payload array (0 = none)
//   LB    : look-back word type (32-bit while n < 2^30)
//   OFF   : int32_t destinations while n < 2^31, else int64_t
//
// Ranking.  Keys are visited in input order within ranking groups of GL
// lanes: item i of lane l of group g is tile position g*GL*ITEMS + i*GL + l.
// For each item the lanes holding the same digit are found with an LDS
// match: every lane ORs its lane bit into its group's slot for the digit,
// then reads the slot back; OR is order-independent, so the mask is exact
// and the ranking stable whatever order the LDS serves the atomics in.  A
// key's rank among equal digits of its group is the group's running count
// for the digit plus the number of peer lanes below it; the highest peer
// lane stores the advanced count and a cleared mask.
//   radix <= 2^8: groups of RANK_GL = 16 lanes; a slot is one 32-bit word,
//     mask in the low half and running count in the high half, so each item
//     costs one OR, one read and one store of 4 bytes per lane.
//   radix 2^9..2^11: whole waves; 64-bit masks for the low 8 digit bits,
//     the bits above matched with one ballot each, and 16-bit counters per
//     wave and digit.
// Radix-2^8 rounds are held to 128 registers, so that two workgroups share
// a compute unit (at the tile sizes above a few spilled registers cost less
// than half the occupancy); radix-2^11 tiles are held to two workgroups by
// their LDS anyway.
template <typename K, int VB, int MAXB, int ITEMS, typename LB, typename OFF, int VB2 = 0, bool SEG = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MAXB <= 8 ? 4 : 1))) void k_onesweep(
    const K* __restrict__ kin0, K* __restrict__ kout0, const void* __restrict__ vin0,
    void* __restrict__ vout0, uint64_t n, int shift, int bits, uint32_t* __restrict__ tile_ctr,
    LB* __restrict__ lb, const uint32_t* __restrict__ ghist, uint32_t* __restrict__ status,
    const Route* __restrict__ route, const void* __restrict__ vin2_ = nullptr,
    void* __restrict__ vout2_ = nullptr, SegOs sg = SegOs{}, uint32_t nx = 0) {
    using V = typename ValT<VB>::type;
    constexpr int RMAX = 1 << MAXB;
    constexpr int RLO = RMAX < 256 ? RMAX : 256;      // slots of the LDS match
    constexpr int T = NT * ITEMS;
    constexpr int PER = (RMAX + NT - 1) / NT;  // digits per thread in the digit scans
    // Radix <= 2^8: keys are ranked in groups of RANK_GL lanes, and a
    // digit's slot holds the group's match mask in its low half and the
    // group's running count of the digit in its high half (a 32-bit slot for
    // 16-lane groups).  Wider radices rank whole waves, with 16-bit counters
    // beside the 64-lane masks.
    constexpr bool HALF = MAXB <= 8;
    constexpr int GL = HALF ? RANK_GL : WAVE;  // lanes per ranking group
    constexpr int NG = NT / GL;                // ranking groups per workgroup
    using Slot = typename std::conditional<(HALF && GL <= 16), uint32_t, uint64_t>::type;
    constexpr int CSH = (int)sizeof(Slot) * 4;  // count field of a slot
    constexpr size_t KEYB = (size_t)T * sizeof(K);
    constexpr size_t VALB = (size_t)T * (VB > VB2 ? VB : VB2);
    constexpr size_t CNTB = HALF ? 0 : (size_t)NW * RMAX * sizeof(uint16_t);
    constexpr size_t MSKB = (size_t)NG * RLO * sizeof(Slot);
    constexpr size_t RANKB = CNTB + MSKB;
    // values get an LDS buffer of their own (and are placed before the
    // look-back) when keys and values fit in 64 KiB together; otherwise
    // they reuse the key buffer after the keys are written
    constexpr bool SEPV = VB != 0 && VB2 == 0 && MAXB <= 8 && KEYB + VALB <= 65536;
    constexpr size_t UB1 = (KEYB > VALB || SEPV) ? KEYB : VALB;
    constexpr size_t UB = UB1 > RANKB ? UB1 : RANKB;
    static_assert(T < 65536, "wave counters are 16-bit");

    __shared__ __align__(16) unsigned char u_raw[UB];
    __shared__ __align__(16) unsigned char v_raw[SEPV ? VALB : 16];
    __shared__ OFF goff[RMAX];        // destination of slot 0 of each digit (SEG: from the segment's start)
    __shared__ uint32_t tot[RMAX];    // this tile's count per digit
    __shared__ uint32_t loc[RMAX];    // first LDS slot of each digit
    __shared__ uint32_t wsum[NW + 1];
    __shared__ uint32_t s_tile;

    uint64_t* wmask = reinterpret_cast<uint64_t*>(u_raw);          // [NG][RLO]
    uint16_t* wcnt = reinterpret_cast<uint16_t*>(u_raw + MSKB);    // [NW][R] (wide radices)
    Slot* gslot = reinterpret_cast<Slot*>(u_raw);                 // [NG][RLO] (radix <= 2^8)
    K* skeys = reinterpret_cast<K*>(u_raw);
    V* svals = reinterpret_cast<V*>(SEPV ? v_raw : u_raw);

    // With a route the buffers follow the rounds actually run: a round whose
    // digit is the same for every key leaves the order as it is and is
    // skipped; executed round e reads what round e-1 wrote (round 0 the
    // input) and writes `out` when an even number of executed rounds follow
    // it (in place: when e is odd, so that round 0 never writes its input).
    const K* __restrict__ kin = kin0;
    K* __restrict__ kout = kout0;
    const void* __restrict__ vin_ = vin0;
    void* __restrict__ vout_ = vout0;
    if (route) {
        const uint32_t m = route->mask;
        const int pass = shift / bits;
        if ((m >> pass) & 1u) return;
        const int e = __popc(~m & ((1u << pass) - 1u));
        const int E = __popc(~m & (route->passes >= 32 ? ~0u : (1u << route->passes) - 1u));
        const bool in_out = route->inplace ? ((e - 1) & 1) != 0 : ((E - e) & 1) == 0;  // round e-1
        const bool to_out = route->inplace ? (e & 1) != 0 : ((E - 1 - e) & 1) == 0;
        kin = reinterpret_cast<const K*>(e == 0 ? route->in : (in_out ? route->out : route->tmp));
        kout = reinterpret_cast<K*>(to_out ? route->out : route->tmp);
        vin_ = e == 0 ? route->vin : (in_out ? route->vout : route->vtmp);
        vout_ = to_out ? route->vout : route->vtmp;
    }
    const V* vin = reinterpret_cast<const V*>(vin_);
    V* vout = reinterpret_cast<V*>(vout_);

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int R = 1 << bits;
    const int lob = bits < 8 ? bits : 8;   // digit bits matched in LDS
    const uint32_t dmask = (uint32_t)R - 1;
    const uint32_t lomask = (1u << lob) - 1;

    // the XCD this workgroup runs on (the XCD order only; segment mode keeps
    // the single counter: the order's extra registers spill there and cost
    // more than the order saves)
    uint32_t xcd = 0;
    if constexpr (!SEG) {
        if (nx) {
            uint32_t xcc;
            asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
            xcd = (xcc & 0xFu) % nx;
        }
    }
    // SEG: the grid covers a bound on the tiles; the workgroups numbered
    // past the tiles in use take no tile id (exactly as many workgroups as
    // tiles take one, so every tile id is taken)
    if constexpr (SEG)
        if (blockIdx.x >= *sg.used) return;
    // Tile id.  Every tile a workgroup waits for in the look-back has a
    // smaller id, and is already held by a running workgroup or will be
    // taken by the next workgroup to start where it belongs:
    //   nx = 0: ids in the order workgroups reach one counter;
    //   nx > 0: chunks of XCD_CHUNK consecutive tiles per XCD, chunk k on XCD
    //   k mod nx, each XCD's workgroups taking its tiles in order from the
    //   XCD's own counter.  The hardware hands workgroup b to XCD b mod nx,
    //   so each XCD runs exactly as many workgroups as its chunks hold tiles
    //   (the grid covers whole rounds of nx chunks; tiles past the last key
    //   end at once), and neighbouring tiles, whose digit runs share cache
    //   lines at their ends, run on one XCD and write through one L2.
    if (tid == 0) {
        uint32_t t;
        if (!SEG && nx) {
            const uint32_t i = atomicAdd(tile_ctr + xcd, 1u);
            t = ((i / XCD_CHUNK) * nx + xcd) * XCD_CHUNK + i % XCD_CHUNK;
        } else {
            t = atomicAdd(tile_ctr, 1u);
        }
        s_tile = t;
    }
    if constexpr (!HALF)
        for (int i = tid; i < NW * R; i += NT) wcnt[i] = 0;
    for (int i = tid; i < (int)(MSKB / 8); i += NT) wmask[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    if constexpr (!SEG)
        if ((uint64_t)tile * T >= n) return;  // past the last key (the XCD order's whole rounds)
    // per look-back block of LBB tiles and digit: the tiles counted so far
    // (bits 26 up) and the sum of their counts (LBB * 2^16 < 2^26)
    // (after the tiles' words: n / T tiles, or in segment mode the bound)
    const size_t ntl = SEG ? (size_t)sg.max_tiles : (size_t)((n + T - 1) / T);
    uint32_t* __restrict__ bwsum = reinterpret_cast<uint32_t*>(lb + ntl * R);
    // SEG: the tiles of all segments in one numbering; a tile covers
    // positions [base, base + nvalid) of its segment [seg_lo, seg_lo +
    // seg_len), its look-back stops at the segment's first tile, and its
    // counts are counted from the segment's start
    uint32_t tl = tile;              // tile within its segment
    uint32_t blk0 = 0;               // look-back block of the segment's first tile
    uint64_t seg_lo = 0, seg_len = n;
    const uint32_t* __restrict__ hist0 = ghist;  // the round's digit counts (of the segment)
    if constexpr (SEG) {
        const SegTile dsc = sg.td[tile];
        if (dsc.len == 0) return;  // past the last tile of the large segments
        tl = dsc.tl;
        blk0 = dsc.bb;
        seg_lo = (uint64_t)dsc.lo;
        seg_len = (uint64_t)dsc.len;
        hist0 = sg.hist + (size_t)dsc.rank * (4 * RMAX) + (size_t)(shift / bits) * RMAX;
    }
    const uint64_t base = seg_lo + (uint64_t)tl * T;
    const uint64_t rem = seg_len - (uint64_t)tl * T;
    const uint32_t nvalid = (uint32_t)(rem < (uint64_t)T ? rem : (uint64_t)T);
    const bool full = nvalid == (uint32_t)T;
    const K* __restrict__ tin = kin + base;

    // ---- load (slots past nvalid hold the largest key: its digit is the
    //      largest of the round and it comes last in input order, so it takes
    //      the last LDS slots and never shifts a real key)
    K k[ITEMS];
    V v[VB ? ITEMS : 1];
    // item i of lane l of ranking group g is tile position g*GL*ITEMS + i*GL + l
    const uint32_t grp = tid / GL, gl = tid % GL;
    const uint32_t wb = grp * (ITEMS * GL) + gl;
    if (full) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) k[i] = tin[wb + i * GL];
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = wb + i * GL;
            k[i] = j < nvalid ? tin[j] : KeyMax<K>::v;
        }
    }
    if constexpr (VB != 0) {
        const V* __restrict__ vtin = vin + base;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = wb + i * GL;
            v[i] = (full || j < nvalid) ? vtin[j] : V(0);
        }
    }

    // ---- rank
    uint32_t dr[ITEMS];  // digit | rank-in-group << 16
    if constexpr (HALF) {
        Slot* wm = gslot + grp * RLO;
        const uint32_t mybit = 1u << gl;
        const uint32_t below = mybit - 1u;
        constexpr uint32_t MMASK = GL >= 32 ? ~0u : (1u << GL) - 1u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = (uint32_t)(k[i] >> shift) & dmask;
            Slot* slot = wm + d;
            // the mask field is the slot's low 32-bit word (the whole slot
            // when slots are 32-bit)
            atomicOr(reinterpret_cast<uint32_t*>(slot), mybit);
            const Slot sv = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t m = (uint32_t)sv & MMASK;
            const uint32_t c = (uint32_t)(sv >> CSH);
            const uint32_t lt = (uint32_t)__popc(m & below);
            const uint32_t cnt = (uint32_t)__popc(m);
            if (lt + 1 == cnt)
                __hip_atomic_store(slot, (Slot)((Slot)(c + cnt) << CSH), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            dr[i] = d | ((c + lt) << 16);
        }
    } else {
        uint16_t* wc = wcnt + wave * R;
        uint64_t* wm = wmask + wave * RLO;
        const uint64_t mybit = 1ull << lane;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = (uint32_t)(k[i] >> shift) & dmask;
            uint64_t* slot = wm + (d & lomask);
            atomicOr((unsigned long long*)slot, (unsigned long long)mybit);
            uint64_t m = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (MAXB > 8 && bits > 8) m &= match_digit<(MAXB > 8 ? MAXB - 8 : 1)>(d >> 8, bits - 8);
            const uint32_t lt = mbcnt(m);
            const uint32_t cnt = (uint32_t)__popcll(m);
            const uint32_t c = wc[d];
            if (lt + 1 == cnt) {
                wc[d] = (uint16_t)(c + cnt);
                __hip_atomic_store(slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            dr[i] = d | ((c + lt) << 16);
        }
    }
    __syncthreads();

    // ---- per digit: tile total (published at once for the tiles that
    //      follow), first LDS slot (exclusive scan over digits) and, per
    //      wave, the slot of the wave's first key of the digit
    {
        uint32_t part[PER];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid * PER + q;
            uint32_t t = 0;
            if (d < R) {
                if constexpr (HALF) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) t += (uint32_t)(gslot[g * RLO + d] >> CSH);
                } else {
#pragma unroll
                    for (int w = 0; w < NW; ++w) t += wcnt[w * R + d];
                }
                tot[d] = t;
                if (tl != 0)
                    st_agent(&lb[(size_t)tile * R + d], (LB)(((LB)FLAG_AGG << LBW<LB>::SH) | (LB)t));
                // this tile's count joins its look-back block's sum, with one
                // more tile counted in the word's top bits
                atomicAdd(&bwsum[(size_t)(blk0 + tl / LBB) * R + d], (1u << BW_SH) | t);
            }
            part[q] = t;
            s += t;
        }
        uint32_t total;
        uint32_t ex = block_excl_scan<NT>(s, wsum, &total);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid * PER + q;
            if (d < R) {
                loc[d] = ex;
                uint32_t run = ex;
                if constexpr (HALF) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const uint32_t c = (uint32_t)(gslot[g * RLO + d] >> CSH);
                        gslot[g * RLO + d] = (Slot)((Slot)run << CSH);
                        run += c;
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const uint32_t c = wcnt[w * R + d];
                        wcnt[w * R + d] = (uint16_t)run;
                        run += c;
                    }
                }
            }
            ex += part[q];
        }
    }

    __syncthreads();  // per-wave slot bases complete

    // ---- LDS slot of every key, then the reorder
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t d = dr[i] & 0xFFFFu;
        if constexpr (HALF)
            dr[i] = (uint32_t)(gslot[grp * RLO + d] >> CSH) + (dr[i] >> 16);
        else
            dr[i] = wcnt[wave * R + d] + (dr[i] >> 16);
    }
    __syncthreads();  // the counters share LDS with the key buffer
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) skeys[dr[i]] = k[i];
    if constexpr (SEPV) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) svals[dr[i]] = v[i];
    }
    __syncthreads();
    // the sorted keys this thread writes out, read from LDS now: half of the
    // workgroup has no look-back to do, and for the other half the reads
    // are done before its wait on the predecessors
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) k[q] = skeys[q * NT + tid];
    // uint32 keys with uint32 values: the values take the same trip now,
    // through the key buffer the keys have just left (measured: 2% faster
    // rounds; other payload widths keep their trip after the key write-out)
    constexpr bool VEARLY = sizeof(K) == 4 && VB == 4 && VB2 == 0;
    if constexpr (VEARLY) {
        if constexpr (!SEPV) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) svals[dr[i]] = v[i];
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) v[q] = svals[q * NT + tid];
    }

    // ---- global position of each digit's first key in this tile.  Taken
    //      after the LDS reorder: by then the tiles before this one have
    //      had longer to publish, so the look-back resolves in fewer steps.
    if (tl == 0) {
        // Tile 0 starts the chain: its exclusive prefix is the exclusive
        // scan of the round's global histogram (SEG: of its segment's).
        uint32_t part[PER];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid * PER + q;
            part[q] = d < R ? hist0[d] : 0u;
            s += part[q];
        }
        uint32_t total;
        uint32_t ex = block_excl_scan<NT>(s, wsum, &total);
        // (the block scan's barrier orders the loc[] writes above)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int d = tid * PER + q;
            if (d < R) {
                st_agent(&lb[(size_t)tile * R + d], (LB)(((LB)FLAG_PRE << LBW<LB>::SH) | (LB)(ex + tot[d])));
                goff[d] = (OFF)((int64_t)ex - (int64_t)loc[d]);
            }
            ex += part[q];
        }
    } else {
        __syncthreads();  // loc[] complete
        // Windowed look-back: each step reads the words of up to LBWIN
        // predecessors at once (independent loads, one memory round trip),
        // then consumes them nearest first, stopping at the first inclusive
        // prefix.  A predecessor that has not published yet (flag 0) is
        // waited for and re-read; no tile is ever skipped.
        for (int d = tid; d < R; d += NT) {
            LB excl = 0;
            int32_t j = (int32_t)tile - 1;  // nearest predecessor not yet consumed (tile ids < 2^31)
            uint32_t spins = 0;
            // first the tiles of this tile's own look-back block, one word
            // each; then whole blocks before it, each read as its last
            // tile's word (an inclusive prefix ends the walk) and its sum
            // (used once every tile of the block has counted); block 0 only
            // by its last tile's prefix, which holds the digit's global base.
            // SEG: the blocks are counted from the segment's first tile
            // (t0), their sums from its block blk0, and the walk ends inside
            // the segment
            const int32_t t0 = (int32_t)(tile - tl);
            const int32_t bfirst = t0 + (int32_t)(tl / LBB) * LBB;
            bool done = false;
            while (!done && j >= bfirst) {
                LB w[LBWIN];
#pragma unroll
                for (int q = 0; q < LBWIN; ++q)
                    w[q] = (j - q >= bfirst) ? ld_agent(&lb[(size_t)(j - q) * R + d]) : (LB)0;
                int used = 0;
#pragma unroll
                for (int q = 0; q < LBWIN; ++q) {
                    if (done || used < q || j - q < bfirst) continue;
                    const uint32_t f = (uint32_t)(w[q] >> LBW<LB>::SH);
                    if (f == 0) continue;
                    excl += w[q] & LBW<LB>::MASK;
                    used = q + 1;
                    if (f == FLAG_PRE) done = true;
                }
                j -= used;
                if (!done && used == 0) {
                    if (++spins > SPIN_LIMIT) {
                        atomicOr(status, STATUS_SPIN);
                        done = true;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            int32_t b = (int32_t)(tl / LBB) - 1;  // nearest block not yet consumed
            while (!done && b >= 0) {
                LB lt[LBWIN_B];
                uint32_t bs[LBWIN_B];
#pragma unroll
                for (int q = 0; q < LBWIN_B; ++q) {
                    const bool in = b - q >= 0;
                    lt[q] = in ? ld_agent(&lb[(size_t)(t0 + (b - q) * LBB + LBB - 1) * R + d]) : (LB)0;
                    bs[q] = (in && b - q > 0) ? ld_agent(&bwsum[(size_t)(blk0 + b - q) * R + d]) : 0u;
                }
                int used = 0;
#pragma unroll
                for (int q = 0; q < LBWIN_B; ++q) {
                    if (done || used < q || b - q < 0) continue;
                    if ((uint32_t)(lt[q] >> LBW<LB>::SH) == FLAG_PRE) {
                        excl += lt[q] & LBW<LB>::MASK;
                        done = true;
                        used = q + 1;
                    } else if (b - q > 0 && (bs[q] >> BW_SH) == (uint32_t)LBB) {
                        excl += (LB)(bs[q] & ((1u << BW_SH) - 1u));
                        used = q + 1;
                    }
                }
                b -= used;
                if (!done && used == 0) {
                    if (++spins > SPIN_LIMIT) {
                        atomicOr(status, STATUS_SPIN);
                        done = true;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            st_agent(&lb[(size_t)tile * R + d],
                     (LB)(((LB)FLAG_PRE << LBW<LB>::SH) | (LB)(excl + tot[d])));
            goff[d] = (OFF)((int64_t)excl - (int64_t)loc[d]);
        }
    }
    __syncthreads();


    // ---- write out: consecutive slots of one digit go to consecutive
    //      addresses, so each digit's run is a coalesced burst.  The
    //      destination is in [0, n) whenever the prefixes are right; the
    //      check keeps a wrong prefix (or an abandoned look-back) from writing
    //      outside the array and reports it instead.
    using UOFF = typename std::make_unsigned<OFF>::type;
    OFF dst[((VB && !VEARLY) || VB2) ? ITEMS : 1];
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
        const uint32_t j = q * NT + tid;
        if (full || j < nvalid) {
            const K key = k[q];
            const uint32_t d = (uint32_t)(key >> shift) & dmask;
            OFF o = goff[d] + (OFF)j;
            if ((uint64_t)(UOFF)o >= seg_len) {
                atomicOr(status, STATUS_RANGE);
                o = -1;
            } else {
                kout[seg_lo + (UOFF)o] = key;
                if constexpr (VEARLY) vout[seg_lo + (UOFF)o] = v[q];
            }
            if constexpr ((VB != 0 && !VEARLY) || VB2 != 0) dst[q] = o;
        }
    }
    if constexpr (VB != 0 && !VEARLY) {
        if constexpr (!SEPV) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) svals[dr[i]] = v[i];
            __syncthreads();
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const uint32_t j = q * NT + tid;
            if ((full || j < nvalid) && dst[q] >= 0) vout[seg_lo + (UOFF)dst[q]] = svals[j];
        }
    }
    if constexpr (VB2 != 0) {
        // the second payload follows the same slots and destinations
        using V2 = typename ValT<VB2>::type;
        const V2* __restrict__ v2in = reinterpret_cast<const V2*>(vin2_) + base;
        V2* __restrict__ v2out = reinterpret_cast<V2*>(vout2_);
        V2* sv2 = reinterpret_cast<V2*>(u_raw);
        V2 w[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = wb + i * GL;
            w[i] = (full || j < nvalid) ? v2in[j] : V2(0);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) sv2[dr[i]] = w[i];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const uint32_t j = q * NT + tid;
            if ((full || j < nvalid) && dst[q] >= 0) v2out[seg_lo + (UOFF)dst[q]] = sv2[j];
        }
    }
}

template <typename K, int VB, int MAXB, int ITEMS, typename LB, typename OFF, int VB2 = 0>
hipError_t launch_pass(const LsdPlan& p, const void* src, void* dst, const void* vsrc, void* vdst,
                       int pass, unsigned char* ws, hipStream_t st, const Route* route,
                       const void* v2src = nullptr, void* v2dst = nullptr) {
    uint32_t* ctr = reinterpret_cast<uint32_t*>(ws + p.off_ctr) + (size_t)pass * CTR_STRIDE;
    LB* lb = reinterpret_cast<LB*>(ws + p.off_lb) + (size_t)pass * p.lb_words;
    const uint32_t* gh = reinterpret_cast<const uint32_t*>(ws + p.off_hist) + (size_t)pass * p.R;
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + p.off_status);
    prof(st, p.kid_scatter, 0);
    hipLaunchKernelGGL((k_onesweep<K, VB, MAXB, ITEMS, LB, OFF, VB2>), dim3((unsigned)p.grid), dim3(NT),
                       0, st, (const K*)src, (K*)dst, vsrc, vdst, (uint64_t)p.n, pass * p.bits, p.bits,
                       ctr, lb, gh, status, route, v2src, v2dst, SegOs{}, p.nx);
    prof(st, p.kid_scatter, 1);
    return hipGetLastError();
}

template <typename K, int VB, int MAXB, int ITEMS>
hipError_t launch_pass_lb(const LsdPlan& p, const void* src, void* dst, const void* vsrc,
                          void* vdst, int pass, unsigned char* ws, hipStream_t st, const Route* route) {
    if (p.n >= (1ull << 31))
        return launch_pass<K, VB, MAXB, ITEMS, uint64_t, int64_t>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    if (p.lb64)
        return launch_pass<K, VB, MAXB, ITEMS, uint64_t, int32_t>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    return launch_pass<K, VB, MAXB, ITEMS, uint32_t, int32_t>(p, src, dst, vsrc, vdst, pass, ws, st, route);
}

template <typename K, int VB>
hipError_t launch_pass_k(const LsdPlan& p, const void* src, void* dst, const void* vsrc,
                         void* vdst, int pass, unsigned char* ws, hipStream_t st, const Route* route) {
    if constexpr (sizeof(K) == 4 && VB == 0) {
        if (p.bits <= 8 && p.tile == NT * LSD_ITEMS_SMALL)
            return launch_pass_lb<K, VB, 8, LSD_ITEMS_SMALL>(p, src, dst, vsrc, vdst, pass, ws, st, route);
        if (p.bits <= 8 && p.tile == NT * LSD_ITEMS_TINY)
            return launch_pass_lb<K, VB, 8, LSD_ITEMS_TINY>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    }
    if (p.bits <= 8)
        return launch_pass_lb<K, VB, 8, lsd_items(sizeof(K), VB, 8)>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    return launch_pass_lb<K, VB, 11, lsd_items(sizeof(K), VB, 11)>(p, src, dst, vsrc, vdst, pass, ws, st, route);
}

// 16-bit digit keys with an 8-byte payload and an optional second one
template <int VB2>
hipError_t launch_pass_k16(const LsdPlan& p, const void* src, void* dst, const void* vsrc,
                           void* vdst, int pass, unsigned char* ws, hipStream_t st,
                           const void* v2src, void* v2dst) {
    if (p.lb64)
        return launch_pass<uint16_t, 8, 8, 16, uint64_t, int64_t, VB2>(p, src, dst, vsrc, vdst, pass, ws,
                                                                        st, nullptr, v2src, v2dst);
    return launch_pass<uint16_t, 8, 8, 16, uint32_t, int32_t, VB2>(p, src, dst, vsrc, vdst, pass, ws, st,
                                                                    nullptr, v2src, v2dst);
}

hipError_t launch_pass_any(const LsdPlan& p, const void* src, void* dst, const void* vsrc,
                           void* vdst, int pass, unsigned char* ws, hipStream_t st, const Route* route,
                           const void* v2src = nullptr, void* v2dst = nullptr) {
    if (p.kb == 2)
        return p.vb2 ? launch_pass_k16<8>(p, src, dst, vsrc, vdst, pass, ws, st, v2src, v2dst)
                     : launch_pass_k16<0>(p, src, dst, vsrc, vdst, pass, ws, st, v2src, v2dst);
    if (p.kb == 4) {
        if (p.vb == 0) return launch_pass_k<uint32_t, 0>(p, src, dst, vsrc, vdst, pass, ws, st, route);
        if (p.vb == 4) return launch_pass_k<uint32_t, 4>(p, src, dst, vsrc, vdst, pass, ws, st, route);
        return launch_pass_k<uint32_t, 8>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    }
    if (p.vb == 0) return launch_pass_k<uint64_t, 0>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    if (p.vb == 4) return launch_pass_k<uint64_t, 4>(p, src, dst, vsrc, vdst, pass, ws, st, route);
    return launch_pass_k<uint64_t, 8>(p, src, dst, vsrc, vdst, pass, ws, st, route);
}

}  // namespace

rs_status fill_u32(void* p, size_t words, uint32_t v, hipStream_t st) {
    if (!words) return RS_OK;
    size_t g = (words + 255) / 256;
    if (g > 4096) g = 4096;
    prof(st, KID_FILL, 0);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, st, (uint32_t*)p, (uint64_t)words, v);
    prof(st, KID_FILL, 1);
    return launch_status();
}

rs_status stream_copy(const void* in, void* out, size_t bytes, hipStream_t st) {
    if (!bytes) return RS_OK;
    const bool aligned = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
    const uint64_t n16 = aligned ? bytes / 16 : 0;
    prof(st, KID_STREAM_COPY, 0);
    if (n16) {
        const uint64_t g = (n16 + COPY_CHUNK16 - 1) / COPY_CHUNK16;
        if (g > 0x7FFFFFFFull) return RS_ERR_UNSUPPORTED;
        hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)g), dim3(256), 0, st, (const uint4*)in, (uint4*)out, n16);
    }
    const uint64_t rest = bytes - 16 * n16;
    if (rest) {
        uint64_t g = (rest + 255) / 256;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)g), dim3(256), 0, st,
                           static_cast<const unsigned char*>(in) + 16 * n16, static_cast<unsigned char*>(out) + 16 * n16,
                           rest);
    }
    prof(st, KID_STREAM_COPY, 1);
    return launch_status();
}

// The XCD order needs the hardware to hand workgroup b to XCD b mod nx, which
// MI355X does with its 256 compute units in 8 XCDs (one partition); on any
// other shape the rounds keep the single counter.  RS_XCD_ORDER=0 turns the
// XCD order off.  Cached per device.
uint32_t xcd_order_count() {
    static std::atomic<int> cache[64];  // 0: not asked yet, else count + 1
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 0;
    }
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        int cus = 0;
        const char* e = getenv("RS_XCD_ORDER");
        const bool off = e && e[0] == '0';
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            cus = 0;
        }
        c = (!off && cus == 256) ? 8 + 1 : 1;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return (uint32_t)(c - 1);
}

bool lsd_plan(size_t n, int kb, int vb, int bits, LsdPlan* p, int vb2, int items) {
    if ((kb != 4 && kb != 8) || (vb != 0 && vb != 4 && vb != 8) || bits < 1 || bits > 11) {
        // the only other shape: 16-bit digit keys, radix 2^8, 8-byte payload(s)
        if (!(kb == 2 && vb == 8 && (vb2 == 0 || vb2 == 8) && bits == 8)) return false;
    }
    if (kb != 2 && vb2 != 0) return false;
    // digit counts, the global histograms and tile 0's prefix are 32-bit
    if ((uint64_t)n >= LSD_MAX_N) return false;
    LsdPlan q;
    q.n = n;
    q.kb = kb;
    q.vb = vb;
    q.bits = bits;
    q.passes = (8 * kb + bits - 1) / bits;
    q.R = 1 << bits;
    q.vb2 = vb2;
    const bool two_tiles = kb == 4 && vb == 0 && bits <= 8;  // the shape with a choice of tile
    if (items != 0 && !(two_tiles && (items == LSD_ITEMS_TINY || items == LSD_ITEMS_SMALL ||
                                      items == lsd_items(4, 0, 8))))
        return false;
    q.tile = NT * (kb == 2 ? 16
                   : (two_tiles && items)                     ? items
                   : (two_tiles && n < LSD_SMALL_N)           ? LSD_ITEMS_SMALL
                                                              : lsd_items(kb, vb, bits <= 8 ? 8 : 11));
    q.tiles = n ? (n + q.tile - 1) / q.tile : 0;
    // the XCD order once every XCD gets at least 8 chunks: with fewer tiles
    // the chunks would crowd onto the first XCDs (32 tiles: two of eight)
    q.nx = q.tiles >= (size_t)8 * XCD_CHUNK * 8 ? xcd_order_count() : 0;
    {
        const size_t round = (size_t)q.nx * XCD_CHUNK;
        q.grid = q.nx ? (q.tiles + round - 1) / round * round : q.tiles;
    }
    q.lb64 = n >= (1ull << 30);
    // per round: the tiles' look-back words, then one 32-bit block sum per
    // look-back block of LBB tiles and digit
    {
        const size_t wb = q.lb64 ? 8 : 4;
        const size_t blocks = (q.tiles + LBB - 1) / LBB;
        q.lb_words = q.tiles * (size_t)q.R + (4 * blocks * (size_t)q.R + wb - 1) / wb;
    }
    size_t off = 0;
    q.off_status = off;
    off += ALIGN;
    q.off_ctr = off;
    off += align_up(sizeof(uint32_t) * CTR_STRIDE * q.passes);
    q.off_hist = off;
    off += align_up(sizeof(uint32_t) * (size_t)q.passes * q.R);
    q.zero_bytes = off - q.off_status;
    q.off_lb = off;
    off += align_up((q.lb64 ? 8 : 4) * q.lb_words * q.passes);
    q.off_tk = off;
    off += align_up((size_t)kb * n);
    q.off_tv = off;
    off += align_up((size_t)vb * n);
    q.off_tv2 = off;
    off += align_up((size_t)vb2 * n);
    q.total = off;
    *p = q;
    return true;
}

// ---- segments sorted by shared onesweep rounds --------------------------------

// a valid segment inside [0, total) of a length the shared rounds take
__device__ __forceinline__ bool segos_large(const int64_t* off, uint64_t s, int64_t total) {
    const int64_t b = off[s], e = off[s + 1];
    return b >= 0 && e > b && e <= total && seg_shared_len((uint64_t)(e - b));
}

// ttile[s] = tiles of the large segments before s, lrank[s] = large segments
// before s, bbase[s] = their look-back blocks before s (entries S: the
// totals); one workgroup scans S in chunks.  Offsets that overlap (invalid:
// reported by the classification) can add up to more than the plan holds:
// then the range error is raised and the totals are set to zero, so that
// no later kernel of the rounds touches a segment.
__global__ __launch_bounds__(1024) void k_segos_scan(const int64_t* __restrict__ off, uint64_t S, int64_t total,
                                                     uint32_t* __restrict__ ttile, uint32_t* __restrict__ lrank,
                                                     uint32_t* __restrict__ bbase, uint64_t max_tiles,
                                                     uint64_t max_blocks, uint64_t max_large,
                                                     uint32_t* __restrict__ status) {
    __shared__ uint32_t wsum[1024 / WAVE + 1];
    const uint32_t tid = threadIdx.x;
    uint64_t carry = 0, carryb = 0, carryl = 0;  // tiles, look-back blocks, large segments
    for (uint64_t c0 = 0; c0 < S; c0 += 1024) {
        const uint64_t s = c0 + tid;
        // per segment at most 2^30 / SEG_OS_TILE tiles: a chunk's sums fit 32 bits
        uint32_t v = 0, vb = 0, vl = 0;
        if (s < S && segos_large(off, s, total)) {
            v = (uint32_t)((off[s + 1] - off[s] + (int64_t)SEG_OS_TILE - 1) / (int64_t)SEG_OS_TILE);
            vb = (v + LBB - 1) / LBB;
            vl = 1;
        }
        uint32_t tt, tb, tl;
        const uint32_t et = block_excl_scan<1024>(v, wsum, &tt);
        const uint32_t eb = block_excl_scan<1024>(vb, wsum, &tb);
        const uint32_t el = block_excl_scan<1024>(vl, wsum, &tl);
        if (s < S) {
            ttile[s] = (uint32_t)(carry + et);
            bbase[s] = (uint32_t)(carryb + eb);
            lrank[s] = (uint32_t)(carryl + el);
        }
        carry += tt;
        carryb += tb;
        carryl += tl;
    }
    if (tid == 0) {
        const bool fits = carry <= max_tiles && carryb <= max_blocks && carryl <= max_large;
        if (!fits) atomicOr(status, STATUS_RANGE);
        ttile[S] = fits ? (uint32_t)carry : 0u;
        lrank[S] = fits ? (uint32_t)carryl : 0u;
        bbase[S] = fits ? (uint32_t)carryb : 0u;
    }
}

// The last s in [0, S) with idx[s] <= t, for a non-decreasing idx: with
// idx an exclusive scan of per-segment counts, the segment that holds item
// t of the concatenated numbering (segments with no items are skipped over,
// as the next one starts at the same value).
__device__ __forceinline__ uint64_t segos_find(const uint32_t* __restrict__ idx, uint64_t S, uint32_t t) {
    uint64_t lo = 0, hi = S;  // idx[lo] <= t < idx[hi] (idx[S] > t)
    while (hi - lo > 1) {
        const uint64_t m = (lo + hi) >> 1;
        if (idx[m] <= t) lo = m;
        else hi = m;
    }
    return lo;
}

// Tile descriptors (unused tiles of the round's grid get length 0), the
// rounds' look-back words and the per-segment histograms zeroed.
__global__ __launch_bounds__(256) void k_segos_desc(const int64_t* __restrict__ off, uint64_t S,
                                                    const uint32_t* __restrict__ ttile,
                                                    const uint32_t* __restrict__ lrank,
                                                    const uint32_t* __restrict__ bbase, SegTile* __restrict__ td,
                                                    uint32_t* __restrict__ hist, uint32_t* __restrict__ lbz,
                                                    uint64_t max_tiles, uint64_t max_blocks) {
    const uint64_t i0 = (uint64_t)blockIdx.x * 256 + threadIdx.x, step = (uint64_t)gridDim.x * 256;
    // round r's words: lbz[r * (max_tiles + max_blocks) * 256 ...], the
    // first ttile[S] tiles' in use, then from max_tiles the first bbase[S]
    // blocks' sums
    const uint64_t zt = (uint64_t)ttile[S] * 256, zb = (uint64_t)bbase[S] * 256;
    for (int r = 0; r < 4; ++r) {
        uint32_t* lr = lbz + (uint64_t)r * (max_tiles + max_blocks) * 256;
        for (uint64_t j = i0; j < zt; j += step) lr[j] = 0u;
        for (uint64_t j = i0; j < zb; j += step) lr[max_tiles * 256 + j] = 0u;
    }
    const uint64_t zh = (uint64_t)lrank[S] * 1024;
    for (uint64_t j = i0; j < zh; j += step) hist[j] = 0u;
    const uint32_t used = ttile[S];
    for (uint64_t t = i0; t < max_tiles; t += step) {
        if (t >= used) {
            td[t] = SegTile{0, 0, 0, 0, 0, 0};
            continue;
        }
        const uint64_t s = segos_find(ttile, S, (uint32_t)t);
        td[t] = SegTile{off[s], off[s + 1] - off[s], (uint32_t)t - ttile[s], lrank[s], bbase[s], 0};
    }
}

// Per-segment digit counts of the four rounds: one workgroup per look-back
// block (LBB tiles of one segment) counts its keys in lane-column LDS
// counters and adds the non-zero counts to its segment's histogram.
__global__ __launch_bounds__(512) void k_segos_hist(const uint32_t* __restrict__ keys, const int64_t* __restrict__ off,
                                                    uint64_t S, const uint32_t* __restrict__ lrank,
                                                    const uint32_t* __restrict__ bbase, uint32_t* __restrict__ hist) {
    constexpr int HC = 8;
    constexpr uint64_t BK = (uint64_t)LBB * SEG_OS_TILE;  // keys per block
    __shared__ uint32_t hc[4 * 256 * HC];
    const uint32_t tid = threadIdx.x, col = tid & (HC - 1);
    const uint32_t nb = bbase[S];
    for (uint32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint64_t s = segos_find(bbase, S, b);
        const uint64_t lo = (uint64_t)off[s] + (uint64_t)(b - bbase[s]) * BK;
        const uint64_t e = (uint64_t)off[s + 1];
        const uint64_t L = e - lo < BK ? e - lo : BK;
        const uint32_t* __restrict__ in = keys + lo;
        for (int i = tid; i < 4 * 256 * HC; i += 512) hc[i] = 0;
        __syncthreads();
        uint64_t q = tid;
        for (; q + 3 * 512 < L; q += 4 * 512) {
            const uint32_t k0 = in[q], k1 = in[q + 512], k2 = in[q + 1024], k3 = in[q + 1536];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                atomicAdd(&hc[(p * 256 + __builtin_amdgcn_ubfe(k0, 8 * p, 8)) * HC + col], 1u);
                atomicAdd(&hc[(p * 256 + __builtin_amdgcn_ubfe(k1, 8 * p, 8)) * HC + col], 1u);
                atomicAdd(&hc[(p * 256 + __builtin_amdgcn_ubfe(k2, 8 * p, 8)) * HC + col], 1u);
                atomicAdd(&hc[(p * 256 + __builtin_amdgcn_ubfe(k3, 8 * p, 8)) * HC + col], 1u);
            }
        }
        for (; q < L; q += 512) {
            const uint32_t k = in[q];
#pragma unroll
            for (int p = 0; p < 4; ++p) atomicAdd(&hc[(p * 256 + __builtin_amdgcn_ubfe(k, 8 * p, 8)) * HC + col], 1u);
        }
        __syncthreads();
        uint32_t* h = hist + (size_t)lrank[s] * 1024;
        for (int r = tid; r < 1024; r += 512) {
            uint32_t c = 0;
#pragma unroll
            for (int cc = 0; cc < HC; ++cc) c += hc[r * HC + ((cc + r) & (HC - 1))];
            if (c) atomicAdd(&h[r], c);
        }
        __syncthreads();
    }
}

rs_status lsd_run(const LsdPlan& p, const void* kin, void* kout, const void* vin, void* vout,
                  void* ws_, hipStream_t st, const void* vin2, void* vout2) {
    if (p.n == 0) return RS_OK;
    unsigned char* ws = static_cast<unsigned char*>(ws_);
    rs_status rc = fill_u32(ws + p.off_status, p.zero_bytes / 4, 0u, st);
    if (rc != RS_OK) return rc;
    // one read of the keys for every round's histogram (+ look-back zeroing)
    {
        const size_t lb_u32 = (p.lb64 ? 2 : 1) * p.lb_words * p.passes;
        size_t g = (p.n + HIST_NT * 16 - 1) / (HIST_NT * 16);
        size_t gz = (lb_u32 + HIST_NT * 16 - 1) / (HIST_NT * 16);
        if (gz > g) g = gz;
        if (g > 4096) g = 4096;
        if (g < 1) g = 1;
        const size_t shm = sizeof(uint32_t) * (size_t)p.passes * p.R;
        uint32_t* gh = reinterpret_cast<uint32_t*>(ws + p.off_hist);
        uint32_t* zp = reinterpret_cast<uint32_t*>(ws + p.off_lb);
        prof(st, p.kid_hist, 0);
        if (p.bits == 8 && p.kb == 4 && p.passes == 4) {
            launch_hist_fixed<uint32_t, 8, 4, 16>(kin, p.n, gh, zp, lb_u32, st);
        } else if (p.bits == 8 && p.kb == 2 && p.passes == 2) {
            launch_hist_fixed<uint16_t, 8, 2, 16>(kin, p.n, gh, zp, lb_u32, st);
        } else if (p.bits == 8 && p.kb == 8 && p.passes == 8) {
            launch_hist_fixed<uint64_t, 8, 8, 8>(kin, p.n, gh, zp, lb_u32, st);
        } else if (p.kb == 2)
            hipLaunchKernelGGL(k_hist<uint16_t>, dim3((unsigned)g), dim3(HIST_NT), shm, st,
                               (const uint16_t*)kin, (uint64_t)p.n, p.bits, p.passes, gh, zp,
                               (uint64_t)lb_u32);
        else if (p.kb == 4)
            hipLaunchKernelGGL(k_hist<uint32_t>, dim3((unsigned)g), dim3(HIST_NT), shm, st,
                               (const uint32_t*)kin, (uint64_t)p.n, p.bits, p.passes, gh, zp,
                               (uint64_t)lb_u32);
        else
            hipLaunchKernelGGL(k_hist<uint64_t>, dim3((unsigned)g), dim3(HIST_NT), shm, st,
                               (const uint64_t*)kin, (uint64_t)p.n, p.bits, p.passes, gh, zp,
                               (uint64_t)lb_u32);
        prof(st, p.kid_hist, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
    }
    // Buffers: the rounds alternate between `out` and the workspace copy so
    // that the last round writes `out`.  For an in-place sort with an odd
    // round count the first round cannot write `out` (it is being read), so
    // the rounds end in the workspace and one copy follows.
    void* tk = ws + p.off_tk;
    void* tv = ws + p.off_tv;
    void* tv2 = ws + p.off_tv2;
    const int P = p.passes;
    if (p.skip) {
        // which rounds run is known only on the device: each round reads the
        // route and finds its buffers there
        Route* rt = reinterpret_cast<Route*>(ws + p.off_status + ROUTE_OFFSET);
        hipLaunchKernelGGL(k_route, dim3(1), dim3(256), 0, st, reinterpret_cast<const uint32_t*>(ws + p.off_hist),
                           P, p.R, (uint64_t)p.n, rt, kin, kout, (void*)tk, vin, vout, (void*)tv);
        if ((rc = launch_status()) != RS_OK) return rc;
        for (int j = 0; j < P; ++j) {
            hipError_t e = launch_pass_any(p, kin, kout, vin, vout, j, ws, st, rt);
            if (e != hipSuccess) return hip_fail(e);
        }
        prof(st, KID_COPY, 0);
        const uint64_t kw = p.n * p.kb / 4, vw = p.n * p.vb / 4;
        size_t g = (kw + 255) / 256;
        if (g > 2048) g = 2048;
        hipLaunchKernelGGL(k_route_copy, dim3((unsigned)g), dim3(256), 0, st, rt, kw, vw);
        prof(st, KID_COPY, 1);
        return launch_status();
    }
    const bool inplace = kin == kout;
    const bool copy_back = inplace && (P % 2 == 1);
    const void* src = kin;
    const void* vsrc = vin;
    const void* v2src = vin2;
    for (int j = 0; j < P; ++j) {
        const int left = P - 1 - j;  // rounds after this one
        bool to_out = (left % 2 == 0);
        if (copy_back) to_out = !to_out;
        void* dst = to_out ? kout : tk;
        void* vdst = to_out ? vout : tv;
        void* v2dst = to_out ? vout2 : tv2;
        hipError_t e = launch_pass_any(p, src, dst, vsrc, vdst, j, ws, st, nullptr, v2src, v2dst);
        if (e != hipSuccess) return hip_fail(e);
        src = dst;
        vsrc = vdst;
        v2src = v2dst;
    }
    if (copy_back) {
        prof(st, KID_COPY, 0);
        hipError_t e = hipMemcpyAsync(kout, tk, p.n * p.kb, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && p.vb)
            e = hipMemcpyAsync(vout, tv, p.n * p.vb, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && p.vb2)
            e = hipMemcpyAsync(vout2, tv2, p.n * p.vb2, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e);
        prof(st, KID_COPY, 1);
    }
    return RS_OK;
}


// The segments of the lengths seg_shared_len takes: tile map and
// histograms, then four rounds of the device-wide round's kernel over all
// their tiles at once (in -> tmp -> out -> tmp -> out), the look-back of
// each tile inside its own segment.
rs_status segos_run(const SegPlan& p, const uint32_t* in, uint32_t* out, uint32_t* tmp, const int64_t* off,
                    uint64_t S, int64_t total, unsigned char* ws, hipStream_t st) {
    if (S == 0 || p.max_tiles == 0) return RS_OK;
    uint32_t* ttile = reinterpret_cast<uint32_t*>(ws + p.off_ttile);
    uint32_t* lrank = reinterpret_cast<uint32_t*>(ws + p.off_lrank);
    uint32_t* bbase = reinterpret_cast<uint32_t*>(ws + p.off_bbase);
    SegTile* td = reinterpret_cast<SegTile*>(ws + p.off_tdesc);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + p.off_shist);
    uint32_t* ctr = reinterpret_cast<uint32_t*>(ws + p.off_osctr);
    uint32_t* lbw = reinterpret_cast<uint32_t*>(ws + p.off_oslb);
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + p.off_status);
    prof(st, KID_SEG_PLAN, 0);
    hipLaunchKernelGGL(k_segos_scan, dim3(1), dim3(1024), 0, st, off, S, total, ttile, lrank, bbase,
                       (uint64_t)p.max_tiles, (uint64_t)p.max_blocks, (uint64_t)p.max_large, status);
    {
        const uint64_t zw = (uint64_t)(p.max_tiles + p.max_blocks) * 256;
        uint64_t g = (zw + 255) / 256;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_segos_desc, dim3((unsigned)g), dim3(256), 0, st, off, S, ttile, lrank, bbase, td, hist,
                           lbw, (uint64_t)p.max_tiles, (uint64_t)p.max_blocks);
        g = p.max_blocks < 4096 ? p.max_blocks : 4096;
        hipLaunchKernelGGL(k_segos_hist, dim3((unsigned)g), dim3(512), 0, st, in, off, S, lrank, bbase, hist);
    }
    prof(st, KID_SEG_PLAN, 1);
    rs_status rc = launch_status();
    if (rc != RS_OK) return rc;
    SegOs sg;
    sg.td = td;
    sg.used = ttile + S;
    sg.max_tiles = (uint32_t)p.max_tiles;
    sg.hist = hist;
    const uint64_t grid = p.max_tiles;
    const uint32_t* src = in;
    for (int r = 0; r < 4; ++r) {
        uint32_t* dst = (r & 1) ? out : tmp;
        prof(st, KID_SEG_ROUND, 0);
        hipLaunchKernelGGL((k_onesweep<uint32_t, 0, 8, 28, uint32_t, int32_t, 0, true>), dim3((unsigned)grid),
                           dim3(NT), 0, st, src, dst, nullptr, nullptr, (uint64_t)0, 8 * r, 8, ctr + (size_t)r * CTR_STRIDE,
                           lbw + (size_t)r * (p.max_tiles + p.max_blocks) * 256, nullptr, status, nullptr, nullptr,
                           nullptr, sg, 0u);
        prof(st, KID_SEG_ROUND, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
        src = dst;
    }
    return RS_OK;
}

}  // namespace rs
