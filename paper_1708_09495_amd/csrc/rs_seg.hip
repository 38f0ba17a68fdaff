// rs_seg.hip -- batched segmented sort (an extension beyond the paper: many
// independent arrays of uneven length).
//
// Plan (three small kernels, all on the device):
//   classify  each segment's length class (lengths in (2^(c-1), 2^c]);
//   scan      class cursors, largest class first;
//   scatter   segment ids into a queue ordered by decreasing class, so the
//             longest segments start first (longest-processing-time order).
// Sort (one persistent kernel): every workgroup pops the next queue entry
// until the queue is empty and sorts that segment by itself, unless the
// shared rounds take it (the default, seg_shared_len: 10,241 .. 14,336 keys
// and 16,385 .. 2^30 - 1 keys):
//   length <= 16384  in LDS, with BTN, OET or the LDS radix sort as the
//                    tuning table says for the length class;
//   longer           with the shared rounds (the default), only segments of
//                    2^30 keys and more; without them (RS_ALGO_LSD, the
//                    block networks' runs) every such segment: the
//                    radix-2^8 count-sort rounds of Section 3 run by the
//                    one workgroup: one read counts all four rounds' digits,
//                    then each round walks the segment's tiles IN ORDER,
//                    ranking each tile stably in LDS and writing each digit's
//                    run at that digit's running offset -- the running
//                    offsets stay in LDS, so no tile waits on another
//                    workgroup.
// Segments are independent, so workgroups never wait on each other and every
// workgroup leaves once the queue is exhausted.  The segments the shared
// rounds take are then sorted together by the device-wide round's kernel
// over all their tiles (segos_run, in rs_lsd.hip).
#include "rs_internal.hpp"
#include "rs_small_dev.h"

namespace rs {
namespace {

constexpr int SG_NT = 512;
constexpr int SG_NW = SG_NT / WAVE;
constexpr int SG_ITEMS = 16;                  // keys per thread of a large-path tile (at most)
constexpr int SG_T = SG_NT * SG_ITEMS;        // keys per tile of the large path (at most)
constexpr int SG_R = 256;                     // radix 2^8
constexpr int SG_P = 4;                       // rounds for 32-bit keys
constexpr int NCLASS = 64;
constexpr int SMEM = 16896 * 4;               // BTN/OET: p*(N+1) words for n_pad <= 16384

// Length class k of the tuning table: lengths in (2^(k-1), 2^k], 0 for one
// key (and for the empty and invalid segments, which are skipped).
__device__ __forceinline__ int len_class(int64_t L) {
    return L <= 1 ? 0 : 64 - __clzll((unsigned long long)(L - 1));
}

// Per-class segment counts: each workgroup counts its segments in LDS and
// adds one word per class to the global counts.
__global__ void k_seg_classify(const int64_t* __restrict__ off, uint64_t S, int64_t total,
                               uint32_t* __restrict__ cnt, uint32_t* __restrict__ status) {
    __shared__ uint32_t lc[NCLASS];
    for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x) lc[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride) {
        const int64_t b = off[s], e = off[s + 1];
        if (b < 0 || e < b || e > total || (s == 0 && b != 0)) atomicOr(status, STATUS_RANGE);
        const int c = (b < 0 || e < b || e > total) ? 0 : len_class(e - b);
        atomicAdd(&lc[c], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x)
        if (lc[i]) atomicAdd(&cnt[i], lc[i]);
}

// One workgroup of NCLASS threads: cursor[c] = number of segments in classes
// above c (the queue lists the largest class first).
__global__ void k_seg_scan(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ cursor) {
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int c = NCLASS - 1; c >= 0; --c) {
            cursor[c] = s;
            s += cnt[c];
        }
    }
}

// Segment ids into the queue, by class: per chunk of the workgroup's
// segments, LDS ranks within each class and one global reservation per class.
__global__ void k_seg_scatter(const int64_t* __restrict__ off, uint64_t S, int64_t total,
                              uint32_t* __restrict__ cursor, uint32_t* __restrict__ order) {
    __shared__ uint32_t lc[NCLASS], lbase[NCLASS];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c0 = (uint64_t)blockIdx.x * blockDim.x; c0 < S; c0 += stride) {
        for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x) lc[i] = 0;
        __syncthreads();
        const uint64_t s = c0 + threadIdx.x;
        int c = 0;
        uint32_t r = 0;
        if (s < S) {
            const int64_t b = off[s], e = off[s + 1];
            c = (b < 0 || e < b || e > total) ? 0 : len_class(e - b);
            r = atomicAdd(&lc[c], 1u);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < NCLASS; i += blockDim.x)
            if (lc[i]) lbase[i] = atomicAdd(&cursor[i], lc[i]);
        __syncthreads();
        if (s < S) {
            const uint32_t pos = lbase[c] + r;
            if (pos < S) order[pos] = (uint32_t)s;
        }
        __syncthreads();
    }
}

// ---- large segments: radix-2^8 rounds by one workgroup ------------------------

// Tiles of T keys over a segment of L keys, and the keys of tile t: every
// index and bound below is 64-bit, so segments up to 2^32 - 1 keys (the
// largest the entry point accepts) never wrap a loop counter.
__host__ __device__ constexpr uint64_t seg_tiles(uint64_t L, uint64_t T) { return (L + T - 1) / T; }
__host__ __device__ constexpr uint32_t seg_tile_keys(uint64_t L, uint64_t t, uint64_t T) {
    return t * T >= L ? 0u : (L - t * T < T ? (uint32_t)(L - t * T) : (uint32_t)T);
}
static_assert(seg_tiles(0xFFFFFFFFull, 8192) == 524288 && seg_tile_keys(0xFFFFFFFFull, 524287, 8192) == 8191 &&
                  seg_tile_keys(0xFFFFFFFFull, 524288, 8192) == 0 && seg_tiles(0xFFFFFFFFull, 4096) == 1048576 &&
                  seg_tile_keys(0xFFFFFFFFull, 1048575, 4096) == 4095,
              "the longest segment's last tile is partial and nothing follows it");

// IT keys per thread: tiles of SG_NT * IT keys (the tuning table picks 8 or
// 16 per length class).
template <int IT>
__device__ void seg_large(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                          uint32_t* __restrict__ tmp, uint64_t L, unsigned char* smem,
                          uint32_t* status) {
    constexpr int TK = SG_NT * IT;  // keys per tile
    uint64_t* wmask = reinterpret_cast<uint64_t*>(smem);              // NW*R
    uint16_t* wcnt = reinterpret_cast<uint16_t*>(smem + 16384);       // NW*R
    uint32_t* skeys = reinterpret_cast<uint32_t*>(smem + 20480);      // T
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + 53248);       // P*R
    uint32_t* run = hist + SG_P * SG_R;                               // R
    uint32_t* loc = run + SG_R;                                       // R
    uint32_t* tot = loc + SG_R;                                       // R
    uint32_t* wsum = tot + SG_R;                                      // NW+1
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // one read counts the digits of all four rounds (four loads in flight)
    // into counters laid out by lane (word = round, digit, lane mod HC; the
    // ranking buffers, not in use yet, hold them), so that lanes on one
    // digit do not pile onto one LDS bank; the columns are summed after
    constexpr int HC = 8;
    static_assert((size_t)SG_P * SG_R * HC * 4 <= 53248, "the column counters fit below the histograms");
    uint32_t* hc = reinterpret_cast<uint32_t*>(smem);
    const uint32_t col = tid & (HC - 1);
    for (int i = tid; i < SG_P * SG_R * HC; i += SG_NT) hc[i] = 0;
    __syncthreads();
    uint64_t q = tid;
    for (; q + 3 * SG_NT < L; q += 4 * SG_NT) {
        const uint32_t k0 = in[q], k1 = in[q + SG_NT], k2 = in[q + 2 * SG_NT], k3 = in[q + 3 * SG_NT];
#pragma unroll
        for (int p = 0; p < SG_P; ++p) {
            atomicAdd(&hc[(p * SG_R + __builtin_amdgcn_ubfe(k0, 8 * p, 8)) * HC + col], 1u);
            atomicAdd(&hc[(p * SG_R + __builtin_amdgcn_ubfe(k1, 8 * p, 8)) * HC + col], 1u);
            atomicAdd(&hc[(p * SG_R + __builtin_amdgcn_ubfe(k2, 8 * p, 8)) * HC + col], 1u);
            atomicAdd(&hc[(p * SG_R + __builtin_amdgcn_ubfe(k3, 8 * p, 8)) * HC + col], 1u);
        }
    }
    for (; q < L; q += SG_NT) {
        const uint32_t k = in[q];
#pragma unroll
        for (int p = 0; p < SG_P; ++p)
            atomicAdd(&hc[(p * SG_R + __builtin_amdgcn_ubfe(k, 8 * p, 8)) * HC + col], 1u);
    }
    __syncthreads();
    for (int r = tid; r < SG_P * SG_R; r += SG_NT) {
        uint32_t c_sum = 0;
#pragma unroll
        for (int c = 0; c < HC; ++c) c_sum += hc[r * HC + ((c + r) & (HC - 1))];
        hist[r] = c_sum;
    }
    __syncthreads();
    for (int i = tid; i < SG_NW * SG_R; i += SG_NT) {
        wmask[i] = 0;
        wcnt[i] = 0;
    }
    const uint64_t mybit = 1ull << lane;
    const uint32_t* src = in;
    for (int p = 0; p < SG_P; ++p) {
        // four rounds: in -> tmp -> out -> tmp -> out
        uint32_t* dst = (p & 1) ? out : tmp;
        const int shift = 8 * p;
        __syncthreads();
        {
            const uint32_t v = tid < (uint32_t)SG_R ? hist[p * SG_R + tid] : 0u;
            uint32_t total;
            const uint32_t ex = block_excl_scan<SG_NT>(v, wsum, &total);
            if (tid < (uint32_t)SG_R) run[tid] = ex;
        }
        // keys of the tile at b (past the end: the largest key); the next
        // tile of the round loads while the current one is written out
        const uint32_t wb = wave * (IT * WAVE) + lane;
        auto load_tile = [&](uint64_t t, uint32_t (&kt)[IT]) {
            const uint32_t nv = seg_tile_keys(L, t, TK);
            const uint32_t* __restrict__ ts = src + t * TK;
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t j = wb + i * WAVE;
                kt[i] = j < nv ? ts[j] : 0xFFFFFFFFu;
            }
        };
        uint32_t kn[IT];
        load_tile(0, kn);
        const uint64_t ntiles = seg_tiles(L, TK);
        for (uint64_t ti = 0; ti < ntiles; ++ti) {
            const uint32_t nvalid = seg_tile_keys(L, ti, TK);
            uint32_t k[IT];
#pragma unroll
            for (int i = 0; i < IT; ++i) k[i] = kn[i];
            __syncthreads();  // run[] set; previous tile finished with wcnt/skeys
            uint32_t dr[IT];
            {
                uint16_t* wc = wcnt + wave * SG_R;
                uint64_t* wm = wmask + wave * SG_R;
#pragma unroll
                for (int i = 0; i < IT; ++i) {
                    const uint32_t d = (k[i] >> shift) & 255u;
                    atomicOr((unsigned long long*)&wm[d], (unsigned long long)mybit);
                    const uint64_t m =
                        __hip_atomic_load(&wm[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const uint32_t lt = mbcnt(m);
                    const uint32_t cnt = (uint32_t)__popcll(m);
                    const uint32_t c = wc[d];
                    if (lt + 1 == cnt) {
                        wc[d] = (uint16_t)(c + cnt);
                        __hip_atomic_store(&wm[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    dr[i] = d | ((c + lt) << 16);
                }
            }
            __syncthreads();
            uint32_t t = 0;
            if (tid < (uint32_t)SG_R) {
                uint32_t s = 0;
#pragma unroll
                for (int w = 0; w < SG_NW; ++w) {
                    const uint32_t c = wcnt[w * SG_R + tid];
                    wcnt[w * SG_R + tid] = (uint16_t)s;
                    s += c;
                }
                t = s;
                tot[tid] = s;
            }
            {
                uint32_t total;
                const uint32_t ex = block_excl_scan<SG_NT>(t, wsum, &total);
                if (tid < (uint32_t)SG_R) loc[tid] = ex;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const uint32_t d = dr[i] & 0xFFFFu;
                skeys[loc[d] + wcnt[wave * SG_R + d] + (dr[i] >> 16)] = k[i];
            }
            __syncthreads();
            load_tile(ti + 1, kn);
            // each digit's run of this tile lands at the digit's running offset
#pragma unroll
            for (int q = 0; q < IT; ++q) {
                const uint32_t j = q * SG_NT + tid;
                if (j < nvalid) {
                    const uint32_t key = skeys[j];
                    const uint32_t d = (key >> shift) & 255u;
                    const uint32_t o = run[d] - loc[d] + j;
                    if ((uint64_t)o < L) dst[o] = key;
                    else atomicOr(status, STATUS_RANGE);
                }
            }
            __syncthreads();
            if (tid < (uint32_t)SG_R) run[tid] += tot[tid];
            for (int i = tid; i < SG_NW * SG_R; i += SG_NT) wcnt[i] = 0;
        }
        src = dst;
    }
}

// ---- small segments in LDS -------------------------------------------------------

__device__ void seg_small(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t L,
                          int algo, int p, unsigned char* smem) {
    uint32_t* sh = reinterpret_cast<uint32_t*>(smem);
    if (algo == RS_ALGO_LDS_RADIX && L <= (uint32_t)SG_NT * 16) {
        uint64_t* wmask = reinterpret_cast<uint64_t*>(smem);
        uint32_t* sk = reinterpret_cast<uint32_t*>(smem);            // aliases the masks
        uint16_t* wcnt = reinterpret_cast<uint16_t*>(smem + 32768);
        uint32_t* loc = reinterpret_cast<uint32_t*>(smem + 36864);
        uint32_t* wsum = loc + 256;
        const uint32_t items = (L + SG_NT - 1) / SG_NT;
        if (items <= 1) lds_radix_sort<1, SG_NT>(in, out, L, wmask, wcnt, loc, wsum, sk);
        else if (items <= 2) lds_radix_sort<2, SG_NT>(in, out, L, wmask, wcnt, loc, wsum, sk);
        else if (items <= 4) lds_radix_sort<4, SG_NT>(in, out, L, wmask, wcnt, loc, wsum, sk);
        else if (items <= 8) lds_radix_sort<8, SG_NT>(in, out, L, wmask, wcnt, loc, wsum, sk);
        else lds_radix_sort<16, SG_NT>(in, out, L, wmask, wcnt, loc, wsum, sk);
        return;
    }
    uint32_t npad = 1;
    while (npad < L) npad <<= 1;
    // p within what a SG_NT-thread workgroup holds: p <= SG_NT, N <= 32
    if (p < 1) p = 1;
    if (p > SG_NT) p = SG_NT;
    if ((uint32_t)p > npad) p = (int)npad;
    while (npad / (uint32_t)p > 32u) p <<= 1;
    const uint32_t N = npad / (uint32_t)p;
    const bool oet = algo == RS_ALGO_OET;
    switch (N) {
        case 1: oet ? oet_sort<1>(in, out, L, p, sh) : btn_sort<1>(in, out, L, p, sh); break;
        case 2: oet ? oet_sort<2>(in, out, L, p, sh) : btn_sort<2>(in, out, L, p, sh); break;
        case 4: oet ? oet_sort<4>(in, out, L, p, sh) : btn_sort<4>(in, out, L, p, sh); break;
        case 8: oet ? oet_sort<8>(in, out, L, p, sh) : btn_sort<8>(in, out, L, p, sh); break;
        case 16: oet ? oet_sort<16>(in, out, L, p, sh) : btn_sort<16>(in, out, L, p, sh); break;
        default: oet ? oet_sort<32>(in, out, L, p, sh) : btn_sort<32>(in, out, L, p, sh); break;
    }
}

__attribute__((amdgpu_waves_per_eu(4))) __global__ __launch_bounds__(SG_NT) void k_seg_sort(const uint32_t* __restrict__ in,
                                                    uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ tmp,
                                                    const int64_t* __restrict__ off, uint64_t S,
                                                    int64_t total, const uint32_t* __restrict__ order,
                                                    uint32_t* __restrict__ qctr, SegTable table,
                                                    uint32_t* __restrict__ status, bool shared) {
    __shared__ __align__(16) unsigned char smem[SMEM];
    __shared__ uint32_t s_item;
    while (true) {
        __syncthreads();  // the previous segment is done with LDS
        if (threadIdx.x == 0) s_item = atomicAdd(qctr, 1u);
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= S) break;  // the queue is finite: every workgroup leaves
        const uint32_t seg = order[item];
        const int64_t b = off[seg], e = off[seg + 1];
        if (b < 0 || e <= b || e > total) continue;  // empty (or reported invalid)
        const uint64_t L = (uint64_t)(e - b);
        if (L > 0xFFFFFFFFull) {
            if (threadIdx.x == 0) atomicOr(status, STATUS_RANGE);
            continue;
        }
        if (shared && seg_shared_len(L)) continue;  // sorted by the shared onesweep rounds
        if (L == 1) {
            if (threadIdx.x == 0) out[b] = in[b];
            continue;
        }
        if (L <= SEG_SMALL_MAX) {
            const int c = len_class((int64_t)L);
            seg_small(in + b, out + b, (uint32_t)L, table.algo[c], table.p[c], smem);
        } else {
            const int c = len_class((int64_t)L);
            if (table.seg_items[c] == 8)
                seg_large<8>(in + b, out + b, tmp + b, L, smem, status);
            else
                seg_large<16>(in + b, out + b, tmp + b, L, smem, status);
        }
    }
}

}  // namespace

// ---- host side -------------------------------------------------------------------

bool seg_plan(uint64_t S, int64_t total, SegPlan* p, bool shared) {
    if (total < 0 || S > 0x7FFFFFFFull) return false;
    SegPlan q;
    size_t off = 0;
    q.off_status = off;
    off += ALIGN;
    q.off_cnt = off;
    off += align_up(sizeof(uint32_t) * (2 * NCLASS + 1));
    q.off_osctr = off;  // the four rounds' tile counters (CTR_STRIDE apart: one per XCD)
    off += align_up(sizeof(uint32_t) * 4 * CTR_STRIDE);
    q.zero_bytes = off - q.off_status;
    q.off_order = off;
    off += align_up(sizeof(uint32_t) * (S ? S : 1));
    q.off_tmp = off;
    off += align_up(sizeof(uint32_t) * (size_t)(total ? total : 1));
    // the large segments' onesweep rounds: at most nl = min(S, total /
    // SEG_OS_MIN) such segments, so at most total / T + nl tiles (a
    // segment's last tile is partial) and tiles / 16 + nl look-back blocks
    q.shared = shared;
    if (shared && (uint64_t)total >= SEG_OS_MIN) {
        const uint64_t nl = (uint64_t)total / SEG_OS_MIN < S ? (uint64_t)total / SEG_OS_MIN : S;
        const uint64_t mt = (uint64_t)total / SEG_OS_TILE + nl;
        if (mt >= (1ull << 31)) return false;
        q.max_tiles = mt;
        q.max_blocks = mt / 16 + nl;
        q.max_large = nl;
        q.off_bbase = off;
        off += align_up(sizeof(uint32_t) * (size_t)(S + 1));
        q.off_ttile = off;
        off += align_up(sizeof(uint32_t) * (size_t)(S + 1));
        q.off_lrank = off;
        off += align_up(sizeof(uint32_t) * (size_t)(S + 1));
        q.off_tdesc = off;
        off += align_up(sizeof(SegTile) * (size_t)mt);
        q.off_shist = off;
        off += align_up(sizeof(uint32_t) * 1024 * (size_t)(nl ? nl : 1));
        q.off_oslb = off;  // per round: the tiles' words, then the blocks' sums
        off += align_up(sizeof(uint32_t) * 256 * 4 * (size_t)(mt + q.max_blocks));
    }
    q.total = off;
    *p = q;
    return true;
}

static int g_seg_grid = 0;

rs_status seg_run(const SegPlan& p, const uint32_t* in, uint32_t* out, const int64_t* offsets,
                  uint64_t S, int64_t total, const SegTable& table, void* ws_, hipStream_t st) {
    if (S == 0) return RS_OK;
    unsigned char* ws = static_cast<unsigned char*>(ws_);
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + p.off_status);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + p.off_cnt);
    uint32_t* cursor = cnt + NCLASS;
    uint32_t* qctr = cursor + NCLASS;
    uint32_t* order = reinterpret_cast<uint32_t*>(ws + p.off_order);
    uint32_t* tmp = reinterpret_cast<uint32_t*>(ws + p.off_tmp);
    rs_status rc = fill_u32(ws + p.off_status, p.zero_bytes / 4, 0u, st);
    if (rc != RS_OK) return rc;
    unsigned g = (unsigned)((S + 255) / 256);
    if (g > 4096) g = 4096;
    prof(st, KID_SEG_PLAN, 0);
    hipLaunchKernelGGL(k_seg_classify, dim3(g), dim3(256), 0, st, offsets, S, total, cnt, status);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(64), 0, st, cnt, cursor);
    hipLaunchKernelGGL(k_seg_scatter, dim3(g), dim3(256), 0, st, offsets, S, total, cursor, order);
    prof(st, KID_SEG_PLAN, 1);
    if ((rc = launch_status()) != RS_OK) return rc;
    if (g_seg_grid == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_seg_sort, SG_NT, 0) != hipSuccess)
            return hip_fail(hipGetLastError());
        g_seg_grid = cus * (per > 0 ? per : 1);
    }
    uint64_t grid = (uint64_t)g_seg_grid;
    if (grid > S) grid = S;
    prof(st, KID_SEG, 0);
    hipLaunchKernelGGL(k_seg_sort, dim3((unsigned)grid), dim3(SG_NT), 0, st, in, out, tmp, offsets, S,
                       total, order, qctr, table, status, p.shared);
    prof(st, KID_SEG, 1);
    if ((rc = launch_status()) != RS_OK) return rc;
    if (!p.shared) return RS_OK;
    return segos_run(p, in, out, tmp, offsets, S, total, ws, st);
}

}  // namespace rs
