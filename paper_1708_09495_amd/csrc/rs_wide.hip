// rs_wide.hip -- count-sort rounds with wide digits (12..16 bits).
//
// The paper's PR2 sorts 32-bit keys in two rounds of radix 2^16 and prices
// the exchange of the p per-processor count arrays at 2prg (Section 3, the
// communication term of the round cost), the term that grows with r.  On the
// GPU that term is the count table: one row of 2^b counters per tile, far too
// large to publish through a look-back per tile, so a wide round is
// reduce-then-scan in four launches:
//
//   k_wide_count   each workgroup counts its tile's digits in LDS (one or
//                  two halves of the digit range) and writes its row;
//   k_wide_cols    every digit's column of the table scanned over the tiles
//                  (exclusive), and the digit's total;
//   k_wide_base    exclusive scan of the totals: each digit's first slot;
//   k_wide_scatter each workgroup walks its tile in sub-tiles, in order:
//                  sorts the sub-tile stably by the b-bit digit in LDS (two
//                  stable 8-bit rounds), then writes every run of equal
//                  digits at the tile's cursor for that digit and advances
//                  the cursor (its row of the table, owned by the workgroup).
//
// With 2^16 digits a 4096-key sub-tile holds ~0.06 keys per digit, so the
// writes land key by key: the locality the wide radix gives up for its
// halved round count.
#include "rs_dev.h"
#include "rs_internal.hpp"

namespace rs {
namespace {

constexpr int WC_NT = 1024;               // count kernel threads
constexpr uint32_t WC_HALF = 1u << 15;    // LDS counters per half (128 KiB)
constexpr int WT_NT = 512;                // scatter kernel threads
constexpr int WT_NW = WT_NT / WAVE;
constexpr int WT_ITEMS = 8;
constexpr uint32_t WT_SUB = WT_NT * WT_ITEMS;  // keys per sub-tile (4096)
constexpr uint32_t WIDE_MAX_TILES = 512;
constexpr int WIDE_PREFETCH_BITS = 14;

template <typename K>
__global__ __launch_bounds__(WC_NT) void k_wide_count(const K* __restrict__ keys, uint64_t n, int shift,
                                                      int bits, uint64_t tile_keys,
                                                      uint32_t* __restrict__ table) {
    __shared__ uint32_t cnt[WC_HALF];
    const uint32_t t = blockIdx.x;
    const uint32_t R = 1u << bits;
    const uint32_t mask = R - 1;
    const uint64_t b0 = (uint64_t)t * tile_keys;
    const uint64_t e0 = b0 + tile_keys < n ? b0 + tile_keys : n;
    const uint32_t halves = R > WC_HALF ? 2u : 1u;
    const uint32_t span = R > WC_HALF ? WC_HALF : R;
    for (uint32_t h = 0; h < halves; ++h) {
        for (uint32_t i = threadIdx.x; i < span; i += WC_NT) cnt[i] = 0;
        __syncthreads();
        const uint32_t lo = h * span;
        for (uint64_t i = b0 + threadIdx.x; i < e0; i += WC_NT) {
            const uint32_t d = ((uint32_t)(keys[i] >> shift) & mask) - lo;
            if (d < span) atomicAdd(&cnt[d], 1u);
        }
        __syncthreads();
        uint32_t* row = table + (size_t)t * R + lo;
        for (uint32_t i = threadIdx.x; i < span; i += WC_NT) row[i] = cnt[i];
        __syncthreads();
    }
}

// One thread per digit: exclusive scan of its column over the tiles.
__global__ __launch_bounds__(256) void k_wide_cols(uint32_t* __restrict__ table, uint32_t tiles, uint32_t R,
                                                   uint32_t* __restrict__ totals) {
    const uint32_t d = blockIdx.x * 256 + threadIdx.x;
    if (d >= R) return;
    uint32_t s = 0;
    uint32_t t = 0;
    for (; t + 8 <= tiles; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = table[(size_t)(t + q) * R + d];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            table[(size_t)(t + q) * R + d] = s;
            s += v[q];
        }
    }
    for (; t < tiles; ++t) {
        const uint32_t v = table[(size_t)t * R + d];
        table[(size_t)t * R + d] = s;
        s += v;
    }
    totals[d] = s;
}

// Exclusive scan of the R digit totals in place (one workgroup).
__global__ __launch_bounds__(1024) void k_wide_base(uint32_t* __restrict__ totals, uint32_t R) {
    __shared__ uint32_t wsum[1024 / WAVE + 1];
    const uint32_t per = (R + 1023) / 1024;
    const uint32_t t = threadIdx.x;
    uint32_t s = 0;
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t d = t * per + q;
        s += d < R ? totals[d] : 0u;
    }
    uint32_t total;
    uint32_t ex = block_excl_scan<1024>(s, wsum, &total);
    for (uint32_t q = 0; q < per; ++q) {
        const uint32_t d = t * per + q;
        if (d < R) {
            const uint32_t v = totals[d];
            totals[d] = ex;
            ex += v;
        }
    }
}

// Block-wide exclusive max-scan (identity 0) of one value per thread.
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* wmax) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, WAVE);
        if (lane >= (uint32_t)o) inc = inc > u ? inc : u;
    }
    if (lane == 63) wmax[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < w; ++q) before = before > wmax[q] ? before : wmax[q];
    uint32_t ex = __shfl_up(inc, 1, WAVE);
    if (lane == 0) ex = 0;
    __syncthreads();
    return ex > before ? ex : before;
}

// PF: the next sub-tile's keys are loaded while the current one is written
// (pays where the writes are most scattered, b >= WIDE_PREFETCH_BITS)
template <typename K, int VB, bool PF>
__global__ __launch_bounds__(WT_NT) void k_wide_scatter(const K* __restrict__ kin, K* __restrict__ kout,
                                                        const void* __restrict__ vin_, void* __restrict__ vout_,
                                                        uint64_t n, int shift, int bits, uint64_t tile_keys,
                                                        uint32_t* __restrict__ table,
                                                        const uint32_t* __restrict__ base,
                                                        uint32_t* __restrict__ status) {
    using V = typename std::conditional<VB == 8, uint64_t, uint32_t>::type;
    constexpr int R8 = 256;
    __shared__ __align__(16) uint64_t wmask[WT_NW * R8];
    __shared__ uint16_t wcnt[WT_NW * R8];
    __shared__ uint32_t loc[R8];
    __shared__ uint32_t wsum[WT_NW + 1];
    __shared__ K sk[WT_SUB];
    __shared__ uint16_t sidx[WT_SUB];
    __shared__ uint32_t runbase[WT_SUB];
    const V* vin = reinterpret_cast<const V*>(vin_);
    V* vout = reinterpret_cast<V*>(vout_);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t t = blockIdx.x;
    const uint32_t R = 1u << bits;
    const uint32_t mask = R - 1;
    uint32_t* cur = table + (size_t)t * R;  // this tile's cursors, owned by this workgroup
    const uint64_t b0 = (uint64_t)t * tile_keys;
    const uint64_t e0 = b0 + tile_keys < n ? b0 + tile_keys : n;
    for (int i = tid; i < WT_NW * R8; i += WT_NT) wmask[i] = 0;
    const uint64_t mybit = 1ull << lane;
    const uint32_t wb = wave * (WT_ITEMS * WAVE) + lane;
    uint16_t* wc = wcnt + wave * R8;
    uint64_t* wm = wmask + wave * R8;
    // keys of the sub-tile at s (past the tile's end: the largest key)
    K kn[WT_ITEMS];
    auto load_sub = [&](uint64_t s) {
        const uint32_t nv = s < e0 ? ((e0 - s) < (uint64_t)WT_SUB ? (uint32_t)(e0 - s) : WT_SUB) : 0u;
#pragma unroll
        for (int i = 0; i < WT_ITEMS; ++i) {
            const uint32_t j = wb + i * WAVE;
            kn[i] = j < nv ? kin[s + j] : KeyMax<K>::v;
        }
    };
    if constexpr (PF) load_sub(b0);
    for (uint64_t s0 = b0; s0 < e0; s0 += WT_SUB) {
        const uint32_t nvalid = (e0 - s0) < (uint64_t)WT_SUB ? (uint32_t)(e0 - s0) : WT_SUB;
        if constexpr (!PF) load_sub(s0);
        K k[WT_ITEMS];
        uint32_t ix[WT_ITEMS];
#pragma unroll
        for (int i = 0; i < WT_ITEMS; ++i) {
            k[i] = kn[i];
            ix[i] = wb + i * WAVE;
        }
        // two stable 8-bit LDS rounds order the sub-tile by its b-bit digit;
        // padding takes the largest digit and, coming last, stays last
#pragma unroll 1
        for (int sub = 0; sub < 2; ++sub) {
            __syncthreads();
            for (int i = tid; i < WT_NW * R8; i += WT_NT) wcnt[i] = 0;
            __syncthreads();
            uint32_t dr[WT_ITEMS];
#pragma unroll
            for (int i = 0; i < WT_ITEMS; ++i) {
                const uint32_t dig = ix[i] >= nvalid ? mask : ((uint32_t)(k[i] >> shift) & mask);
                const uint32_t d = (dig >> (8 * sub)) & 255u;
                atomicOr((unsigned long long*)&wm[d], (unsigned long long)mybit);
                const uint64_t m = __hip_atomic_load(&wm[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const uint32_t lt = mbcnt(m);
                const uint32_t c = wc[d];
                if (lt + 1 == (uint32_t)__popcll(m)) {
                    wc[d] = (uint16_t)(c + lt + 1);
                    __hip_atomic_store(&wm[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                dr[i] = d | ((c + lt) << 16);
            }
            __syncthreads();
            uint32_t tot = 0;
            if (tid < (uint32_t)R8) {
                uint32_t s = 0;
#pragma unroll
                for (int w = 0; w < WT_NW; ++w) {
                    const uint32_t c = wcnt[w * R8 + tid];
                    wcnt[w * R8 + tid] = (uint16_t)s;
                    s += c;
                }
                tot = s;
            }
            uint32_t total;
            const uint32_t ex = block_excl_scan<WT_NT>(tot, wsum, &total);
            if (tid < (uint32_t)R8) loc[tid] = ex;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < WT_ITEMS; ++i) {
                const uint32_t d = dr[i] & 0xFFFFu;
                const uint32_t slot = loc[d] + wc[d] + (dr[i] >> 16);
                sk[slot] = k[i];
                sidx[slot] = (uint16_t)ix[i];
            }
            __syncthreads();
            if (sub == 0) {
#pragma unroll
                for (int i = 0; i < WT_ITEMS; ++i) {
                    k[i] = sk[wb + i * WAVE];
                    ix[i] = sidx[wb + i * WAVE];
                }
            }
        }
        if constexpr (PF) load_sub(s0 + WT_SUB);
        // runs of equal digits among the nvalid sorted keys: thread tid owns
        // positions [tid*ITEMS, tid*ITEMS + ITEMS); a key's run head is the
        // last head position at or before it
        const uint32_t j0 = tid * WT_ITEMS;
        uint32_t dg[WT_ITEMS];
        uint32_t last_head = 0;
#pragma unroll
        for (int q = 0; q < WT_ITEMS; ++q) {
            const uint32_t j = j0 + q;
            dg[q] = j < nvalid ? ((uint32_t)(sk[j] >> shift) & mask) : R;
            const uint32_t prev = j == 0 ? R + 1 : (q ? dg[q - 1] : ((uint32_t)(sk[j - 1] >> shift) & mask));
            if (j < nvalid && dg[q] != prev) last_head = j;
        }
        const uint32_t head_in = block_excl_max(last_head, wsum);
        uint32_t h = head_in;
        // Run tails take their digit's cursor and advance it.  The sub-tile
        // is sorted by digit, so each digit has one run here and the tails'
        // cursors are distinct: every load is issued before any store.
        uint32_t hq[WT_ITEMS], c0[WT_ITEMS], bq[WT_ITEMS];
        uint32_t tails = 0;
#pragma unroll
        for (int q = 0; q < WT_ITEMS; ++q) {
            const uint32_t j = j0 + q;
            if (j < nvalid) {
                const uint32_t prev =
                    j == 0 ? R + 1 : (q ? dg[q - 1] : ((uint32_t)(sk[j - 1] >> shift) & mask));
                if (dg[q] != prev) h = j;
                const uint32_t next = q + 1 < WT_ITEMS ? dg[q + 1]
                                      : (j + 1 < nvalid ? ((uint32_t)(sk[j + 1] >> shift) & mask) : R);
                if (dg[q] != next) tails |= 1u << q;
            }
            hq[q] = h;
        }
#pragma unroll
        for (int q = 0; q < WT_ITEMS; ++q) {
            if (tails & (1u << q)) {
                c0[q] = cur[dg[q]];
                bq[q] = base[dg[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < WT_ITEMS; ++q) {
            if (tails & (1u << q)) {
                cur[dg[q]] = c0[q] + (j0 + q - hq[q] + 1);
                runbase[hq[q]] = bq[q] + c0[q];
            }
        }
        __syncthreads();
        h = head_in;
#pragma unroll
        for (int q = 0; q < WT_ITEMS; ++q) {
            const uint32_t j = j0 + q;
            if (j < nvalid) {
                const uint32_t prev =
                    j == 0 ? R + 1 : (q ? dg[q - 1] : ((uint32_t)(sk[j - 1] >> shift) & mask));
                if (dg[q] != prev) h = j;
                const uint64_t o = (uint64_t)runbase[h] + (j - h);
                if (o < n) {
                    kout[o] = sk[j];
                    if constexpr (VB != 0) vout[o] = vin[s0 + sidx[j]];
                } else {
                    atomicOr(status, STATUS_RANGE);
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

bool wide_plan(size_t n, int kb, int vb, int bits, WidePlan* p) {
    if ((kb != 4 && kb != 8) || (vb != 0 && vb != 4 && vb != 8) || bits < 12 || bits > 16) return false;
    if ((uint64_t)n >= (1ull << 32)) return false;  // 32-bit counts and cursors
    WidePlan q;
    q.n = n;
    q.kb = kb;
    q.vb = vb;
    q.bits = bits;
    q.R = 1u << bits;
    q.passes = (8 * kb + bits - 1) / bits;
    // whole sub-tiles per tile and at most WIDE_MAX_TILES tiles: the table
    // holds tiles * 2^b counters
    const uint64_t subs = (n + WT_SUB - 1) / WT_SUB;
    const uint64_t per = (subs + WIDE_MAX_TILES - 1) / WIDE_MAX_TILES;
    q.tile_keys = (per ? per : 1) * WT_SUB;
    q.tiles = (uint32_t)((n + q.tile_keys - 1) / q.tile_keys);
    size_t off = 0;
    q.off_status = off;
    off += ALIGN;
    q.off_table = off;
    off += align_up((size_t)4 * q.R * (q.tiles ? q.tiles : 1));
    q.off_base = off;
    off += align_up((size_t)4 * q.R);
    q.off_tk = off;
    off += align_up((size_t)kb * n);
    q.off_tv = off;
    off += align_up((size_t)vb * n);
    q.total = off;
    *p = q;
    return true;
}

template <typename K, int VB>
static rs_status wide_pass(const WidePlan& p, const void* src, void* dst, const void* vsrc, void* vdst, int pass,
                           unsigned char* ws, hipStream_t st) {
    uint32_t* table = reinterpret_cast<uint32_t*>(ws + p.off_table);
    uint32_t* base = reinterpret_cast<uint32_t*>(ws + p.off_base);
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + p.off_status);
    const int shift = pass * p.bits;
    prof(st, KID_WIDE_COUNT, 0);
    hipLaunchKernelGGL(k_wide_count<K>, dim3(p.tiles), dim3(WC_NT), 0, st, (const K*)src, (uint64_t)p.n, shift,
                       p.bits, (uint64_t)p.tile_keys, table);
    hipLaunchKernelGGL(k_wide_cols, dim3((p.R + 255) / 256), dim3(256), 0, st, table, p.tiles, p.R, base);
    hipLaunchKernelGGL(k_wide_base, dim3(1), dim3(1024), 0, st, base, p.R);
    prof(st, KID_WIDE_COUNT, 1);
    rs_status rc = launch_status();
    if (rc != RS_OK) return rc;
    prof(st, KID_WIDE_SCATTER, 0);
    if (p.bits >= WIDE_PREFETCH_BITS)
        hipLaunchKernelGGL((k_wide_scatter<K, VB, true>), dim3(p.tiles), dim3(WT_NT), 0, st, (const K*)src,
                           (K*)dst, vsrc, vdst, (uint64_t)p.n, shift, p.bits, (uint64_t)p.tile_keys, table, base,
                           status);
    else
        hipLaunchKernelGGL((k_wide_scatter<K, VB, false>), dim3(p.tiles), dim3(WT_NT), 0, st, (const K*)src,
                           (K*)dst, vsrc, vdst, (uint64_t)p.n, shift, p.bits, (uint64_t)p.tile_keys, table, base,
                           status);
    prof(st, KID_WIDE_SCATTER, 1);
    return launch_status();
}

static rs_status wide_pass_any(const WidePlan& p, const void* src, void* dst, const void* vsrc, void* vdst,
                               int pass, unsigned char* ws, hipStream_t st) {
    if (p.kb == 4) {
        if (p.vb == 0) return wide_pass<uint32_t, 0>(p, src, dst, vsrc, vdst, pass, ws, st);
        if (p.vb == 4) return wide_pass<uint32_t, 4>(p, src, dst, vsrc, vdst, pass, ws, st);
        return wide_pass<uint32_t, 8>(p, src, dst, vsrc, vdst, pass, ws, st);
    }
    if (p.vb == 0) return wide_pass<uint64_t, 0>(p, src, dst, vsrc, vdst, pass, ws, st);
    if (p.vb == 4) return wide_pass<uint64_t, 4>(p, src, dst, vsrc, vdst, pass, ws, st);
    return wide_pass<uint64_t, 8>(p, src, dst, vsrc, vdst, pass, ws, st);
}

rs_status wide_run(const WidePlan& p, const void* kin, void* kout, const void* vin, void* vout, void* ws_,
                   hipStream_t st) {
    if (p.n == 0) return RS_OK;
    unsigned char* ws = static_cast<unsigned char*>(ws_);
    rs_status rc = fill_u32(ws + p.off_status, ALIGN / 4, 0u, st);
    if (rc != RS_OK) return rc;
    void* tk = ws + p.off_tk;
    void* tv = ws + p.off_tv;
    const int P = p.passes;
    // ping-pong so that the last round writes kout; in place with an odd
    // round count ends in the temporaries and copies back
    const bool copy_back = kin == kout && (P % 2 == 1);
    const void* src = kin;
    const void* vsrc = vin;
    for (int j = 0; j < P; ++j) {
        bool to_out = ((P - 1 - j) % 2 == 0);
        if (copy_back) to_out = !to_out;
        void* dst = to_out ? kout : tk;
        void* vdst = to_out ? vout : tv;
        if ((rc = wide_pass_any(p, src, dst, vsrc, vdst, j, ws, st)) != RS_OK) return rc;
        src = dst;
        vsrc = vdst;
    }
    if (copy_back) {
        prof(st, KID_COPY, 0);
        hipError_t e = hipMemcpyAsync(kout, tk, p.n * p.kb, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess && p.vb) e = hipMemcpyAsync(vout, tv, p.n * p.vb, hipMemcpyDeviceToDevice, st);
        prof(st, KID_COPY, 1);
        if (e != hipSuccess) return hip_fail(e);
    }
    return RS_OK;
}

}  // namespace rs
