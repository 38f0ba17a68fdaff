// rs_small_dev.h -- one workgroup sorts one small array held on chip
// (device functions shared by the batch kernels and the segmented kernel).
//
// BTN and OET are the paper's block networks (Section 2, the BTN and OET
// paragraphs; Section 3, Eq. Tb and Eq. To): p "processors" each own a run
// of N keys, every run is sorted first, then a network of merge-splits runs
// over the p runs -- Batcher's bitonic sorter on p wires in
// lg p (lg p + 1)/2 stages (BTN), or p rounds of odd-even transposition
// between neighbours (OET).  Here a processor is a GPU thread and its run
// lives in its registers:
//
//   * the array is padded to n_pad = next power of two >= n with the
//     largest key and split into p runs of N = n_pad / p keys (p and N
//     powers of two, N <= 64); keys are dealt to runs round-robin so the
//     loads coalesce (the output of a sort does not depend on which keys
//     start in which run);
//   * each run is sorted by a bitonic network on registers (the paper sorts
//     runs with its serial radix sort; any correct local sort gives the
//     same runs);
//   * a merge-split of runs A and B (both ascending) keeps
//     min(A[i], B[N-1-i]) (the N smallest keys) or max(...) (the N
//     largest), a bitonic sequence, and sorts it with a bitonic merge in
//     registers -- the bitonic-merge identity replaces a serial merge, so
//     every step is data-independent;
//   * the partner's run comes from a lane of the same wavefront through a
//     cross-lane permute (no barrier), or through LDS with a barrier when
//     the partner is in another wavefront.
//
// LDS radix: the radix-2^8 count-sort rounds of Section 3 done entirely in
// one workgroup's LDS, with the stable LDS-match ranking of the device-wide
// rounds.
//
// Every function here must be called by all threads of the workgroup
// (they contain barriers); threads at or beyond p hold padding only.
#pragma once
#include "rs_dev.h"

namespace rs {

// ---- register networks ------------------------------------------------------

template <typename K>
__device__ __forceinline__ void cx(K& a, K& b) {  // a <= b afterwards
    const K lo = a < b ? a : b;
    const K hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// Bitonic sorting network on N registers, ascending.
template <int N, typename K>
__device__ __forceinline__ void reg_sort(K (&a)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0) cx(a[i], a[l]);
                    else cx(a[l], a[i]);
                }
            }
        }
    }
}

// Sorts a bitonic sequence of N registers ascending (half-cleaner cascade).
template <int N, typename K>
__device__ __forceinline__ void reg_bitonic_merge(K (&a)[N]) {
#pragma unroll
    for (int j = N >> 1; j >= 1; j >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int l = i ^ j;
            if (l > i) cx(a[i], a[l]);
        }
    }
}

// Merge-split with the partner's run `b` given reversed (b[i] = B[N-1-i]):
// keep the N smallest (low) or the N largest keys, sorted ascending.
template <int N, typename K>
__device__ __forceinline__ void merge_split_rev(K (&a)[N], const K (&b)[N], bool low) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const K x = a[i], y = b[i];
        a[i] = low ? (x < y ? x : y) : (x < y ? y : x);
    }
    reg_bitonic_merge<N>(a);
}

__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int j) {
    return (uint32_t)__shfl_xor((int)v, j, WAVE);
}
__device__ __forceinline__ uint32_t lane_from(uint32_t v, int src) {
    return (uint32_t)__shfl((int)v, src, WAVE);
}

// v of lane (lane ^ J), J known at compile time: DPP quad permutations for
// J = 1, 2 (no LDS traffic), a swizzle within 32 lanes for J = 4..16, the
// LDS permute for J = 32.
template <int J>
__device__ __forceinline__ uint32_t lane_xor_c(uint32_t v) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm 1,0,3,2
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    } else if constexpr (J < 32) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);   // xor J, 32-lane groups
    } else {
        return lane_xor(v, J);
    }
}

// Partner's run, reversed, from lane (lane ^ J) of this wave.
template <int N, int J>
__device__ __forceinline__ void fetch_rev_xor_c(const uint32_t (&a)[N], uint32_t (&b)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = lane_xor_c<J>(a[N - 1 - i]);
}

// Partner's run, reversed, from a lane of this wave (j < 64, uniform).
template <int N>
__device__ __forceinline__ void fetch_rev_xor(const uint32_t (&a)[N], uint32_t (&b)[N], int j) {
    switch (j) {
        case 1: fetch_rev_xor_c<N, 1>(a, b); break;
        case 2: fetch_rev_xor_c<N, 2>(a, b); break;
        case 4: fetch_rev_xor_c<N, 4>(a, b); break;
        case 8: fetch_rev_xor_c<N, 8>(a, b); break;
        case 16: fetch_rev_xor_c<N, 16>(a, b); break;
        default: fetch_rev_xor_c<N, 32>(a, b); break;
    }
}

// Padded blocked layout of the runs in LDS: run t starts at t*(N+1), so that
// lanes touching element i of consecutive runs hit different banks.
template <int N>
__device__ __forceinline__ void runs_to_lds(uint32_t* sh, int t, const uint32_t (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[t * (N + 1) + i] = a[i];
}
template <int N>
__device__ __forceinline__ void rev_from_lds(const uint32_t* sh, int l, uint32_t (&b)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = sh[l * (N + 1) + N - 1 - i];
}

// Deal the instance's keys round-robin into runs; pad with the largest key.
template <int N>
__device__ __forceinline__ void load_runs(const uint32_t* __restrict__ src, uint32_t n, int p, int t,
                                          bool active, uint32_t (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t q = (uint32_t)i * (uint32_t)p + (uint32_t)t;
        a[i] = (active && q < n) ? src[q] : 0xFFFFFFFFu;
    }
}

// Run t is block t of the sorted output; stage through LDS so that the
// global writes coalesce.
template <int N>
__device__ __forceinline__ void store_runs(uint32_t* sh, uint32_t* __restrict__ dst, uint32_t n, int p,
                                           int t, bool active, const uint32_t (&a)[N]) {
    __syncthreads();
    if (active) runs_to_lds<N>(sh, t, a);
    __syncthreads();
    const uint32_t npad = (uint32_t)p * N;
    for (uint32_t q = threadIdx.x; q < npad && q < n; q += blockDim.x) dst[q] = sh[q + q / N];
}

// BTN on p runs of N keys; sh holds p*(N+1) words.  Requires p <= blockDim.x.
template <int N>
__device__ __forceinline__ void btn_sort(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                         uint32_t n, int p, uint32_t* sh) {
    const int t = threadIdx.x;
    const bool active = t < p;
    uint32_t a[N], b[N];
    load_runs<N>(src, n, p, t, active, a);
    reg_sort<N>(a);
    // Batcher's network on p wires: wire t meets t^j; the pair ascends when
    // bit k of t is clear; t keeps the smaller half when it is the lower
    // wire of an ascending pair or the upper wire of a descending one.
    for (int k = 2; k <= p; k <<= 1) {
        for (int j = k >> 1; j >= 1; j >>= 1) {
            const bool asc = (t & k) == 0;
            const bool low = ((t & j) == 0) == asc;
            if (j < WAVE) {
                fetch_rev_xor<N>(a, b, j);   // every lane takes part
            } else {
                __syncthreads();
                if (active) runs_to_lds<N>(sh, t, a);
                __syncthreads();
                if (active) rev_from_lds<N>(sh, t ^ j, b);
            }
            if (active) merge_split_rev<N>(a, b, low);
        }
    }
    store_runs<N>(sh, dst, n, p, t, active, a);
}

// OET on p runs of N keys; sh holds p*(N+1) words.  Requires p <= blockDim.x.
template <int N>
__device__ __forceinline__ void oet_sort(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                         uint32_t n, int p, uint32_t* sh) {
    const int t = threadIdx.x;
    const bool active = t < p;
    const int lane = t & (WAVE - 1);
    uint32_t a[N], b[N];
    load_runs<N>(src, n, p, t, active, a);
    reg_sort<N>(a);
    const bool multiwave = p > WAVE;
    // p rounds; round r pairs (i, i+1) with i = r (mod 2); the lower run
    // keeps the smaller half.
    for (int r = 0; r < p; ++r) {
        const bool even = (r & 1) == 0;
        // partner: even rounds t^1; odd rounds t+1 for odd t, t-1 for even t
        const int partner = even ? (t ^ 1) : ((t & 1) ? t + 1 : t - 1);
        const bool has = active && partner >= 0 && partner < p;
        const int src_lane = even ? (lane ^ 1) : (((lane & 1) ? lane + 1 : lane - 1) & (WAVE - 1));
        if (even) {
#pragma unroll
            for (int i = 0; i < N; ++i) b[i] = lane_xor_c<1>(a[N - 1 - i]);
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) b[i] = lane_from(a[N - 1 - i], src_lane);
        }
        if (!even && multiwave) {
            // odd rounds: lanes 63 and 0 pair with the neighbouring wave
            __syncthreads();
            if (active && (lane == 0 || lane == WAVE - 1)) runs_to_lds<N>(sh, t, a);
            __syncthreads();
            if (has && (lane == 0 || lane == WAVE - 1)) rev_from_lds<N>(sh, partner, b);
        }
        if (has) merge_split_rev<N>(a, b, t < partner);
    }
    store_runs<N>(sh, dst, n, p, t, active, a);
}

// Stable radix-2^8 rounds in LDS over n <= NT*ITEMS keys; blockDim.x == NT.
//   wmask: NW*256 u64, wcnt: NW*256 u16, loc: 256 u32, wsum: NW+1 u32,
//   sk: NT*ITEMS u32 (may alias wmask: the masks are re-zeroed every round).
template <int ITEMS, int NT>
__device__ __forceinline__ void lds_radix_sort(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                               uint32_t n, uint64_t* wmask, uint16_t* wcnt,
                                               uint32_t* loc, uint32_t* wsum, uint32_t* sk) {
    constexpr int NW = NT / WAVE;
    constexpr int R = 256;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wb = wave * (ITEMS * WAVE) + lane;
    uint32_t k[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = wb + i * WAVE;
        k[i] = j < n ? src[j] : 0xFFFFFFFFu;   // pads sort last and stay last
    }
    const uint64_t mybit = 1ull << lane;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = pass * 8;
        __syncthreads();  // previous round's reads of sk are done
        for (int i = tid; i < NW * R; i += NT) {
            wcnt[i] = 0;
            wmask[i] = 0;
        }
        __syncthreads();
        uint32_t dr[ITEMS];
        uint16_t* wc = wcnt + wave * R;
        uint64_t* wm = wmask + wave * R;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = (k[i] >> shift) & 255u;
            atomicOr((unsigned long long*)&wm[d], (unsigned long long)mybit);
            const uint64_t m = __hip_atomic_load(&wm[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const uint32_t lt = mbcnt(m);
            const uint32_t cnt = (uint32_t)__popcll(m);
            const uint32_t c = wc[d];
            if (lt + 1 == cnt) {
                wc[d] = (uint16_t)(c + cnt);
                __hip_atomic_store(&wm[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            dr[i] = d | ((c + lt) << 16);
        }
        __syncthreads();
        uint32_t tot = 0;
        if (tid < (uint32_t)R) {
            uint32_t s = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = wcnt[w * R + tid];
                wcnt[w * R + tid] = (uint16_t)s;
                s += c;
            }
            tot = s;
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<NT>(tot, wsum, &total);
        if (tid < (uint32_t)R) loc[tid] = ex;
        __syncthreads();
        uint32_t slot[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = dr[i] & 0xFFFFu;
            slot[i] = loc[d] + wcnt[wave * R + d] + (dr[i] >> 16);
        }
        __syncthreads();  // sk may alias the masks
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) sk[slot[i]] = k[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) k[i] = sk[wb + i * WAVE];
    }
    for (uint32_t q = tid; q < n; q += NT) dst[q] = sk[q];
}

}  // namespace rs
