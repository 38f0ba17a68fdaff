// rs_small.hip -- one workgroup sorts one small array held on chip.
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
// one workgroup's LDS (stable ranking as in the device-wide rounds), the
// radix comparator at the same n.
#include <type_traits>

#include "rs_dev.h"
#include "rs_internal.hpp"

namespace rs {
namespace {

// ---- register networks ----------------------------------------------------

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

// Partner's run, reversed, from a lane of this wave.
template <int N>
__device__ __forceinline__ void fetch_rev_xor(const uint32_t (&a)[N], uint32_t (&b)[N], int j) {
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = lane_xor(a[N - 1 - i], j);
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

// Load instance keys round-robin into runs; pad with the largest key.
template <int N>
__device__ __forceinline__ void load_runs(const uint32_t* __restrict__ src, uint32_t n, int p, int t,
                                          uint32_t (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t q = (uint32_t)i * (uint32_t)p + (uint32_t)t;
        a[i] = q < n ? src[q] : 0xFFFFFFFFu;
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

// ---- BTN --------------------------------------------------------------------

// n_pad <= 16384, so p = n_pad / N threads never exceed 16384 / N.
constexpr int net_threads(int N) { return N >= 64 ? 256 : (N >= 32 ? 512 : 1024); }

template <int N>
__global__ __launch_bounds__(net_threads(N)) void k_btn(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                              uint32_t n, int p) {
    extern __shared__ uint32_t sh[];
    const int t = threadIdx.x;
    const bool active = t < p;
    const size_t off = (size_t)blockIdx.x * n;
    uint32_t a[N], b[N];
    if (active) load_runs<N>(in + off, n, p, t, a);
    else {
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = 0xFFFFFFFFu;
    }
    reg_sort<N>(a);
    // Batcher's network on p wires: wire t meets t^j; the pair ascends when
    // bit k of t is clear; t keeps the smaller half when it is the lower
    // wire of an ascending pair or the upper wire of a descending one.
    for (int k = 2; k <= p; k <<= 1) {
        for (int j = k >> 1; j >= 1; j >>= 1) {
            const bool asc = (t & k) == 0;
            const bool low = ((t & j) == 0) == asc;
            if (j < WAVE) {
                fetch_rev_xor<N>(a, b, j);   // all lanes take part
            } else {
                __syncthreads();
                if (active) runs_to_lds<N>(sh, t, a);
                __syncthreads();
                if (active) rev_from_lds<N>(sh, t ^ j, b);
            }
            if (active) merge_split_rev<N>(a, b, low);
        }
    }
    store_runs<N>(sh, out + off, n, p, t, active, a);
}

// ---- OET --------------------------------------------------------------------

template <int N>
__global__ __launch_bounds__(net_threads(N)) void k_oet(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                              uint32_t n, int p) {
    extern __shared__ uint32_t sh[];
    const int t = threadIdx.x;
    const bool active = t < p;
    const int lane = t & (WAVE - 1);
    const size_t off = (size_t)blockIdx.x * n;
    uint32_t a[N], b[N];
    if (active) load_runs<N>(in + off, n, p, t, a);
    else {
#pragma unroll
        for (int i = 0; i < N; ++i) a[i] = 0xFFFFFFFFu;
    }
    reg_sort<N>(a);
    const bool multiwave = p > WAVE;
    // p rounds; round r pairs (i, i+1) with i = r (mod 2); the lower run
    // keeps the smaller half.
    for (int r = 0; r < p; ++r) {
        const bool even = (r & 1) == 0;
        // partner: even rounds t^1; odd rounds t+1 for odd t, t-1 for even t
        const int partner = even ? (t ^ 1) : ((t & 1) ? t + 1 : t - 1);
        const bool has = active && partner >= 0 && partner < p;
        if (even || !multiwave) {
            // within a wave: lane partner = lane ^ 1 (even) or lane +- 1 (odd)
            const int src = even ? (lane ^ 1) : (((lane & 1) ? lane + 1 : lane - 1) & (WAVE - 1));
#pragma unroll
            for (int i = 0; i < N; ++i) b[i] = lane_from(a[N - 1 - i], src);
        } else {
            // odd rounds across waves: lanes 0 and 63 pair with the
            // neighbouring wave; everyone else stays within the wave
            const int src = ((lane & 1) ? lane + 1 : lane - 1) & (WAVE - 1);
#pragma unroll
            for (int i = 0; i < N; ++i) b[i] = lane_from(a[N - 1 - i], src);
            __syncthreads();
            if (active && (lane == 0 || lane == WAVE - 1)) runs_to_lds<N>(sh, t, a);
            __syncthreads();
            if (has && (lane == 0 || lane == WAVE - 1)) rev_from_lds<N>(sh, partner, b);
        }
        if (has) merge_split_rev<N>(a, b, t < partner);
    }
    store_runs<N>(sh, out + off, n, p, t, active, a);
}

// ---- LDS radix -----------------------------------------------------------------

constexpr int LR_NT = 512;
constexpr int LR_NW = LR_NT / WAVE;

// Stable radix-2^8 rounds in LDS over n <= LR_NT*ITEMS keys (one instance).
template <int ITEMS>
__global__ __launch_bounds__(LR_NT) void k_lds_radix(const uint32_t* __restrict__ in,
                                                     uint32_t* __restrict__ out, uint32_t n) {
    constexpr int T = LR_NT * ITEMS;
    constexpr int R = 256;
    __shared__ uint64_t wmask[LR_NW * R];
    __shared__ uint16_t wcnt[LR_NW * R];
    __shared__ uint32_t loc[R];
    __shared__ uint32_t wsum[LR_NW + 1];
    extern __shared__ uint32_t sk[];  // T keys
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t off = (size_t)blockIdx.x * n;
    const uint32_t wb = wave * (ITEMS * WAVE) + lane;
    uint32_t k[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = wb + i * WAVE;
        k[i] = j < n ? in[off + j] : 0xFFFFFFFFu;   // pads sort last and stay last
    }
    const uint64_t mybit = 1ull << lane;
    for (int i = tid; i < LR_NW * R; i += LR_NT) wmask[i] = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = pass * 8;
        for (int i = tid; i < LR_NW * R; i += LR_NT) wcnt[i] = 0;
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
            for (int w = 0; w < LR_NW; ++w) {
                const uint32_t c = wcnt[w * R + tid];
                wcnt[w * R + tid] = (uint16_t)s;
                s += c;
            }
            tot = s;
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<LR_NT>(tot, wsum, &total);
        if (tid < (uint32_t)R) loc[tid] = ex;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = dr[i] & 0xFFFFu;
            sk[loc[d] + wcnt[wave * R + d] + (dr[i] >> 16)] = k[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) k[i] = sk[wb + i * WAVE];
    }
    for (uint32_t q = tid; q < n; q += LR_NT) out[off + q] = sk[q];
}

}  // namespace

// ---- host side ----------------------------------------------------------------

uint32_t small_npad(uint32_t n) {
    uint32_t m = 1;
    while (m < n) m <<= 1;
    return m;
}

bool small_valid_p(uint32_t n, int p) {
    if (n == 0) return true;
    const uint32_t npad = small_npad(n);
    if (p < 1 || p > 1024 || (p & (p - 1)) || (uint32_t)p > npad) return false;
    return npad / (uint32_t)p <= 64;
}

int small_default_p(int algo, uint32_t n) {
    const uint32_t npad = small_npad(n ? n : 1);
    // BTN: runs of 8 keys (fewer stages than N = 1, cheap register merges);
    // OET: the fewest processors the register runs allow (p rounds).
    uint32_t p = algo == RS_ALGO_OET ? npad / 64 : npad / 8;
    if (p < 1) p = 1;
    if (p > 1024) p = 1024;
    while (npad / p > 64) p <<= 1;
    return (int)p;
}

template <int N>
static hipError_t launch_net(int algo, const uint32_t* in, uint32_t* out, uint32_t n, size_t count, int p,
                             hipStream_t st) {
    const int threads = p < WAVE ? WAVE : p;
    const size_t shm = sizeof(uint32_t) * (size_t)p * (N + 1);
    if (algo == RS_ALGO_BTN)
        hipLaunchKernelGGL(k_btn<N>, dim3((unsigned)count), dim3(threads), shm, st, in, out, n, p);
    else
        hipLaunchKernelGGL(k_oet<N>, dim3((unsigned)count), dim3(threads), shm, st, in, out, n, p);
    return hipGetLastError();
}

template <int ITEMS>
static hipError_t launch_lr(const uint32_t* in, uint32_t* out, uint32_t n, size_t count, hipStream_t st) {
    const size_t shm = sizeof(uint32_t) * (size_t)LR_NT * ITEMS;
    hipLaunchKernelGGL(k_lds_radix<ITEMS>, dim3((unsigned)count), dim3(LR_NT), shm, st, in, out, n);
    return hipGetLastError();
}

rs_status small_run(int algo, const uint32_t* in, uint32_t* out, uint32_t n, size_t count, int p,
                    hipStream_t st) {
    if (n == 0 || count == 0) return RS_OK;
    hipError_t e = hipSuccess;
    prof(st, KID_BATCH, 0);
    if (algo == RS_ALGO_LDS_RADIX) {
        const uint32_t items = (n + LR_NT - 1) / LR_NT;
        if (items <= 1) e = launch_lr<1>(in, out, n, count, st);
        else if (items <= 2) e = launch_lr<2>(in, out, n, count, st);
        else if (items <= 4) e = launch_lr<4>(in, out, n, count, st);
        else if (items <= 8) e = launch_lr<8>(in, out, n, count, st);
        else if (items <= 16) e = launch_lr<16>(in, out, n, count, st);
        else e = launch_lr<32>(in, out, n, count, st);
    } else {
        const uint32_t N = small_npad(n) / (uint32_t)p;
        switch (N) {
            case 1: e = launch_net<1>(algo, in, out, n, count, p, st); break;
            case 2: e = launch_net<2>(algo, in, out, n, count, p, st); break;
            case 4: e = launch_net<4>(algo, in, out, n, count, p, st); break;
            case 8: e = launch_net<8>(algo, in, out, n, count, p, st); break;
            case 16: e = launch_net<16>(algo, in, out, n, count, p, st); break;
            case 32: e = launch_net<32>(algo, in, out, n, count, p, st); break;
            default: e = launch_net<64>(algo, in, out, n, count, p, st); break;
        }
    }
    prof(st, KID_BATCH, 1);
    return e == hipSuccess ? RS_OK : hip_fail(e);
}

}  // namespace rs
