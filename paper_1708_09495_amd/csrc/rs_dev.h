// rs_dev.h -- device helpers shared by the librs kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int WAVE = 64;

template <typename T> struct KeyMax;
template <> struct KeyMax<uint16_t> { static constexpr uint16_t v = 0xFFFFu; };
template <> struct KeyMax<uint32_t> { static constexpr uint32_t v = 0xFFFFFFFFu; };
template <> struct KeyMax<uint64_t> { static constexpr uint64_t v = ~0ull; };

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of m below this lane (v_mbcnt_lo / v_mbcnt_hi).
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Mask of the lanes of this wave whose `bits`-bit digit equals this lane's
// (the wave64 form of a match-any): one ballot per digit bit.  Must be
// called with every lane of the wave active.
template <int MAXBITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits) {
    uint64_t m = ~0ull;
#pragma unroll
    for (int k = 0; k < MAXBITS; ++k) {
        if (k < bits) {
            const bool b = (d >> k) & 1u;
            const uint64_t v = ballot(b);
            m &= b ? v : ~v;
        }
    }
    return m;
}

// Wave-level inclusive scan of a 32-bit value (Hillis-Steele over 64 lanes).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o, WAVE);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; NT threads, `wsum` is
// NT/64 words of LDS.  Returns the exclusive prefix; *total gets the sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
    constexpr int NW = NT / WAVE;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = lane < (uint32_t)NW ? wsum[lane] : 0u;
        uint32_t xi = wave_incl_scan(x);
        if (lane < (uint32_t)NW) wsum[lane] = xi - x;
        if (lane == NW - 1) wsum[NW] = xi;
    }
    __syncthreads();
    uint32_t r = inc - v + wsum[w];
    *total = wsum[NW];
    __syncthreads();
    return r;
}

// Relaxed atomics at agent scope: coherent across the XCDs' L2 caches.
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace rs
