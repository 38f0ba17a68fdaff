// gen_dev.hip -- device twin of the uniform-key generators in gen.c.  The
// same counter-based SplitMix64 stream (Steele, Lea and Flood 2014): element
// i is the i-th output of a generator seeded with `seed`, so host and device
// give identical bits.  Used to fill inputs too large to stage through host
// memory.  Holds no sorting arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_uniform_u32(uint64_t seed, uint32_t* out, uint64_t start, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (uint32_t)(mix64(seed + (start + i + 1) * 0x9E3779B97F4A7C15ULL) >> 32);
}

__global__ void k_uniform_u64(uint64_t seed, uint64_t* out, uint64_t start, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = mix64(seed + (start + i + 1) * 0x9E3779B97F4A7C15ULL);
}

__global__ void k_iota_u32(uint32_t* out, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (uint32_t)i;
}

__global__ void k_iota_u64(uint64_t* out, uint64_t n) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = i;
}

unsigned grid_for(uint64_t n) {
    uint64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return g ? (unsigned)g : 1u;
}

}  // namespace

// out[i] = high 32 bits of SplitMix64(seed) output start + i, i in [0, n).
extern "C" int gen_dev_uniform_u32(uint64_t seed, void* out, uint64_t start, uint64_t n,
                                   void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_uniform_u32, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, seed,
                       (uint32_t*)out, start, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" int gen_dev_uniform_u64(uint64_t seed, void* out, uint64_t start, uint64_t n,
                                   void* stream) {
    if (!n) return 0;
    hipLaunchKernelGGL(k_uniform_u64, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, seed,
                       (uint64_t*)out, start, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// out[i] = i (payload = original index).
extern "C" int gen_dev_iota(void* out, uint64_t n, int bytes, void* stream) {
    if (!n) return 0;
    if (bytes == 4)
        hipLaunchKernelGGL(k_iota_u32, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                           (uint32_t*)out, n);
    else
        hipLaunchKernelGGL(k_iota_u64, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                           (uint64_t*)out, n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
