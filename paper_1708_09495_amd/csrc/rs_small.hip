// rs_small.hip -- batches of small arrays, one workgroup per array: BTN,
// OET and the LDS radix sort (device functions in rs_small_dev.h).
#include "rs_internal.hpp"
#include "rs_small_dev.h"

namespace rs {
namespace {

// n_pad <= 16384, so p = n_pad / N threads never exceed 16384 / N.
constexpr int net_threads(int N) { return N >= 64 ? 256 : (N >= 32 ? 512 : 1024); }

template <int N>
__global__ __launch_bounds__(net_threads(N)) void k_btn(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, uint32_t n, int p) {
    extern __shared__ uint32_t sh[];
    const size_t off = (size_t)blockIdx.x * n;
    btn_sort<N>(in + off, out + off, n, p, sh);
}

template <int N>
__global__ __launch_bounds__(net_threads(N)) void k_oet(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, uint32_t n, int p) {
    extern __shared__ uint32_t sh[];
    const size_t off = (size_t)blockIdx.x * n;
    oet_sort<N>(in + off, out + off, n, p, sh);
}

constexpr int LR_NT = 512;
constexpr int LR_NW = LR_NT / WAVE;

template <int ITEMS>
__global__ __launch_bounds__(LR_NT) void k_lds_radix(const uint32_t* __restrict__ in,
                                                     uint32_t* __restrict__ out, uint32_t n) {
    __shared__ uint64_t wmask[LR_NW * 256];
    __shared__ uint16_t wcnt[LR_NW * 256];
    __shared__ uint32_t loc[256];
    __shared__ uint32_t wsum[LR_NW + 1];
    extern __shared__ uint32_t sk[];
    const size_t off = (size_t)blockIdx.x * n;
    lds_radix_sort<ITEMS, LR_NT>(in + off, out + off, n, wmask, wcnt, loc, wsum, sk);
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
