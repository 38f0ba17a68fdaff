// rs_tune.hip -- the autotuner: times every small-array algorithm and every
// valid p for each length class on the device it runs on, installs the
// fastest per class in the tuning table, and reports every timing, including
// the device-wide LSD sort of one array per launch (the radix side of the
// small-n crossover the paper observes on CPUs, Section 4, Observation 6).
#include <math.h>
#include <vector>

#include "rs_internal.hpp"

namespace rs {
namespace {

// Tuning input only (the tuner's timings do not depend on the values'
// provenance): a SplitMix64-style finaliser of the index.
__global__ void k_fill_hash(uint32_t* __restrict__ p, uint64_t n, uint64_t seed) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        p[i] = (uint32_t)((z ^ (z >> 31)) >> 32);
    }
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    Timer() { ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

size_t tune_ws_bytes(int instances) {
    LsdPlan lp;
    lsd_plan(SMALL_CAP_U32, 4, 0, 8, &lp);
    return align_up((size_t)instances * SMALL_CAP_U32 * 4) * 2 + align_up(lp.total);
}

}  // namespace rs

using namespace rs;

extern "C" int rs_tune_run(void* ws, size_t ws_bytes, int instances, void* stream,
                           rs_tune_result* out, int max) {
    if (instances < 1 || instances > 65536 || !out || max < 1) return -RS_ERR_INVALID;
    const size_t need = tune_ws_bytes(instances);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % ALIGN)) return -RS_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* w = static_cast<unsigned char*>(ws);
    uint32_t* in = reinterpret_cast<uint32_t*>(w);
    uint32_t* dst = reinterpret_cast<uint32_t*>(w + align_up((size_t)instances * SMALL_CAP_U32 * 4));
    void* lws = w + 2 * align_up((size_t)instances * SMALL_CAP_U32 * 4);
    LsdPlan lp;
    lsd_plan(SMALL_CAP_U32, 4, 0, 8, &lp);
    const uint64_t total = (uint64_t)instances * SMALL_CAP_U32;
    hipLaunchKernelGGL(k_fill_hash, dim3(4096), dim3(256), 0, st, in, total, 0x70e3ull);
    if (hipGetLastError() != hipSuccess) return -RS_ERR_HIP;
    Timer tm;
    int k = 0;
    SegTable& table = tune_table();
    auto time_ms = [&](auto&& launch, int reps) -> double {
        launch();  // warm-up
        if (!tm.ok || hipEventRecord(tm.a, st) != hipSuccess) return (double)NAN;
        for (int r = 0; r < reps; ++r) launch();
        if (hipEventRecord(tm.b, st) != hipSuccess || hipEventSynchronize(tm.b) != hipSuccess) return (double)NAN;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, tm.a, tm.b) != hipSuccess) return (double)NAN;
        return (double)ms / reps;
    };
    for (int c = 1; c <= 14; ++c) {
        const uint32_t n = 1u << c;
        // the instances are packed back to back at stride n
        struct Cand {
            int algo, p;
        };
        std::vector<Cand> cands;
        cands.push_back({RS_ALGO_LDS_RADIX, 0});
        for (int p = 1; p <= 1024; p <<= 1)
            if (small_valid_p(n, p)) {
                cands.push_back({RS_ALGO_BTN, p});
                cands.push_back({RS_ALGO_OET, p});
            }
        double best = INFINITY;
        int best_algo = RS_ALGO_BTN, best_p = small_default_p(RS_ALGO_BTN, n);
        const int first = k;
        for (const Cand& cd : cands) {
            const double ms = time_ms([&] { small_run(cd.algo, in, dst, n, (size_t)instances, cd.p, st); }, 3);
            const double single = time_ms([&] { small_run(cd.algo, in, dst, n, 1, cd.p, st); }, 5);
            if (k < max) {
                out[k].size_log2 = c;
                out[k].algo = cd.algo;
                out[k].p = cd.p;
                out[k].chosen = 0;
                out[k].us_per_array = ms * 1e3 / instances;
                out[k].us_single = single * 1e3;
                ++k;
            }
            if (ms < best) {
                best = ms;
                best_algo = cd.algo;
                best_p = cd.p;
            }
        }
        for (int i = first; i < k; ++i)
            if (out[i].algo == best_algo && out[i].p == best_p) out[i].chosen = 1;
        table.algo[c] = (int8_t)best_algo;
        table.p[c] = (int16_t)(best_algo == RS_ALGO_LDS_RADIX ? 0 : best_p);
        // the device-wide LSD sort, one array per launch sequence
        LsdPlan p1;
        lsd_plan(n, 4, 0, 8, &p1);
        const double lsd = time_ms([&] { lsd_run(p1, in, dst, nullptr, nullptr, lws, st); }, 5);
        if (k < max) {
            out[k].size_log2 = c;
            out[k].algo = RS_ALGO_LSD;
            out[k].p = 0;
            out[k].chosen = 0;
            out[k].us_per_array = lsd * 1e3;
            out[k].us_single = lsd * 1e3;
            ++k;
        }
    }
    table.algo[0] = table.algo[1];
    table.p[0] = 1;
    return k;
}
