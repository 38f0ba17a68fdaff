// rs_tune.hip -- the autotuner: times every small-array algorithm and every
// valid p for each length class on the device it runs on (or, model-guided,
// only the p a fitted cost model in the form of the paper's T_b and T_o
// predicts best), installs the fastest per class in the tuning table, and
// reports every timing, including the device-wide LSD sort of one array per
// launch (the radix side of the small-n crossover the paper observes on
// CPUs, Section 4, Observation 6); above the small classes it picks the
// radix and tile of single arrays and the tile of large segments.
#include <math.h>

#include <cmath>
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

// Offsets of S segments of L keys each: off[i] = i * L, i = 0..S.
__global__ void k_even_offsets(int64_t* __restrict__ off, uint64_t S, uint64_t L) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= S; i += stride) off[i] = (int64_t)(i * L);
}

constexpr int TUNE_LSD_MAX = 24;  // largest class of the single-array LSD timings
// largest class of the segment timings (the tile of the one-workgroup
// rounds: RS_ALGO_LSD segments, the block networks' runs, segments of 2^30
// keys and more; the shared device-wide rounds have no tile choice)
constexpr int TUNE_SEG_MAX = 20;
// A segment class is timed only with enough segments to occupy every
// workgroup slot of the persistent launch at once (its throughput, not the
// latency of a few segments, decides the batched workload).
constexpr uint64_t TUNE_SEG_MIN_COUNT = 512;
constexpr double TUNE_MARGIN = 0.03;

struct LsdCand {
    int bits, items;
};
constexpr LsdCand LSD_CANDS[] = {{8, 16}, {8, 28}, {11, 0}, {8, 8}};

// Largest class the tuner times with `instances` small arrays of workspace.
int tune_cmax(int instances) {
    const uint64_t N = (uint64_t)instances * SMALL_CAP_U32;
    int c = 14;
    while (c < TUNE_LSD_MAX && (1ull << (c + 1)) <= N) ++c;
    return c;
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

// Cost model of one workgroup sorting an array of npad keys with p
// processors holding runs of N = npad / p keys, in the form of the paper's
// T_b and T_o (Section 3): a local sort of each run, then S merge-split
// stages (BTN: lg p (lg p + 1) / 2; OET: p rounds), each a bitonic merge of
// two runs and an exchange.  With many arrays in one launch the machine is
// saturated, so an array costs the work of all p processors, plus a share
// of the launch:
//   t = c0 * npad lg N (lg N + 1) / 4        compare-exchanges of the local sorts
//     + c1 * S npad (lg N + 1)               compare-exchanges of the stages
//     + c2 * S p                             fixed cost of a processor's stage
//     + c3                                   per array, whatever p.
constexpr int NF = 4;
void model_features(int algo, uint32_t npad, int p, double f[NF]) {
    const double N = (double)npad / p, lgN = log2(N), lgp = log2((double)p);
    const double S = algo == RS_ALGO_OET ? (double)p : lgp * (lgp + 1.0) / 2.0;
    f[0] = (double)npad * lgN * (lgN + 1.0) / 4.0;
    f[1] = S * (double)npad * (lgN + 1.0);
    f[2] = S * (double)p;
    f[3] = 1.0;
}

// Least squares for the NF constants, each row weighted by 1 / t (so the
// fit minimises relative error).  Returns false for a singular system.
bool model_fit(const std::vector<double>& F, const std::vector<double>& t, double c[NF]) {
    double A[NF][NF] = {}, b[NF] = {};
    for (size_t i = 0; i < t.size(); ++i) {
        const double* f = &F[NF * i];
        const double w = 1.0 / (t[i] * t[i]);
        for (int r = 0; r < NF; ++r) {
            b[r] += w * f[r] * t[i];
            for (int q = 0; q < NF; ++q) A[r][q] += w * f[r] * f[q];
        }
    }
    // Gaussian elimination with partial pivoting
    for (int col = 0; col < NF; ++col) {
        int piv = col;
        for (int r = col + 1; r < NF; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (fabs(A[piv][col]) < 1e-300) return false;
        for (int q = 0; q < NF; ++q) {
            const double tmp = A[col][q];
            A[col][q] = A[piv][q];
            A[piv][q] = tmp;
        }
        const double tb = b[col];
        b[col] = b[piv];
        b[piv] = tb;
        for (int r = col + 1; r < NF; ++r) {
            const double m = A[r][col] / A[col][col];
            for (int q = col; q < NF; ++q) A[r][q] -= m * A[col][q];
            b[r] -= m * b[col];
        }
    }
    for (int r = NF - 1; r >= 0; --r) {
        double v = b[r];
        for (int q = r + 1; q < NF; ++q) v -= A[r][q] * c[q];
        c[r] = v / A[r][r];
    }
    return true;
}

double model_us(int algo, uint32_t npad, int p, const double c[NF]) {
    double f[NF];
    model_features(algo, npad, p, f);
    double t = 0;
    for (int q = 0; q < NF; ++q) t += c[q] * f[q];
    return t;
}

}  // namespace

// Workspace of the tuner: the input and output arrays of instances * 16384
// keys, then the largest LSD or segmented-sort workspace it times, then the
// segment offsets.
namespace {
size_t tune_inner_bytes(int instances) {
    const uint64_t N = (uint64_t)instances * SMALL_CAP_U32;
    LsdPlan lp;
    lsd_plan(SMALL_CAP_U32, 4, 0, 8, &lp);
    size_t inner = lp.total;
    const int cmax = tune_cmax(instances);
    for (int c = 15; c <= cmax; ++c)
        for (const LsdCand& cd : LSD_CANDS)
            if (lsd_plan(1ull << c, 4, 0, cd.bits, &lp, 0, cd.items) && lp.total > inner) inner = lp.total;
    SegPlan sp;
    if (cmax >= 15 && seg_plan(N >> 15, (int64_t)N, &sp) && sp.total > inner) inner = sp.total;
    return align_up(inner);
}
}  // namespace

size_t tune_ws_bytes(int instances) {
    const uint64_t N = (uint64_t)instances * SMALL_CAP_U32;
    return align_up((size_t)N * 4) * 2 + tune_inner_bytes(instances) + align_up(8 * ((N >> 15) + 1));
}

}  // namespace rs

using namespace rs;

namespace {
int tune_impl(void* ws, size_t ws_bytes, int instances, void* stream, rs_tune_result* out, int max,
              bool model) {
    if (instances < 1 || instances > 65536 || !out || max < 1) return -RS_ERR_INVALID;
    const size_t need = tune_ws_bytes(instances);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % ALIGN)) return -RS_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned char* w = static_cast<unsigned char*>(ws);
    uint32_t* in = reinterpret_cast<uint32_t*>(w);
    uint32_t* dst = reinterpret_cast<uint32_t*>(w + align_up((size_t)instances * SMALL_CAP_U32 * 4));
    void* lws = w + 2 * align_up((size_t)instances * SMALL_CAP_U32 * 4);
    const int cmax = tune_cmax(instances);
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
    // Model-guided: the constants of the cost model above are fitted, per
    // algorithm, to timings of three p (smallest, middle, largest valid) in
    // four classes; then every class times only the p the model predicts
    // fastest and its two neighbours (and the LDS radix sort).
    double coef[2][NF] = {};
    bool fitted[2] = {false, false};
    std::vector<double> cal_ms[2][15];  // [algo][class] timings by p index, NaN if not timed
    if (model) {
        constexpr int CAL[4] = {4, 7, 10, 13};
        for (int ai = 0; ai < 2; ++ai) {
            const int algo = ai ? RS_ALGO_OET : RS_ALGO_BTN;
            std::vector<double> F, T;
            for (int c : CAL) {
                const uint32_t n = 1u << c;
                std::vector<int> ps;
                for (int p = 1; p <= 1024; p <<= 1)
                    if (small_valid_p(n, p)) ps.push_back(p);
                cal_ms[ai][c].assign(ps.size(), (double)NAN);
                const size_t pick[3] = {0, ps.size() / 2, ps.size() - 1};
                for (size_t i : pick) {
                    if (!std::isnan(cal_ms[ai][c][i])) continue;
                    const double ms =
                        time_ms([&] { small_run(algo, in, dst, n, (size_t)instances, ps[i], st); }, 3);
                    cal_ms[ai][c][i] = ms;
                    double f[NF];
                    model_features(algo, small_npad(n), ps[i], f);
                    F.insert(F.end(), f, f + NF);
                    T.push_back(ms * 1e3 / instances);
                }
            }
            fitted[ai] = model_fit(F, T, coef[ai]);
        }
    }
    for (int c = 1; c <= 14 && model; ++c) {
        const uint32_t n = 1u << c, npad = small_npad(n);
        double best = INFINITY;
        int best_algo = RS_ALGO_BTN, best_p = small_default_p(RS_ALGO_BTN, n);
        const int first = k;
        auto record = [&](int algo, int p, double ms, double single, double pred) {
            if (k < max) {
                out[k] = rs_tune_result{};
                out[k].size_log2 = c;
                out[k].algo = algo;
                out[k].p = p;
                out[k].us_per_array = ms * 1e3 / instances;
                out[k].us_single = single * 1e3;
                out[k].us_model = pred;
                ++k;
            }
            if (ms < best) {
                best = ms;
                best_algo = algo;
                best_p = p;
            }
        };
        {
            const double ms = time_ms([&] { small_run(RS_ALGO_LDS_RADIX, in, dst, n, (size_t)instances, 0, st); }, 3);
            const double single = time_ms([&] { small_run(RS_ALGO_LDS_RADIX, in, dst, n, 1, 0, st); }, 5);
            record(RS_ALGO_LDS_RADIX, 0, ms, single, (double)NAN);
        }
        for (int ai = 0; ai < 2; ++ai) {
            const int algo = ai ? RS_ALGO_OET : RS_ALGO_BTN;
            std::vector<int> ps;
            for (int p = 1; p <= 1024; p <<= 1)
                if (small_valid_p(n, p)) ps.push_back(p);
            std::vector<double> pred(ps.size());
            size_t arg = 0;
            for (size_t i = 0; i < ps.size(); ++i) {
                pred[i] = fitted[ai] ? model_us(algo, npad, ps[i], coef[ai]) : 0.0;
                if (pred[i] < pred[arg]) arg = i;
            }
            for (size_t i = 0; i < ps.size(); ++i) {
                const bool timed = i + 1 >= arg && i <= arg + 1;  // the predicted best and its neighbours
                if (!timed && fitted[ai]) {
                    if (k < max) {
                        out[k] = rs_tune_result{};
                        out[k].size_log2 = c;
                        out[k].algo = algo;
                        out[k].p = ps[i];
                        out[k].us_per_array = (double)NAN;
                        out[k].us_single = (double)NAN;
                        out[k].us_model = pred[i];
                        ++k;
                    }
                    continue;
                }
                double ms = (c < 15 && i < cal_ms[ai][c].size()) ? cal_ms[ai][c][i] : (double)NAN;
                if (std::isnan(ms))
                    ms = time_ms([&] { small_run(algo, in, dst, n, (size_t)instances, ps[i], st); }, 3);
                const double single = time_ms([&] { small_run(algo, in, dst, n, 1, ps[i], st); }, 5);
                record(algo, ps[i], ms, single, fitted[ai] ? pred[i] : (double)NAN);
            }
        }
        for (int i = first; i < k; ++i)
            if (out[i].algo == best_algo && out[i].p == best_p && !std::isnan(out[i].us_per_array)) out[i].chosen = 1;
        table.algo[c] = (int8_t)best_algo;
        table.p[c] = (int16_t)(best_algo == RS_ALGO_LDS_RADIX ? 0 : best_p);
        LsdPlan p1;
        lsd_plan(n, 4, 0, 8, &p1);
        const double lsd = time_ms([&] { lsd_run(p1, in, dst, nullptr, nullptr, lws, st); }, 5);
        if (k < max) {
            out[k] = rs_tune_result{};
            out[k].size_log2 = c;
            out[k].algo = RS_ALGO_LSD;
            out[k].radix_bits = 8;
            out[k].us_per_array = lsd * 1e3;
            out[k].us_single = lsd * 1e3;
            out[k].us_model = (double)NAN;
            ++k;
        }
    }
    for (int c = 1; c <= 14 && !model; ++c) {
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
                out[k] = rs_tune_result{};
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
            out[k] = rs_tune_result{};
            out[k].size_log2 = c;
            out[k].algo = RS_ALGO_LSD;
            out[k].radix_bits = 8;
            out[k].us_per_array = lsd * 1e3;
            out[k].us_single = lsd * 1e3;
            ++k;
        }
    }
    table.algo[0] = table.algo[1];
    table.p[0] = 1;

    // Larger classes: the single-array LSD sort's radix and tile, and the
    // tile of a segment sorted by one workgroup's radix rounds.
    const uint64_t N = (uint64_t)instances * SMALL_CAP_U32;
    int64_t* off = reinterpret_cast<int64_t*>(static_cast<unsigned char*>(lws) + tune_inner_bytes(instances));
    // Each candidate is timed twice, the candidates interleaved, and keeps
    // its faster time; a candidate replaces the library's default only when
    // it is at least TUNE_MARGIN faster (timings of one batch vary by a few
    // per cent from run to run).
    for (int c = 15; c <= cmax; ++c) {
        const uint64_t n = 1ull << c;
        constexpr int NL = (int)(sizeof(LSD_CANDS) / sizeof(LSD_CANDS[0]));
        double lt[NL];
        LsdPlan pl[NL];
        bool okp[NL];
        for (int q = 0; q < NL; ++q) {
            lt[q] = INFINITY;
            okp[q] = lsd_plan(n, 4, 0, LSD_CANDS[q].bits, &pl[q], 0, LSD_CANDS[q].items);
        }
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < NL; ++q)
                if (okp[q]) {
                    const double ms = time_ms([&] { lsd_run(pl[q], in, dst, nullptr, nullptr, lws, st); }, 5);
                    lt[q] = ms < lt[q] ? ms : lt[q];
                }
        // the default: radix 2^8, 16-key tiles below 2^23 keys, 28 above
        const int def = n < (1ull << 23) ? 0 : 1;
        int best = def;
        for (int q = 0; q < NL; ++q)
            if (okp[q] && lt[q] < lt[best]) best = q;
        const int pick = lt[best] < lt[def] * (1.0 - TUNE_MARGIN) ? best : def;
        for (int q = 0; q < NL; ++q)
            if (okp[q] && k < max) {
                out[k] = rs_tune_result{};
                out[k].size_log2 = c;
                out[k].algo = RS_ALGO_LSD;
                out[k].radix_bits = LSD_CANDS[q].bits;
                out[k].tile_items = LSD_CANDS[q].items;
                out[k].chosen = q == pick;
                out[k].us_per_array = lt[q] * 1e3;
                out[k].us_single = lt[q] * 1e3;
                ++k;
            }
        table.radix[c] = (int8_t)LSD_CANDS[pick].bits;
        table.items[c] = (int8_t)LSD_CANDS[pick].items;
        if (c > TUNE_SEG_MAX) continue;
        // S segments of 2^c keys, each sorted by one workgroup's rounds (no
        // shared rounds), as one batch with each tile size
        const uint64_t S = N >> c;
        SegPlan sp;
        if (S < TUNE_SEG_MIN_COUNT || !seg_plan(S, (int64_t)(S * n), &sp, false)) continue;
        hipLaunchKernelGGL(k_even_offsets, dim3(64), dim3(256), 0, st, off, S, n);
        if (hipGetLastError() != hipSuccess) return -RS_ERR_HIP;
        constexpr int SEG_CANDS[2] = {16, 8};  // the default first
        double stt[2] = {INFINITY, INFINITY};
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < 2; ++q) {
                SegTable t2 = table;
                t2.seg_items[c] = (int8_t)SEG_CANDS[q];
                const double ms =
                    time_ms([&] { seg_run(sp, in, dst, off, S, (int64_t)(S * n), t2, lws, st); }, 3);
                stt[q] = ms < stt[q] ? ms : stt[q];
            }
        const int spick = stt[1] < stt[0] * (1.0 - TUNE_MARGIN) ? 1 : 0;
        for (int q = 0; q < 2; ++q)
            if (k < max) {
                out[k] = rs_tune_result{};
                out[k].size_log2 = c;
                out[k].algo = RS_ALGO_AUTO;
                out[k].seg_tile_items = SEG_CANDS[q];
                out[k].chosen = q == spick;
                out[k].us_per_array = stt[q] * 1e3 / (double)S;
                out[k].us_single = NAN;
                ++k;
            }
        table.seg_items[c] = (int8_t)SEG_CANDS[spick];
    }
    if (hipStreamSynchronize(st) != hipSuccess) return -RS_ERR_HIP;
    return k;
}
}  // namespace

extern "C" int rs_tune_run(void* ws, size_t ws_bytes, int instances, void* stream,
                           rs_tune_result* out, int max) {
    return tune_impl(ws, ws_bytes, instances, stream, out, max, false);
}

extern "C" int rs_tune_run_model(void* ws, size_t ws_bytes, int instances, void* stream,
                                 rs_tune_result* out, int max) {
    return tune_impl(ws, ws_bytes, instances, stream, out, max, true);
}
