// rs_learned.hip -- learned-CDF bucket sort (an extension beyond the paper)
// for uint64 keys with an optional uint64 payload, stable.
//
//   1. sample 2^18 keys (with replacement, seeded) and sort the sample with
//      the LSD rounds; every 4th sorted key is a training point with the
//      mid-rank target (#{s < k} + #{s <= k}) / 2m over the whole sample;
//   2. train a monotone MLP 1 -> 32 -> 32 -> 1 (weights = softplus of free
//      parameters, tanh hidden units, sigmoid output) on (feature, target)
//      with Adam, all steps in one cooperative launch; the feature is by
//      default the key's place among 4,096 sample quantiles;
//   3. calibrate the output against the sample at 1,025 knots and invert it
//      into 65535 key splitters: s_j = the least key whose bucket is at
//      least j (bisection over keys); a prefix max makes them non-decreasing,
//      so bucket(key) = #{j : s_j <= key} is monotone in the key by
//      construction;
//   4. bucket id of every key: a search tree over the last splitter of every
//      group of four, breadth-first in LDS, then the group in two loads;
//   5. two stable radix-2^8 rounds on the 16-bit bucket id carry each key
//      and value into its bucket, in input order within the bucket;
//   6. every bucket of up to 6,144 pairs is sorted stably in LDS (on the top
//      16 bits of key - bucket start, runs tied there by insertion); a bucket
//      of one key is already in order; crowded and larger buckets are listed;
//   7. listed buckets: crowded ones ranked on every bit, mid-size ones split
//      into sub-ranges sorted in LDS by any workgroup, the largest by the LSD
//      rounds; if too many keys need that, or a final check finds the output
//      unsorted, the whole array is sorted by the LSD rounds from the
//      untouched input.
// Every path ends in the stable sort of the input, so the output does not
// depend on how well the network fits; the fit only decides the speed.
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/rs_learned.h"
#include "rs_dev.h"
#include "rs_internal.hpp"

namespace rs {
namespace {

constexpr int H = 32;
constexpr int NP = 4 * H + H * H + 1;  // 1153 free parameters
constexpr int P_V1 = 0, P_B1 = H, P_V2 = 2 * H, P_B2 = 2 * H + H * H, P_V3 = P_B2 + H, P_B3 = P_V3 + H;
constexpr uint32_t NB = 65536;         // buckets
constexpr uint32_t MS = 1u << 18;      // keys sampled and sorted (targets, calibration)
constexpr uint32_t M = 65536;          // training points: every (MS/M)-th sorted sample key
constexpr uint32_t MSTRIDE = MS / M;
constexpr int TR_NT = 256;             // training threads per workgroup
constexpr int BS_NT = 512;             // bucket-sort threads per workgroup
constexpr int BS_ITEMS = 12;
constexpr uint32_t BS_CAP = BS_NT * BS_ITEMS;  // 6144 pairs
constexpr int AS_NT = 1024;            // assignment threads per workgroup
constexpr int AS_KEYS = 8;             // keys per assignment thread
constexpr int TOP = 16384;             // splitter groups held in LDS (their last entries)
constexpr int GS = (int)NB / TOP;       // splitters per group
constexpr int LG_TOP = 14;             // lg TOP
static_assert((1 << LG_TOP) == TOP, "TOP is 2^LG_TOP");
constexpr int GBUF = NP + 1;           // gradient buffer: parameters + loss
constexpr uint32_t MID_CAP = 1u << 20; // largest bucket sorted by one workgroup
constexpr uint32_t MID_GRID = 1024;    // workgroups sorting the mid-size buckets
constexpr uint32_t TASK_CAP = 1u << 16; // LDS sorts listed for any workgroup to take
constexpr uint32_t TASK_FULL = 1u << 31;  // task flag: a crowded bucket, in place, every bit
constexpr int KNOTS = 1024;            // calibration intervals of the network output
constexpr int QK = 4096;               // key-quantile intervals of the piecewise-linear feature

struct State {
    uint64_t kmin, kmax;
    double inv_span, inv_logspan;
    int32_t mode;          // feature: 0 linear in the key, 1 linear in log2(key),
                           // 2 piecewise linear between the sample's key quantiles
    uint32_t reach;        // number of reachable splitters
    float loss;            // last training loss (mean squared error)
    uint32_t ovf_buckets;          // buckets over the LDS capacity
    unsigned long long ovf_keys;   // keys in them
    uint32_t mid_buckets;          // buckets split and sorted by k_bucket_mid
    uint32_t big_buckets;          // buckets too big for one workgroup (host fallback)
    unsigned long long big_keys;
    uint32_t unsorted;
    uint32_t err;
    uint32_t mid_tasks;    // entries reserved in the mid-size task list
    uint32_t pad_;
    uint64_t qk[QK + 1];   // sample keys at quantiles g/QK (mode 2)
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float softplusf_(float v) { return v > 20.f ? v : log1pf(expf(v)); }
__device__ __forceinline__ float sigmoidf_(float v) { return 1.f / (1.f + expf(-v)); }

// Feature of a key, computed in double and rounded once to float.  Mode 2
// (the default): the key's position among the sample's key quantiles qk[g]
// (g/QK of the sample at or below), linear inside each interval, so the
// feature spreads the keys nearly evenly over [0, 1] whatever their range and
// keeps float resolution where the keys are dense.  Modes 0/1: the position
// in [kmin, kmax], linear or log-scaled.  Every mode is non-decreasing in
// the key.
__device__ __forceinline__ float feat(uint64_t k, const State& s) {
    if (s.mode == 2) {
        if (k <= s.qk[0]) return 0.f;
        if (k >= s.qk[QK]) return 1.f;
        int lo = 0, hi = QK;  // qk[lo] <= k < qk[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s.qk[mid] <= k) lo = mid;
            else hi = mid;
        }
        const double f = (double)(k - s.qk[lo]) / (double)(s.qk[hi] - s.qk[lo]);
        double x = ((double)lo + f) * (1.0 / QK);
        x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
        return (float)x;
    }
    const uint64_t d = k > s.kmin ? k - s.kmin : 0ull;
    double x = s.mode ? log2((double)d + 1.0) * s.inv_logspan : (double)d * s.inv_span;
    x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
    return (float)x;
}

// Network weights in LDS: softplus of the free parameters (and its
// derivative, the logistic function, for the backward pass).
struct Mlp {
    float w1[H], b1[H], w2[H * H], b2[H], w3[H], b3;
    float s1[H], s2[H * H], s3[H];
};

__device__ void mlp_derive(const float* raw, Mlp& W, bool with_sig) {
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
        const float v = raw[p];
        if (p < P_B1) {
            W.w1[p] = softplusf_(v);
            if (with_sig) W.s1[p] = sigmoidf_(v);
        } else if (p < P_V2) {
            W.b1[p - P_B1] = v;
        } else if (p < P_B2) {
            W.w2[p - P_V2] = softplusf_(v);
            if (with_sig) W.s2[p - P_V2] = sigmoidf_(v);
        } else if (p < P_V3) {
            W.b2[p - P_B2] = v;
        } else if (p < P_B3) {
            W.w3[p - P_V3] = softplusf_(v);
            if (with_sig) W.s3[p - P_V3] = sigmoidf_(v);
        } else {
            W.b3 = v;
        }
    }
}

// Forward pass with a fixed order of operations (ascending input index,
// one fused multiply-add per term).
__device__ __forceinline__ float mlp_fwd(const Mlp& W, float x, float (&h1)[H], float (&h2)[H]) {
#pragma unroll
    for (int i = 0; i < H; ++i) h1[i] = tanhf(fmaf(W.w1[i], x, W.b1[i]));
#pragma unroll 4
    for (int o = 0; o < H; ++o) {
        float s = W.b2[o];
#pragma unroll
        for (int i = 0; i < H; ++i) s = fmaf(W.w2[o * H + i], h1[i], s);
        h2[o] = tanhf(s);
    }
    float z = W.b3;
#pragma unroll
    for (int o = 0; o < H; ++o) z = fmaf(W.w3[o], h2[o], z);
    return 1.f / (1.f + expf(-z));
}

__device__ __forceinline__ float mlp_y(const Mlp& W, float x) {
    float h1[H], h2[H];
    return mlp_fwd(W, x, h1, h2);
}

// Calibration: knot[g] is the network output at the sample's g/KNOTS
// quantile (non-decreasing), and u = (g + (y - knot[g]) / (knot[g+1] -
// knot[g])) / KNOTS maps each interval between knots to an equal share of
// (0, 1): the sample fixes how much of the key mass lies between knots, the
// network how it spreads inside each interval.  The map stays monotone.
__device__ __forceinline__ float calibrate(float y, const float* knot) {
    if (y <= knot[0]) return 0.f;
    if (y >= knot[KNOTS]) return 1.f;
    int lo = 0, hi = KNOTS;  // knot[lo] <= y < knot[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (knot[mid] <= y) lo = mid;
        else hi = mid;
    }
    const float d = knot[lo + 1] - knot[lo];
    const float f = d > 0.f ? (y - knot[lo]) / d : 0.f;
    return ((float)lo + fminf(fmaxf(f, 0.f), 1.f)) * (1.0f / (float)KNOTS);
}

// bucket of a key from its feature x: min(NB - 1, floor(NB * calibrated y))
__device__ __forceinline__ uint32_t bucket_of_x(const Mlp& W, const float* knot, float x, int use_net) {
    const float y = use_net ? mlp_y(W, x) : x;
    const float b = calibrate(y, knot) * (float)NB;
    return b >= (float)(NB - 1) ? NB - 1 : (b <= 0.f ? 0u : (uint32_t)b);
}

__device__ __forceinline__ uint32_t bucket_of(const Mlp& W, const State& s, const float* knot, uint64_t k,
                                              int use_net) {
    return bucket_of_x(W, knot, feat(k, s), use_net);
}

// ---- 1. sample, setup, targets ----------------------------------------------

__global__ void k_sample(const uint64_t* __restrict__ keys, uint64_t n, uint64_t seed,
                         uint64_t* __restrict__ sample) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MS) sample[i] = keys[mix64(seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL) % n];
}

__global__ void k_setup(const uint64_t* __restrict__ s, State* st, int mode_req) {
    if (blockIdx.x != 0) return;
    for (int g = threadIdx.x; g <= QK; g += blockDim.x) {
        const uint64_t i = (uint64_t)g * MS / QK;
        st->qk[g] = s[i < MS ? i : MS - 1];
    }
    if (threadIdx.x != 0) return;
    const uint64_t kmin = s[0], kmax = s[MS - 1];
    const uint64_t span = kmax - kmin;
    st->kmin = kmin;
    st->kmax = kmax;
    st->inv_span = span ? 1.0 / (double)span : 0.0;
    const double ls = log2((double)span + 1.0);
    st->inv_logspan = span ? 1.0 / ls : 0.0;
    st->mode = mode_req >= 0 ? mode_req : 2;
}

// Training point i is the middle key of the i-th group of MSTRIDE sorted
// sample keys; its target is its mid-rank in the whole sorted sample.
__global__ void k_targets(const uint64_t* __restrict__ s, const State* __restrict__ st,
                          float* __restrict__ xs, float* __restrict__ ts) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const uint64_t k = s[i * MSTRIDE + MSTRIDE / 2];
    uint32_t lo = 0, hi = MS;  // first index with s >= k
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t first = lo;
    lo = first;
    hi = MS;  // first index with s > k
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s[mid] <= k) lo = mid + 1;
        else hi = mid;
    }
    xs[i] = feat(k, *st);
    ts[i] = (float)(((double)first + (double)lo) / (2.0 * (double)MS));
}

// ---- 2. training -------------------------------------------------------------------
//
// Each Adam step is two ordinary launches on the caller's stream: k_grad
// (every workgroup adds the gradient of its samples into one buffer) and
// k_adam (the update of every parameter, which also clears the buffer for
// the next step).  Stream order is the only synchronisation between steps.

struct TrainCfg {
    float lr, beta1, beta2, eps;
    uint32_t m;        // samples
    int grad_only;     // 1: one gradient over all m samples, scaled by 1/m
};

// Data-dependent initialisation from the sorted sample's features xs:
// hidden unit i of layer 1 starts as a step centred in the i-th of 32
// equal-mass slices of the sample, as steep as that slice is narrow, so the
// units sit where the keys are; layer 2 starts near the identity (a unit
// weight on the diagonal, about 3e-4 elsewhere) and the output layer sums the
// units into (0, 1).  Training then refines every parameter.
__device__ float inv_softplus(float w) { return w > 20.f ? w : logf(expm1f(w)); }

// Output layer at the start: after the first two layers every unit swings
// between about -A and +A (A = tanh(1)), so z = b3 + sum w3_i h2_i climbs
// by A (w3_k + w3_k+1) between the centres of slices k and k+1.  The
// weights make that climb the logit difference of the centres' target CDF
// values (k + 1/2)/H, so sigmoid(z) starts close to the sample's CDF.
__device__ float logit_mid(int k) {
    const float q = ((float)k + 0.5f) / (float)H;
    return logf(q / (1.f - q));
}
__device__ float init_w3(int k) {
    const float A = 0.7615942f;
    const int a = k > 0 ? k - 1 : 0, b = k < H - 1 ? k : H - 2;
    const float dl = logit_mid(a + 1) - logit_mid(a), dr = logit_mid(b + 1) - logit_mid(b);
    return (dl + dr) / (4.f * A);
}

__device__ float init_param(int p, const float* __restrict__ xs, uint32_t m) {
    if (p < P_B2 && p >= P_V2) {
        const int o = (p - P_V2) / H, i = (p - P_V2) % H;
        return o == i ? inv_softplus(1.0f) : -8.0f;
    }
    if (p < P_V2) {
        const int i = p < P_B1 ? p : p - P_B1;
        const float lo = xs[(uint64_t)i * m / H];
        const float hi = xs[(uint64_t)(i + 1) * m / H < m ? (uint64_t)(i + 1) * m / H : m - 1];
        const float c = 0.5f * (lo + hi);
        float w = 2.0f / fmaxf(hi - lo, 1e-6f);
        w = fminf(w, 1e6f);
        return p < P_B1 ? inv_softplus(w) : -w * c;
    }
    if (p < P_V3) return 0.0f;                                  // b2
    if (p < P_B3) return inv_softplus(init_w3(p - P_V3));       // w3
    // b3: z at the middle slice's centre equals its target logit
    const float A = 0.7615942f;
    float acc = 0.f;
    for (int i = 0; i < H; ++i)
        if (i != H / 2) acc += (i < H / 2 ? A : -A) * init_w3(i);
    return logit_mid(H / 2) - acc;
}

// Parameters at the start of training (one thread per parameter).
__global__ void k_train_init(const float* __restrict__ xs, uint32_t m, float* __restrict__ params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NP) params[p] = init_param(p, xs, m);
}

// Gradient of the mean squared error through the softplus, added into gbuf
// (gbuf[NP] gets the summed squared error).  Training step `step`: workgroup
// g of G takes the TR_NT samples starting at ((step * G + g) * TR_NT) mod m,
// so that one step sees a batch of G * TR_NT samples and the steps cycle
// through the set; the mean is over that batch.  grad_only: workgroup g takes
// slices g, g + G, ... of all m samples, and the mean is over m.
__global__ __launch_bounds__(TR_NT) void k_grad(const float* __restrict__ xs, const float* __restrict__ ts,
                                                const float* __restrict__ params, float* __restrict__ gbuf,
                                                TrainCfg cfg, int step) {
    __shared__ float raw[NP], gl[GBUF];
    __shared__ Mlp W;
    __shared__ float A[TR_NT][H + 1], Hm[TR_NT][H + 1];
    __shared__ float xsl[TR_NT], dzl[TR_NT], e2[TR_NT];
    const int t = threadIdx.x;
    const uint32_t G = gridDim.x, g = blockIdx.x;
    for (int p = t; p < NP; p += TR_NT) raw[p] = params[p];
    for (int p = t; p < GBUF; p += TR_NT) gl[p] = 0.f;
    __syncthreads();
    mlp_derive(raw, W, true);
    __syncthreads();
    const uint32_t bsz = cfg.grad_only ? cfg.m : G * TR_NT;
    const uint32_t slices = cfg.grad_only ? (cfg.m + TR_NT - 1) / TR_NT : 1u;
    const uint32_t sl_first = cfg.grad_only ? g : 0u;
    const uint32_t sl_step = cfg.grad_only ? G : 1u;
    for (uint32_t sl = sl_first; sl < slices; sl += sl_step) {
        const uint32_t base = cfg.grad_only ? sl * TR_NT
                                            : (uint32_t)((((uint64_t)step * G + g) * TR_NT) % cfg.m);
        const uint32_t i = base + t;
        const bool live = i < cfg.m;
        const float x = live ? xs[i] : 0.f, tt = live ? ts[i] : 0.f;
        float h1[H], h2[H];
        const float y = mlp_fwd(W, x, h1, h2);
        const float e = live ? (y - tt) : 0.f;
        const float dz = (2.f * e / (float)bsz) * y * (1.f - y);
        float da2[H];
#pragma unroll
        for (int o = 0; o < H; ++o) da2[o] = dz * W.w3[o] * (1.f - h2[o] * h2[o]);
        __syncthreads();
#pragma unroll
        for (int o = 0; o < H; ++o) {
            A[t][o] = da2[o];
            Hm[t][o] = h1[o];
        }
        xsl[t] = x;
        dzl[t] = dz;
        e2[t] = e * e;
        __syncthreads();
        {   // dW2 (4 entries per thread) and db2
            const int o = t >> 3, i0 = (t & 7) * 4;
            float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f, asum = 0.f;
            for (int s = 0; s < TR_NT; ++s) {
                const float a = A[s][o];
                acc0 = fmaf(a, Hm[s][i0 + 0], acc0);
                acc1 = fmaf(a, Hm[s][i0 + 1], acc1);
                acc2 = fmaf(a, Hm[s][i0 + 2], acc2);
                acc3 = fmaf(a, Hm[s][i0 + 3], acc3);
                asum += a;
            }
            gl[P_V2 + o * H + i0 + 0] += acc0 * W.s2[o * H + i0 + 0];
            gl[P_V2 + o * H + i0 + 1] += acc1 * W.s2[o * H + i0 + 1];
            gl[P_V2 + o * H + i0 + 2] += acc2 * W.s2[o * H + i0 + 2];
            gl[P_V2 + o * H + i0 + 3] += acc3 * W.s2[o * H + i0 + 3];
            if ((t & 7) == 0) gl[P_B2 + o] += asum;
        }
        // da1 = (W2^T da2) (1 - h1^2); dz * h2 for the output weights
        float da1[H];
#pragma unroll
        for (int i = 0; i < H; ++i) da1[i] = 0.f;
#pragma unroll 4
        for (int o = 0; o < H; ++o) {
#pragma unroll
            for (int i = 0; i < H; ++i) da1[i] = fmaf(da2[o], W.w2[o * H + i], da1[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < H; ++i) {
            Hm[t][i] = da1[i] * (1.f - h1[i] * h1[i]);
            A[t][i] = dz * h2[i];
        }
        __syncthreads();
        if (t < H) {
            float sb = 0.f, sv = 0.f;
            for (int s = 0; s < TR_NT; ++s) {
                sb += Hm[s][t];
                sv = fmaf(Hm[s][t], xsl[s], sv);
            }
            gl[P_B1 + t] += sb;
            gl[P_V1 + t] += sv * W.s1[t];
        } else if (t < 2 * H) {
            float sv = 0.f;
            for (int s = 0; s < TR_NT; ++s) sv += A[s][t - H];
            gl[P_V3 + t - H] += sv * W.s3[t - H];
        } else if (t == 2 * H) {
            float sb = 0.f;
            for (int s = 0; s < TR_NT; ++s) sb += dzl[s];
            gl[P_B3] += sb;
        } else if (t == 2 * H + 1) {
            float se = 0.f;
            for (int s = 0; s < TR_NT; ++s) se += e2[s];
            gl[NP] += se;
        }
        __syncthreads();
    }
    for (int p = t; p < GBUF; p += TR_NT)
        if (gl[p] != 0.f) atomicAdd(&gbuf[p], gl[p]);
}

// One Adam step (Kingma and Ba, bias-corrected; step counts from 0) on every
// parameter, from the gradient in gbuf; thread p owns parameter p and its
// two moments.  With `clear`, gbuf is zeroed for the next step, and the
// batch's mean squared error is stored as the reported loss.
__global__ void k_adam(float* __restrict__ params, float* __restrict__ m1, float* __restrict__ m2,
                       float* __restrict__ gbuf, TrainCfg cfg, int step, uint32_t bsz, State* __restrict__ st,
                       int clear) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NP) {
        const float gr = gbuf[p];
        const float c1 = 1.f - powf(cfg.beta1, (float)(step + 1));
        const float c2 = 1.f - powf(cfg.beta2, (float)(step + 1));
        const float a = cfg.beta1 * m1[p] + (1.f - cfg.beta1) * gr;
        const float v = cfg.beta2 * m2[p] + (1.f - cfg.beta2) * gr * gr;
        m1[p] = a;
        m2[p] = v;
        params[p] -= cfg.lr * (a / c1) / (sqrtf(v / c2) + cfg.eps);
    } else if (p == NP && st) {
        st->loss = gbuf[NP] / (float)bsz;
    }
    if (clear && p < GBUF) gbuf[p] = 0.f;
}

// ---- 3a. calibration knots ------------------------------------------------------------

__global__ __launch_bounds__(256) void k_calibrate(const float* __restrict__ params,
                                                   const uint64_t* __restrict__ sorted,
                                                   const State* __restrict__ st, float* __restrict__ knot,
                                                   int use_net) {
    constexpr int PER = (KNOTS + 1 + 255) / 256;
    __shared__ Mlp W;
    __shared__ float raw[NP];
    __shared__ float part[256];
    __shared__ State S;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) raw[p] = params[p];
    for (uint32_t i = threadIdx.x; i < sizeof(State) / 8; i += blockDim.x)
        reinterpret_cast<uint64_t*>(&S)[i] = reinterpret_cast<const uint64_t*>(st)[i];
    __syncthreads();
    mlp_derive(raw, W, false);
    __syncthreads();
    // knot g: the network output at the sample's g/KNOTS quantile; thread t
    // holds knots [t*PER, t*PER + PER) and takes their running maximum
    float kv[PER];
    float m = -1.f;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int g = threadIdx.x * PER + q;
        if (g <= KNOTS) {
            const uint64_t i = (uint64_t)g * MS / KNOTS;
            const float x = feat(sorted[i < MS ? i : MS - 1], S);
            const float y = use_net ? mlp_y(W, x) : x;
            m = y > m ? y : m;
        }
        kv[q] = m;
    }
    // exclusive maximum over the threads before this one (the knots must not
    // decrease even where float rounding bends the network)
    part[threadIdx.x] = m;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const float v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : -1.f;
        __syncthreads();
        if (v > part[threadIdx.x]) part[threadIdx.x] = v;
        __syncthreads();
    }
    const float before = threadIdx.x ? part[threadIdx.x - 1] : -1.f;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int g = threadIdx.x * PER + q;
        if (g <= KNOTS) knot[g] = kv[q] > before ? kv[q] : before;
    }
}

// ---- 3. splitters ------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_splitters(const float* __restrict__ params, State* __restrict__ st,
                                                   const float* __restrict__ knot_g, uint64_t* __restrict__ spl,
                                                   int use_net) {
    __shared__ Mlp W;
    __shared__ float raw[NP];
    __shared__ float knot[KNOTS + 1];
    __shared__ State S;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) raw[p] = params[p];
    for (int g = threadIdx.x; g <= KNOTS; g += blockDim.x) knot[g] = knot_g[g];
    for (uint32_t i = threadIdx.x; i < sizeof(State) / 8; i += blockDim.x)
        reinterpret_cast<uint64_t*>(&S)[i] = reinterpret_cast<const uint64_t*>(st)[i];
    __syncthreads();
    mlp_derive(raw, W, false);
    __syncthreads();
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x + 1;  // 1 .. NB-1
    if (j >= NB) {
        if (j == NB) spl[NB - 1] = ~0ull;  // pad entry
        return;
    }
    const uint32_t blo = bucket_of(W, S, knot, S.kmin, use_net);
    const uint32_t bhi = bucket_of(W, S, knot, S.kmax, use_net);
    uint64_t r;
    if (j <= blo) r = 0;
    else if (j > bhi) r = ~0ull;  // no key reaches bucket j
    else {
        // bucket(k) = g(feat(k)) with g non-decreasing on floats in [0, 1]:
        // first the smallest float feature x* with g(x*) >= j, by bisection
        // over the bit patterns of [0, 1] (ordered like the values, at most
        // 30 network evaluations), then the smallest key whose feature
        // reaches x*, by bisection over the keys with the feature alone.
        // That key is the smallest with bucket(k) >= j, the same splitter a
        // bisection over the keys with the whole bucket map finds.
        const float xlo = feat(S.kmin, S), xhi = feat(S.kmax, S);  // g(xlo) < j <= g(xhi)
        uint32_t blo_f = __float_as_uint(xlo), bhi_f = __float_as_uint(xhi);
        while (bhi_f - blo_f > 1) {
            const uint32_t mid = blo_f + (bhi_f - blo_f) / 2;
            if (bucket_of_x(W, knot, __uint_as_float(mid), use_net) >= j) bhi_f = mid;
            else blo_f = mid;
        }
        const float xs = __uint_as_float(bhi_f);
        uint64_t lo = S.kmin, hi = S.kmax;  // feat(lo) < x* <= feat(hi)
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (feat(mid, S) >= xs) hi = mid;
            else lo = mid;
        }
        r = hi;
    }
    spl[j - 1] = r;
    if (j == 1) st->reach = bhi;
}

// Test hook: every key's bucket from the network directly (feature,
// network, calibration; the definition the splitters invert).
__global__ __launch_bounds__(256) void k_direct_ids(const uint64_t* __restrict__ keys, uint64_t n,
                                                    const float* __restrict__ params,
                                                    const State* __restrict__ st,
                                                    const float* __restrict__ knot_g, int use_net,
                                                    uint16_t* __restrict__ out) {
    __shared__ Mlp W;
    __shared__ float raw[NP];
    __shared__ float knot[KNOTS + 1];
    __shared__ State S;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) raw[p] = params[p];
    for (int g = threadIdx.x; g <= KNOTS; g += blockDim.x) knot[g] = knot_g[g];
    for (uint32_t i = threadIdx.x; i < sizeof(State) / 8; i += blockDim.x)
        reinterpret_cast<uint64_t*>(&S)[i] = reinterpret_cast<const uint64_t*>(st)[i];
    __syncthreads();
    mlp_derive(raw, W, false);
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (uint16_t)bucket_of(W, S, knot, keys[i], use_net);
}

// Prefix maximum over the splitters (one workgroup of 1024 threads): makes
// them non-decreasing even where float rounding bends the network.
__global__ __launch_bounds__(1024) void k_split_fix(uint64_t* __restrict__ spl) {
    __shared__ uint64_t part[1024];
    const int t = threadIdx.x;
    constexpr int PER = NB / 1024;
    uint64_t m = 0;
    for (int q = 0; q < PER; ++q) {
        const uint64_t v = spl[t * PER + q];
        m = v > m ? v : m;
    }
    part[t] = m;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint64_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        if (v > part[t]) part[t] = v;
        __syncthreads();
    }
    uint64_t run = t ? part[t - 1] : 0;
    for (int q = 0; q < PER; ++q) {
        const uint64_t v = spl[t * PER + q];
        run = v > run ? v : run;
        spl[t * PER + q] = run;
    }
}

// ---- 4. bucket ids --------------------------------------------------------------------

// The last splitter of every group, in breadth-first (Eytzinger) order: the
// search over groups 0 .. TOP-2 is a complete binary tree of depth
// lg TOP whose node t (1 <= t < TOP, at depth d = floor(lg t)) is group
// ((t - 2^d) << (lg TOP - d)) + 2^(lg TOP - 1 - d) - 1.  Each depth is then
// contiguous in LDS, so the lanes of a wave reading one depth hit
// different banks (sorted order puts all nodes of a depth a power of two
// apart: in one bank).  Entry 0 holds the last group's last splitter.
__global__ void k_top(const uint64_t* __restrict__ spl, uint64_t* __restrict__ topg) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= TOP) return;
    uint32_t grp = TOP - 1;
    if (t > 0) {
        const int d = 31 - __clz(t);
        grp = ((t - (1u << d)) << (LG_TOP - d)) + (1u << (LG_TOP - 1 - d)) - 1;
    }
    topg[t] = spl[(uint32_t)GS * grp + (GS - 1)];
}

__global__ __launch_bounds__(AS_NT) void k_assign(const uint64_t* __restrict__ keys, uint64_t n,
                                                  const uint64_t* __restrict__ spl,
                                                  const uint64_t* __restrict__ topg,
                                                  const State* __restrict__ st, uint16_t* __restrict__ bid) {
    __shared__ uint64_t top[TOP];  // last splitters of the groups, breadth-first (k_top)
    for (int b = threadIdx.x; b < TOP; b += AS_NT) top[b] = topg[b];
    const uint32_t reach = st->reach;
    __syncthreads();
    const uint64_t per_block = (uint64_t)AS_NT * AS_KEYS;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < n; base += (uint64_t)gridDim.x * per_block) {
        uint64_t k[AS_KEYS];
        uint32_t lo[AS_KEYS];
#pragma unroll
        for (int q = 0; q < AS_KEYS; ++q) {
            const uint64_t i = base + (uint64_t)q * AS_NT + threadIdx.x;
            k[q] = i < n ? keys[i] : 0;
            lo[q] = 0;
        }
        // number of groups whose last splitter is <= key: lg TOP steps down
        // the breadth-first tree, one bit of the count per depth
#pragma unroll
        for (int q = 0; q < AS_KEYS; ++q) lo[q] = 1;
#pragma unroll
        for (int d = 0; d < LG_TOP; ++d) {
#pragma unroll
            for (int q = 0; q < AS_KEYS; ++q) lo[q] = 2 * lo[q] + (top[lo[q]] <= k[q] ? 1u : 0u);
        }
#pragma unroll
        for (int q = 0; q < AS_KEYS; ++q) lo[q] -= TOP;
#pragma unroll
        for (int q = 0; q < AS_KEYS; ++q) {
            const uint64_t i = base + (uint64_t)q * AS_NT + threadIdx.x;
            // a key at or above the last group's last splitter takes bucket NB
            const bool past = top[0] <= k[q];
            const uint32_t gi = past ? (uint32_t)TOP - 1 : lo[q];
            uint32_t c = 0;
            if constexpr (GS == 4) {
                // within the group the last entry is > key: its first three
                // come in two independent 16-byte loads and are counted
                const ulonglong2* g2 = reinterpret_cast<const ulonglong2*>(spl + 4u * gi);
                const ulonglong2 x = g2[0], y = g2[1];
                c = (uint32_t)(x.x <= k[q]) + (uint32_t)(x.y <= k[q]) + (uint32_t)(y.x <= k[q]);
            } else {
                // halvings over the group's first GS - 1 entries
                const uint64_t* g = spl + (uint32_t)GS * gi;
#pragma unroll
                for (int step = GS / 2; step >= 1; step >>= 1)
                    if (g[c + step - 1] <= k[q]) c += step;
            }
            const uint32_t ub = past ? NB : (uint32_t)GS * gi + c;
            const uint32_t b = ub < reach ? ub : reach;
            if (i < n) bid[i] = (uint16_t)(b < NB ? b : NB - 1);
        }
    }
}

// ---- 6. buckets ----------------------------------------------------------------------

// start[b] = first position of bucket b in the sorted ids.  Each thread
// takes 8 consecutive ids with one 16-byte load, plus the id just before
// them (in the neighbouring thread's cache line); the array's ragged end and
// a base not 16-byte aligned take the one-id loop.
__global__ void k_bucket_first(const uint16_t* __restrict__ bid, uint64_t n, uint32_t* __restrict__ start) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(bid) & 15u) == 0) {
        const uint64_t groups = n / 8;
        const uint4* b8 = reinterpret_cast<const uint4*>(bid);
        for (uint64_t g = t0; g < groups; g += stride) {
            const uint4 v = b8[g];
            uint32_t id[8] = {v.x & 0xFFFFu, v.x >> 16, v.y & 0xFFFFu, v.y >> 16,
                              v.z & 0xFFFFu, v.z >> 16, v.w & 0xFFFFu, v.w >> 16};
            const uint64_t i = g * 8;
            const uint32_t prev = i ? bid[i - 1] : 0xFFFFFFFFu;
            if (id[0] != prev) start[id[0]] = (uint32_t)i;
#pragma unroll
            for (int r = 1; r < 8; ++r)
                if (id[r] != id[r - 1]) start[id[r]] = (uint32_t)(i + r);
        }
        done = groups * 8;
    }
    for (uint64_t i = done + t0; i < n; i += stride)
        if (i == 0 || bid[i] != bid[i - 1]) start[bid[i]] = (uint32_t)i;
}

// start[b] = min over b' >= b of start[b'] (empty buckets start where the
// next non-empty one does); one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_bucket_fix(uint32_t* __restrict__ start) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    constexpr int PER = NB / 1024;
    const int hi = NB - 1 - t * PER;  // this thread's chunk, walked downwards
    uint32_t m = start[NB];
    uint32_t loc = 0xFFFFFFFFu;
    for (int q = 0; q < PER; ++q) {
        const uint32_t v = start[hi - q];
        loc = v < loc ? v : loc;
    }
    part[t] = loc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = t >= o ? part[t - o] : 0xFFFFFFFFu;
        __syncthreads();
        if (v < part[t]) part[t] = v;
        __syncthreads();
    }
    uint32_t run = t ? part[t - 1] : 0xFFFFFFFFu;
    run = m < run ? m : run;
    for (int q = 0; q < PER; ++q) {
        const uint32_t v = start[hi - q];
        run = v < run ? v : run;
        start[hi - q] = run;
    }
}

// Mid-size bucket (above the LDS capacity): one workgroup runs stable
// radix-2^8 rounds on key - mn over global memory, as many rounds as the
// bucket's key range needs, walking its tiles in order with running digit
// offsets in LDS (the tiles of one bucket never wait on another workgroup).
// Data ping-pongs between the bucket's place and the same place in a
// scratch array; values follow their keys by gathering from the tile.
template <int VB>
__device__ __forceinline__ void bucket_global_lsd(uint64_t* __restrict__ ka, uint64_t* __restrict__ va,
                                  uint64_t* __restrict__ kb, uint64_t* __restrict__ vb, uint32_t L,
                                  uint64_t mn, uint64_t mx, uint64_t* sk, uint16_t* sidx, uint16_t* wcnt,
                                  uint32_t* loc, uint32_t* wsum, uint32_t* tot, uint32_t* run, int sh0 = 0,
                                  int nrounds = 0, bool copy_back = true) {
    constexpr int NW = BS_NT / WAVE;
    constexpr int R = 256;
    uint64_t* wmask = sk;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rounds = nrounds > 0 ? nrounds : (64 - __clzll((unsigned long long)(mx - mn)) + 7) / 8;
    const uint64_t mybit = 1ull << lane;
    const uint32_t wb = wave * (BS_ITEMS * WAVE) + lane;
    for (int r = 0; r < rounds; ++r) {
        const int shift = sh0 + 8 * r;
        uint64_t* sk_src = (r & 1) ? kb : ka;
        uint64_t* sv_src = (r & 1) ? vb : va;
        uint64_t* dk = (r & 1) ? ka : kb;
        uint64_t* dv = (r & 1) ? va : vb;
        __syncthreads();
        if (tid < (uint32_t)R) tot[tid] = 0;
        __syncthreads();
        for (uint32_t q = tid; q < L; q += BS_NT) atomicAdd(&tot[((sk_src[q] - mn) >> shift) & 255u], 1u);
        __syncthreads();
        {
            const uint32_t v = tid < (uint32_t)R ? tot[tid] : 0u;
            uint32_t total;
            const uint32_t ex = block_excl_scan<BS_NT>(v, wsum, &total);
            if (tid < (uint32_t)R) run[tid] = ex;
        }
        for (uint32_t base = 0; base < L; base += BS_CAP) {
            const uint32_t nvalid = (L - base) < BS_CAP ? (L - base) : BS_CAP;
            uint64_t k[BS_ITEMS];
#pragma unroll
            for (int i = 0; i < BS_ITEMS; ++i) {
                const uint32_t j = wb + i * WAVE;
                k[i] = j < nvalid ? sk_src[base + j] : ~0ull;
            }
            __syncthreads();
            for (int i = tid; i < NW * R; i += BS_NT) {
                wcnt[i] = 0;
                wmask[i] = 0;
            }
            __syncthreads();
            uint32_t dr[BS_ITEMS];
            {
                uint16_t* wc = wcnt + wave * R;
                uint64_t* wm = wmask + wave * R;
#pragma unroll
                for (int i = 0; i < BS_ITEMS; ++i) {
                    const uint32_t j = wb + i * WAVE;
                    const uint32_t d = j >= nvalid ? 255u : (uint32_t)(((k[i] - mn) >> shift) & 255u);
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
            if (tid < (uint32_t)R) {
                uint32_t s2 = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const uint32_t c = wcnt[w * R + tid];
                    wcnt[w * R + tid] = (uint16_t)s2;
                    s2 += c;
                }
                t = s2;
                tot[tid] = s2;
            }
            {
                uint32_t total;
                const uint32_t ex = block_excl_scan<BS_NT>(t, wsum, &total);
                if (tid < (uint32_t)R) loc[tid] = ex;
            }
            __syncthreads();
            uint32_t slot[BS_ITEMS];
#pragma unroll
            for (int i = 0; i < BS_ITEMS; ++i) {
                const uint32_t d = dr[i] & 0xFFFFu;
                slot[i] = loc[d] + wcnt[wave * R + d] + (dr[i] >> 16);
            }
            __syncthreads();  // sk aliases the match slots
#pragma unroll
            for (int i = 0; i < BS_ITEMS; ++i) {
                sk[slot[i]] = k[i];
                sidx[slot[i]] = (uint16_t)(wb + i * WAVE);
            }
            __syncthreads();
            for (uint32_t j = tid; j < nvalid; j += BS_NT) {
                const uint64_t key = sk[j];
                const uint32_t d = (uint32_t)(((key - mn) >> shift) & 255u);
                const uint32_t o = run[d] - loc[d] + j;
                if (o < L) {
                    dk[o] = key;
                    if constexpr (VB != 0) dv[o] = sv_src[base + sidx[j]];
                }
            }
            __syncthreads();
            // the padding of a short tile ranked last in digit 255: not keys
            if (tid < (uint32_t)R) run[tid] += tot[tid] - (tid == R - 1 ? BS_CAP - nvalid : 0u);
        }
    }
    if ((rounds & 1) && copy_back) {
        // an odd number of rounds ends in the scratch copy
        __syncthreads();
        for (uint32_t q = tid; q < L; q += BS_NT) {
            ka[q] = kb[q];
            if constexpr (VB != 0) va[q] = vb[q];
        }
    }
}

// LDS workspace of the bucket sort.
struct BucketSmem {
    uint64_t sk[BS_CAP];        // keys in slot order (also the LDS match slots, NW*R)
    uint16_t sidx[BS_CAP];      // their positions in the source
    uint16_t wcnt[(BS_NT / WAVE) * 256];
    uint32_t loc[256];
    uint32_t wsum[BS_NT / WAVE + 1];
    uint64_t rmin[BS_NT / WAVE], rmax[BS_NT / WAVE];
    uint32_t tot[256], run[256];
    uint32_t sub_end[256];      // mid-size split: end of each sub-range
    uint32_t maxrun;
};

// Minimum and maximum of v over the workgroup (every thread gets both).
__device__ __forceinline__ void wg_minmax(uint64_t& mn, uint64_t& mx, BucketSmem& sm) {
    constexpr int NW = BS_NT / WAVE;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t a = __shfl_xor(mn, o, WAVE), c = __shfl_xor(mx, o, WAVE);
        mn = a < mn ? a : mn;
        mx = c > mx ? c : mx;
    }
    __syncthreads();
    if (lane == 0) {
        sm.rmin[wave] = mn;
        sm.rmax[wave] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mn = sm.rmin[w] < mn ? sm.rmin[w] : mn;
        mx = sm.rmax[w] > mx ? sm.rmax[w] : mx;
    }
}

// Stable LDS rounds on the 8-bit digits ((k - mn) >> sh) >> 8r, r < rounds,
// of the keys in registers (k, original positions ix); each round leaves
// the keys in slot order in sm.sk / sm.sidx and reloads k, ix from there.
__device__ __forceinline__ void lds_rounds(uint64_t (&k)[BS_ITEMS], uint32_t (&ix)[BS_ITEMS], uint32_t L, uint64_t mn, int sh,
                           int rounds, BucketSmem& sm) {
    constexpr int NW = BS_NT / WAVE;
    constexpr int R = 256;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wb = wave * (BS_ITEMS * WAVE) + lane;
    const uint64_t mybit = 1ull << lane;
    uint64_t* wmask = sm.sk;
#pragma unroll 1
    for (int r = 0; r < rounds; ++r) {
        const int shift = sh + 8 * r;
        __syncthreads();
        for (int i = tid; i < NW * R; i += BS_NT) {
            sm.wcnt[i] = 0;
            wmask[i] = 0;
        }
        __syncthreads();
        uint32_t dr[BS_ITEMS];
        uint16_t* wc = sm.wcnt + wave * R;
        uint64_t* wm = wmask + wave * R;
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            // an item past the bucket in every lane of the wave is skipped;
            // padding (index >= L) takes the largest digit and comes last
            if (wave * (BS_ITEMS * WAVE) + i * WAVE >= L) {
                dr[i] = 0;
                continue;
            }
            const uint32_t d = ix[i] >= L ? 255u : (uint32_t)(((k[i] - mn) >> shift) & 255u);
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
        uint32_t t = 0;
        if (tid < (uint32_t)R) {
            uint32_t s2 = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = sm.wcnt[w * R + tid];
                sm.wcnt[w * R + tid] = (uint16_t)s2;
                s2 += c;
            }
            t = s2;
        }
        uint32_t total;
        const uint32_t ex = block_excl_scan<BS_NT>(t, sm.wsum, &total);
        if (tid < (uint32_t)R) sm.loc[tid] = ex;
        __syncthreads();
        uint32_t slot[BS_ITEMS];
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            if (wave * (BS_ITEMS * WAVE) + i * WAVE >= L) continue;
            const uint32_t d = dr[i] & 0xFFFFu;
            slot[i] = sm.loc[d] + sm.wcnt[wave * R + d] + (dr[i] >> 16);
        }
        __syncthreads();  // sk aliases the match slots
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            if (wave * (BS_ITEMS * WAVE) + i * WAVE >= L) continue;
            sm.sk[slot[i]] = k[i];
            sm.sidx[slot[i]] = (uint16_t)ix[i];
        }
        __syncthreads();
        // slots past the bucket were not all written: they are padding
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            const uint32_t j = wb + i * WAVE;
            k[i] = j < L ? sm.sk[j] : ~0ull;
            ix[i] = j < L ? sm.sidx[j] : j;
        }
    }
}

// Stable sort in LDS of L <= BS_CAP pairs from (sk_src, sv_src) to
// (kd, vd) (the two may be the same place).  With full = false the keys are
// ordered by their top 16 significant bits above the minimum (at most two
// 8-bit LDS rounds); keys still tied on those bits sit in short runs in input
// order and are finished by an insertion sort per run.  If some run is long
// (keys crowded into a sliver of the range) nothing is written and false is
// returned: the caller ranks that bucket on every bit (full = true) instead.
// The range is the keys' own minimum and maximum, or, when bounded, the
// caller's [lo, hi] known to hold every key (a bucket's splitters), which
// spares the reduction over the keys.
template <int VB>
__device__ __forceinline__ bool lds_sort(const uint64_t* sk_src, const uint64_t* sv_src, uint64_t* kd,
                                         uint64_t* vd, uint32_t L, BucketSmem& sm, bool full,
                                         bool bounded = false, uint64_t lo = 0, uint64_t hi = 0) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wb = wave * (BS_ITEMS * WAVE) + lane;
    uint64_t k[BS_ITEMS];
    uint32_t ix[BS_ITEMS];
    uint64_t mn = ~0ull, mx = 0;
#pragma unroll
    for (int i = 0; i < BS_ITEMS; ++i) {
        const uint32_t j = wb + i * WAVE;
        k[i] = j < L ? sk_src[j] : ~0ull;
        ix[i] = j;
        if (!bounded && j < L) {
            mn = k[i] < mn ? k[i] : mn;
            mx = k[i] > mx ? k[i] : mx;
        }
    }
    if (bounded) {
        mn = lo;
        mx = hi;
    } else {
        wg_minmax(mn, mx, sm);
    }
    if (mn == mx) {  // one distinct key: already in order
        if (kd != sk_src)
            for (uint32_t j = tid; j < L; j += BS_NT) {
                kd[j] = sk_src[j];
                if constexpr (VB != 0) vd[j] = sv_src[j];
            }
        __syncthreads();
        return true;
    }
    const int sig = 64 - __clzll((unsigned long long)(mx - mn));  // significant bits of the range
    const int sh = (!full && sig > 16) ? sig - 16 : 0;
    lds_rounds(k, ix, L, mn, sh, (sig - sh + 7) / 8, sm);
    if (sh > 0) {
        // Runs of keys equal on the ranked bits are finished by a stable
        // insertion sort by key (sidx follows), done by the thread holding
        // the run's first slot.  Ties are found in registers: the slot before
        // j = wb + 64 i is lane - 1 of item i, the last lane of item i - 1, or
        // (first slot of a wave) read from LDS.  A run only permutes its own
        // slots, all of one cell, so a cell read at a run's edge while its
        // owner sorts it is the same at every stage.  A run longer than 64
        // fails the bucket.
        if (tid == 0) sm.maxrun = 0;
        __syncthreads();
        uint64_t tmask[BS_ITEMS];  // per item: the lanes whose slot ties with the one before
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            const uint32_t j = wb + i * WAVE;
            uint64_t p = __shfl_up(k[i], 1, WAVE);
            if (i > 0) {
                const uint64_t q = __shfl(k[i > 0 ? i - 1 : 0], 63, WAVE);
                if (lane == 0) p = q;
            } else if (lane == 0) {
                p = j > 0 ? sm.sk[j - 1] : k[i];
            }
            tmask[i] = __ballot(j > 0 && j < L && ((p - mn) >> sh) == ((k[i] - mn) >> sh));
        }
        uint32_t starts = 0;  // items whose slot starts a run of two or more
#pragma unroll
        for (int i = 0; i < BS_ITEMS; ++i) {
            const uint32_t j = wb + i * WAVE;
            const bool t = (tmask[i] >> lane) & 1ull;
            bool nt;
            if (lane < 63) nt = (tmask[i] >> (lane + 1)) & 1ull;
            else if (i + 1 < BS_ITEMS) nt = tmask[i + 1 < BS_ITEMS ? i + 1 : i] & 1ull;
            else nt = j + 1 < L && ((sm.sk[j + 1] - mn) >> sh) == ((k[i] - mn) >> sh);
            if (!t && nt && j < L) starts |= 1u << i;
        }
        while (starts) {
            const int i = __builtin_ctz(starts);
            starts &= starts - 1;
            const uint32_t j = wb + i * WAVE;
            const uint64_t c = (sm.sk[j] - mn) >> sh;
            uint32_t e = j + 2;
            while (e < L && e - j <= 64 && ((sm.sk[e] - mn) >> sh) == c) ++e;
            if (e - j > 64) {
                atomicMax(&sm.maxrun, e - j);
                continue;
            }
            for (uint32_t a = j + 1; a < e; ++a) {
                const uint64_t kv = sm.sk[a];
                const uint16_t iv = sm.sidx[a];
                uint32_t q = a;
                while (q > j && sm.sk[q - 1] > kv) {
                    sm.sk[q] = sm.sk[q - 1];
                    sm.sidx[q] = sm.sidx[q - 1];
                    --q;
                }
                sm.sk[q] = kv;
                sm.sidx[q] = iv;
            }
        }
        __syncthreads();
        if (sm.maxrun > 64) {
            __syncthreads();
            return false;
        }
    }
    // keys in sk; values gathered by original position, then both written
    constexpr int PQ = (BS_CAP + BS_NT - 1) / BS_NT;
    uint64_t v[VB ? PQ : 1];
    if constexpr (VB != 0) {
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const uint32_t j = q * BS_NT + tid;
            if (j < L) v[q] = sv_src[sm.sidx[j]];
        }
    }
    __syncthreads();
    for (uint32_t j = tid; j < L; j += BS_NT) kd[j] = sm.sk[j];
    if constexpr (VB != 0) {
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const uint32_t j = q * BS_NT + tid;
            if (j < L) vd[j] = v[q];
        }
    }
    __syncthreads();
    return true;
}

// Stable sort of one bucket of up to BS_CAP pairs (and the caller's cap) in
// LDS; keys (and values) are in place in (keys, vals) at [start[b],
// start[b+1]).  A larger bucket is listed: up to MID_CAP for k_bucket_mid,
// beyond that for the host.
template <int VB>
__global__ __launch_bounds__(BS_NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bucket_sort(uint64_t* __restrict__ keys, uint64_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ start, uint32_t cap,
                                                       State* __restrict__ st,
                                                       uint32_t* __restrict__ ovf_list,
                                                       uint32_t* __restrict__ mid_list,
                                                       const uint64_t* __restrict__ spl) {
    __shared__ BucketSmem sm;
    const uint32_t b = blockIdx.x;
    const uint32_t s0 = start[b], s1 = start[b + 1];
    if (s1 <= s0 + 1) return;
    const uint32_t L = s1 - s0;
    // Bucket b holds the keys in [spl[b-1], spl[b]) (from 0 for b = 0): a
    // range of one key means one distinct key, already in input order.
    {
        const uint64_t lo = b ? spl[b - 1] : 0ull;
        const uint64_t hi = spl[b];
        if (b < st->reach && hi > lo && hi - lo == 1) return;
    }
    if (L <= cap && L <= BS_CAP) {
        uint64_t* kb = keys + s0;
        uint64_t* vbk = VB ? vals + s0 : nullptr;
        // below the reach every key of bucket b is in [spl[b-1], spl[b])
        const bool bounded = b < st->reach;
        const uint64_t lo = b ? spl[b - 1] : 0ull;
        const uint64_t hi = spl[b];
        if (!lds_sort<VB>(kb, vbk, kb, vbk, L, sm, false, bounded && hi > lo, lo, hi - 1) &&
            threadIdx.x == 0) {
            // crowded keys: ranked on every bit by k_bucket_mid
            const uint32_t at = atomicAdd(&st->mid_buckets, 1u);
            if (at < NB) mid_list[at] = b;
        }
        return;
    }
    if (threadIdx.x == 0) {
        atomicAdd(&st->ovf_buckets, 1u);
        atomicAdd(&st->ovf_keys, (unsigned long long)L);
        if (L > MID_CAP) {
            // too big for one workgroup: the host sorts it with the LSD rounds
            const uint32_t at = atomicAdd(&st->big_buckets, 1u);
            atomicAdd(&st->big_keys, (unsigned long long)L);
            if (at < NB) ovf_list[at] = b;
        } else {
            const uint32_t at = atomicAdd(&st->mid_buckets, 1u);
            if (at < NB) mid_list[at] = b;
        }
    }
}

// The listed buckets, one workgroup each at a time: crowded ones within the
// LDS capacity are ranked on every bit; mid-size ones (above the capacity,
// up to MID_CAP) are split first.  One stable round through the scratch arrays
// splits a bucket into 2^t sub-ranges of equal key width (the keys of one
// bucket spread almost evenly over its range), about half an LDS load each;
// each sub-range is then sorted in LDS back into place, and a sub-range
// still too large takes the global-memory rounds.
// Reserves n entries of the task list for the calling workgroup (thread 0
// reserves, every thread gets the answer): the index of the first, or
// TASK_CAP when the list is full (then the caller does the work itself).  A
// reservation that runs past the end marks its entries inside the list empty.
__device__ uint32_t reserve_tasks(State* st, uint2* tasks, uint32_t n, BucketSmem& sm) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t base = atomicAdd(&st->mid_tasks, n);
        sm.maxrun = base + n <= TASK_CAP ? base : TASK_CAP;
        for (uint32_t i = base; base + n > TASK_CAP && i < TASK_CAP; ++i) tasks[i] = make_uint2(0u, 0u);
    }
    __syncthreads();
    const uint32_t r = sm.maxrun;
    __syncthreads();
    return r;
}

template <int VB>
__global__ __launch_bounds__(BS_NT) void k_bucket_mid(uint64_t* __restrict__ keys, uint64_t* __restrict__ vals,
                                                      const uint32_t* __restrict__ start,
                                                      State* __restrict__ st,
                                                      const uint32_t* __restrict__ mid_list,
                                                      uint64_t* __restrict__ scr_k, uint64_t* __restrict__ scr_v,
                                                      uint2* __restrict__ tasks) {
    __shared__ BucketSmem sm;
    const uint32_t tid = threadIdx.x;
    const uint32_t count = st->mid_buckets < NB ? st->mid_buckets : NB;
    for (uint32_t w = blockIdx.x; w < count; w += gridDim.x) {
        const uint32_t b = mid_list[w];
        const uint32_t s0 = start[b], L = start[b + 1] - s0;
        uint64_t* kb = keys + s0;
        uint64_t* vbk = VB ? vals + s0 : nullptr;
        uint64_t* sck = scr_k + s0;
        uint64_t* scv = VB ? scr_v + s0 : nullptr;
        if (L <= BS_CAP) {  // a crowded bucket from k_bucket_sort
            const uint32_t at = reserve_tasks(st, tasks, 1, sm);
            if (at < TASK_CAP) {
                if (tid == 0) tasks[at] = make_uint2(s0, L | TASK_FULL);
                continue;
            }
            lds_sort<VB>(kb, vbk, kb, vbk, L, sm, true);
            continue;
        }
        uint64_t mn = ~0ull, mx = 0;
        for (uint32_t q = tid; q < L; q += BS_NT) {
            const uint64_t v = kb[q];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        wg_minmax(mn, mx, sm);
        if (mn == mx) continue;  // one distinct key: already in order
        int t = 1;
        while (t < 8 && ((uint64_t)BS_CAP << (t - 1)) < 2ull * L) ++t;
        const int sig = 64 - __clzll((unsigned long long)(mx - mn));
        const int sh2 = sig > t ? sig - t : 0;
        bucket_global_lsd<VB>(kb, vbk, sck, scv, L, mn, mx, sm.sk, sm.sidx, sm.wcnt, sm.loc, sm.wsum, sm.tot,
                              sm.run, sh2, 1, false);
        __syncthreads();
        if (tid < 256u) sm.sub_end[tid] = sm.run[tid];  // ends of the sub-ranges
        __syncthreads();
        const uint32_t nsub = 1u << t;
        // the sub-ranges are listed for k_bucket_sub, so that every
        // workgroup shares the LDS sorts of the few mid-size buckets
        const uint32_t at = reserve_tasks(st, tasks, nsub, sm);
        if (at < TASK_CAP) {
            if (tid < nsub) {
                const uint32_t a = tid ? sm.sub_end[tid - 1] : 0u;
                tasks[at + tid] = make_uint2(s0 + a, sm.sub_end[tid] - a);
            }
            continue;
        }
        for (uint32_t d = 0; d < nsub; ++d) {
            const uint32_t a = __builtin_amdgcn_readfirstlane(d ? sm.sub_end[d - 1] : 0u);
            const uint32_t c = __builtin_amdgcn_readfirstlane(sm.sub_end[d] - a);
            if (c == 0) continue;
            if (c <= BS_CAP) {
                if (!lds_sort<VB>(sck + a, VB ? scv + a : nullptr, kb + a, VB ? vbk + a : nullptr, c, sm, false))
                    lds_sort<VB>(sck + a, VB ? scv + a : nullptr, kb + a, VB ? vbk + a : nullptr, c, sm, true);
                continue;
            }
            // crowded sub-range: back into place, then the global-memory rounds
            uint64_t smn = ~0ull, smx = 0;
            for (uint32_t q = tid; q < c; q += BS_NT) {
                const uint64_t v = sck[a + q];
                kb[a + q] = v;
                if constexpr (VB != 0) vbk[a + q] = scv[a + q];
                smn = v < smn ? v : smn;
                smx = v > smx ? v : smx;
            }
            wg_minmax(smn, smx, sm);
            if (smn != smx)
                bucket_global_lsd<VB>(kb + a, VB ? vbk + a : nullptr, sck + a, VB ? scv + a : nullptr, c, smn,
                                      smx, sm.sk, sm.sidx, sm.wcnt, sm.loc, sm.wsum, sm.tot, sm.run);
            __syncthreads();
        }
    }
}

// The listed LDS sorts, one workgroup each at a time: a sub-range of a
// split bucket goes from the scratch arrays back into place (a crowded one by
// the global-memory rounds); a crowded bucket is ranked on every bit in
// place.
template <int VB>
__global__ __launch_bounds__(BS_NT) void k_bucket_sub(uint64_t* __restrict__ keys, uint64_t* __restrict__ vals,
                                                      const State* __restrict__ st, const uint2* __restrict__ tasks,
                                                      uint64_t* __restrict__ scr_k, uint64_t* __restrict__ scr_v) {
    __shared__ BucketSmem sm;
    const uint32_t tid = threadIdx.x;
    const uint32_t count = st->mid_tasks < TASK_CAP ? st->mid_tasks : TASK_CAP;
    for (uint32_t w = blockIdx.x; w < count; w += gridDim.x) {
        const uint2 tk = tasks[w];
        const uint32_t a = tk.x, c = tk.y & ~TASK_FULL;
        if (c == 0) continue;
        uint64_t* kb = keys + a;
        uint64_t* vbk = VB ? vals + a : nullptr;
        if (tk.y & TASK_FULL) {
            lds_sort<VB>(kb, vbk, kb, vbk, c, sm, true);
            continue;
        }
        uint64_t* sck = scr_k + a;
        uint64_t* scv = VB ? scr_v + a : nullptr;
        if (c <= BS_CAP) {
            if (!lds_sort<VB>(sck, scv, kb, vbk, c, sm, false)) lds_sort<VB>(sck, scv, kb, vbk, c, sm, true);
            continue;
        }
        uint64_t smn = ~0ull, smx = 0;
        for (uint32_t q = tid; q < c; q += BS_NT) {
            const uint64_t v = sck[q];
            kb[q] = v;
            if constexpr (VB != 0) vbk[q] = scv[q];
            smn = v < smn ? v : smn;
            smx = v > smx ? v : smx;
        }
        wg_minmax(smn, smx, sm);
        if (smn != smx)
            bucket_global_lsd<VB>(kb, vbk, sck, scv, c, smn, smx, sm.sk, sm.sidx, sm.wcnt, sm.loc, sm.wsum, sm.tot,
                                  sm.run);
        __syncthreads();
    }
}

__global__ void k_check_sorted(const uint64_t* __restrict__ keys, uint64_t n, State* __restrict__ st) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride)
        bad |= keys[i - 1] > keys[i];
    if (ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->unsorted, 1u);
}

// Planted bucket-sort error (test hook): the first and last pair of the
// output trade places.
template <int VB>
__global__ void k_fault_swap(uint64_t* __restrict__ keys, uint64_t* __restrict__ vals, uint64_t n) {
    if (threadIdx.x != 0 || n < 2) return;
    const uint64_t k = keys[0];
    keys[0] = keys[n - 1];
    keys[n - 1] = k;
    if constexpr (VB != 0) {
        const uint64_t v = vals[0];
        vals[0] = vals[n - 1];
        vals[n - 1] = v;
    }
}

// Folds the status word of an inner LSD sort (sample, bucket-id rounds,
// large buckets, fallback) into the learned path's own error word.
__global__ void k_or_status(const uint32_t* __restrict__ src, State* __restrict__ st) {
    if (threadIdx.x == 0 && *src) atomicOr(&st->err, *src);
}

__global__ void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ x,
                              float* __restrict__ y, uint64_t m) {
    __shared__ Mlp W;
    __shared__ float raw[NP];
    for (int p = threadIdx.x; p < NP; p += blockDim.x) raw[p] = params[p];
    __syncthreads();
    mlp_derive(raw, W, false);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) y[i] = mlp_y(W, x[i]);
}

}  // namespace

// ---- host side --------------------------------------------------------------------

namespace {

LearnOpts g_opts = {8, 1e-2f, 1, (int32_t)BS_CAP, -1, 0.25, 64, 64};

struct LearnLayout {
    size_t off_state, off_sample, off_sorted, off_sample_ws, off_xs, off_ts, off_params, off_gbuf,
        off_spl, off_top, off_task, off_knot, off_start, off_ovf, off_mid, off_bid0, off_big, total;
    LsdPlan sample_plan, pass_plan, fb_plan;
};

bool learn_layout(size_t n, int vb, LearnLayout* L) {
    LearnLayout q;
    if (!lsd_plan(MS, 8, 0, 8, &q.sample_plan)) return false;
    if (!lsd_plan(n, 2, 8, 8, &q.pass_plan, vb)) return false;
    q.sample_plan.kid_hist = q.sample_plan.kid_scatter = KID_LEARN_SAMPLE;
    q.pass_plan.kid_scatter = KID_LEARN_PASS;
    if (!lsd_plan(n, 8, vb, 8, &q.fb_plan)) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes ? bytes : 1);
        return o;
    };
    q.off_state = take(sizeof(State));
    q.off_sample = take(8 * (size_t)MS);
    q.off_sorted = take(8 * (size_t)MS);
    q.off_sample_ws = take(q.sample_plan.total);
    q.off_xs = take(4 * (size_t)M);
    q.off_ts = take(4 * (size_t)M);
    q.off_params = take(4 * (size_t)NP);
    q.off_gbuf = take(4 * (size_t)GBUF * 3);
    q.off_spl = take(8 * (size_t)NB);
    q.off_top = take(8 * (size_t)TOP);
    q.off_task = take(sizeof(uint2) * (size_t)TASK_CAP);
    q.off_knot = take(4 * (size_t)(KNOTS + 1));
    q.off_start = take(4 * ((size_t)NB + 1));
    q.off_ovf = take(4 * (size_t)NB);
    q.off_mid = take(4 * (size_t)NB);
    q.off_bid0 = take(2 * n);
    // the rounds' workspace and the final bucket ids, or the fallback's
    // workspace (never live at the same time)
    const size_t learned_big = align_up(q.pass_plan.total) + align_up(2 * n);
    q.off_big = take(learned_big > q.fb_plan.total ? learned_big : q.fb_plan.total);
    q.total = off;
    *L = q;
    return true;
}

// Test hooks (host copies, process-wide): parameters used instead of
// training, and splitters used instead of the network's.
struct Inject {
    bool weights = false;
    int fault = 0;  // RS_LEARNED_FAULT_*
    std::vector<float> params;
    std::vector<uint64_t> spl;
    uint16_t* direct = nullptr;    // device: each key's bucket from the network directly
    uint16_t* assigned = nullptr;  // device: each key's bucket from the splitters
};
Inject g_inject;

}  // namespace

LearnOpts& learn_opts() { return g_opts; }

size_t learned_ws_bytes(size_t n, int vb) {
    LearnLayout L;
    if (!learn_layout(n, vb, &L)) return 0;
    return L.total;
}

// Folds an inner LSD plan's status word into st->err (device side, in
// stream order).
static rs_status or_status(const unsigned char* plan_ws, const LsdPlan& p, State* st, hipStream_t s) {
    hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<const uint32_t*>(plan_ws + p.off_status), st);
    return launch_status();
}

rs_status learned_run(const void* kin, void* kout, const void* vin, void* vout, size_t n, int vb,
                      void* ws_, size_t ws_bytes, hipStream_t s, LearnReport* rep) {
    memset(rep, 0, sizeof(*rep));
    LearnLayout L;
    if (!learn_layout(n, vb, &L)) return RS_ERR_UNSUPPORTED;
    if (!ws_ || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws_) % ALIGN)) return RS_ERR_WORKSPACE;
    unsigned char* ws = static_cast<unsigned char*>(ws_);
    State* st = reinterpret_cast<State*>(ws + L.off_state);
    rep->err_word = &st->err;
    uint64_t* sample = reinterpret_cast<uint64_t*>(ws + L.off_sample);
    uint64_t* sorted = reinterpret_cast<uint64_t*>(ws + L.off_sorted);
    float* xs = reinterpret_cast<float*>(ws + L.off_xs);
    float* ts = reinterpret_cast<float*>(ws + L.off_ts);
    float* params = reinterpret_cast<float*>(ws + L.off_params);
    float* gbuf = reinterpret_cast<float*>(ws + L.off_gbuf);
    uint64_t* spl = reinterpret_cast<uint64_t*>(ws + L.off_spl);
    uint64_t* topg = reinterpret_cast<uint64_t*>(ws + L.off_top);
    float* knot = reinterpret_cast<float*>(ws + L.off_knot);
    uint32_t* start = reinterpret_cast<uint32_t*>(ws + L.off_start);
    uint32_t* ovf = reinterpret_cast<uint32_t*>(ws + L.off_ovf);
    uint32_t* mid = reinterpret_cast<uint32_t*>(ws + L.off_mid);
    uint16_t* bid0 = reinterpret_cast<uint16_t*>(ws + L.off_bid0);
    unsigned char* big = ws + L.off_big;
    uint16_t* bid1 = reinterpret_cast<uint16_t*>(big + align_up(L.pass_plan.total));
    const LearnOpts opt = g_opts;
    rs_status rc;
    hipError_t e;

    // 1. sample and targets
    if ((rc = fill_u32(st, sizeof(State) / 4, 0u, s)) != RS_OK) return rc;
    if ((rc = fill_u32(gbuf, GBUF * 3, 0u, s)) != RS_OK) return rc;
    prof(s, KID_LEARN_SAMPLE, 0);
    hipLaunchKernelGGL(k_sample, dim3(MS / 256), dim3(256), 0, s, (const uint64_t*)kin, (uint64_t)n,
                       (uint64_t)0x1A7E5EEDull, sample);
    prof(s, KID_LEARN_SAMPLE, 1);
    if ((rc = launch_status()) != RS_OK) return rc;
    if ((rc = lsd_run(L.sample_plan, sample, sorted, nullptr, nullptr, ws + L.off_sample_ws, s)) != RS_OK)
        return rc;
    if ((rc = or_status(ws + L.off_sample_ws, L.sample_plan, st, s)) != RS_OK) return rc;
    prof(s, KID_LEARN_SAMPLE, 0);
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, s, sorted, st, opt.feature_mode);
    hipLaunchKernelGGL(k_targets, dim3(M / 256), dim3(256), 0, s, sorted, st, xs, ts);
    prof(s, KID_LEARN_SAMPLE, 1);
    if ((rc = launch_status()) != RS_OK) return rc;

    // 2. training: per Adam step one gradient launch and one update launch
    //    (the gradient buffer, then the two moment vectors, in gbuf)
    if (opt.use_network) {
        if (g_inject.weights) {
            if ((e = hipMemcpyAsync(params, g_inject.params.data(), 4 * (size_t)NP, hipMemcpyHostToDevice, s)) !=
                hipSuccess)
                return hip_fail(e);
        } else {
            const TrainCfg cfg{opt.lr, 0.9f, 0.999f, 1e-8f, M, 0};
            const int grid = opt.train_blocks;
            float* m1 = gbuf + GBUF;
            float* m2 = gbuf + 2 * GBUF;
            prof(s, KID_LEARN_TRAIN, 0);
            hipLaunchKernelGGL(k_train_init, dim3((NP + 255) / 256), dim3(256), 0, s, xs, M, params);
            for (int step = 0; step < opt.train_steps; ++step) {
                hipLaunchKernelGGL(k_grad, dim3(grid), dim3(TR_NT), 0, s, xs, ts, params, gbuf, cfg, step);
                hipLaunchKernelGGL(k_adam, dim3((GBUF + 255) / 256), dim3(256), 0, s, params, m1, m2, gbuf, cfg,
                                   step, (uint32_t)grid * TR_NT, st, 1);
            }
            prof(s, KID_LEARN_TRAIN, 1);
            if ((rc = launch_status()) != RS_OK) return rc;
        }
    }

    // 3. calibration knots, splitters
    prof(s, KID_LEARN_SPLIT, 0);
    hipLaunchKernelGGL(k_calibrate, dim3(1), dim3(256), 0, s, params, sorted, st, knot, opt.use_network);
    hipLaunchKernelGGL(k_splitters, dim3(NB / 256), dim3(256), 0, s, params, st, knot, spl, opt.use_network);
    if (g_inject.fault == RS_LEARNED_FAULT_SPLITTERS) {
        // test hook: the caller's splitters replace the network's, as given
        if ((e = hipMemcpyAsync(spl, g_inject.spl.data(), 8 * (size_t)(NB - 1), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return hip_fail(e);
    } else {
        hipLaunchKernelGGL(k_split_fix, dim3(1), dim3(1024), 0, s, spl);
    }
    hipLaunchKernelGGL(k_top, dim3(TOP / 256), dim3(256), 0, s, spl, topg);
    prof(s, KID_LEARN_SPLIT, 1);
    if ((rc = launch_status()) != RS_OK) return rc;

    // 4. bucket ids
    {
        uint64_t g = (n + AS_NT * AS_KEYS - 1) / (AS_NT * AS_KEYS);
        if (g > 256) g = 256;  // each workgroup loads the 128 KiB table once
        prof(s, KID_LEARN_ASSIGN, 0);
        hipLaunchKernelGGL(k_assign, dim3((unsigned)g), dim3(AS_NT), 0, s, (const uint64_t*)kin, (uint64_t)n,
                           spl, topg, st, bid0);
        prof(s, KID_LEARN_ASSIGN, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
    }
    if (g_inject.direct) {
        // test hook: both bucket maps of every key, for the caller to compare
        uint64_t g = (n + 255) / 256;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_direct_ids, dim3((unsigned)g), dim3(256), 0, s, (const uint64_t*)kin, (uint64_t)n,
                           params, st, knot, opt.use_network, g_inject.direct);
        if ((rc = launch_status()) != RS_OK) return rc;
        if ((e = hipMemcpyAsync(g_inject.assigned, bid0, 2 * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return hip_fail(e);
    }
    // 5. two stable rounds on the bucket id carry keys and values
    if ((rc = lsd_run(L.pass_plan, bid0, bid1, kin, kout, big, s, vb ? vin : nullptr, vb ? vout : nullptr)) !=
        RS_OK)
        return rc;
    if ((rc = or_status(big, L.pass_plan, st, s)) != RS_OK) return rc;
    // 6. bucket bounds, per-bucket sort
    if ((rc = fill_u32(start, NB + 1, (uint32_t)n, s)) != RS_OK) return rc;
    {
        uint64_t g = (n + 255) / 256;
        if (g > 8192) g = 8192;
        prof(s, KID_LEARN_BUCKET, 0);
        hipLaunchKernelGGL(k_bucket_first, dim3((unsigned)g), dim3(256), 0, s, bid1, (uint64_t)n, start);
        hipLaunchKernelGGL(k_bucket_fix, dim3(1), dim3(1024), 0, s, start);
        const uint32_t cap = (uint32_t)(opt.bucket_cap > 0 && opt.bucket_cap < (int)BS_CAP ? opt.bucket_cap : BS_CAP);
        // scratch for mid-size buckets: the rounds' temporary key and value
        // arrays, free again once the bucket ids have been sorted
        uint64_t* scr_k = reinterpret_cast<uint64_t*>(big + L.pass_plan.off_tv);
        uint64_t* scr_v = vb ? reinterpret_cast<uint64_t*>(big + L.pass_plan.off_tv2) : nullptr;
        if (vb)
            hipLaunchKernelGGL(k_bucket_sort<8>, dim3(NB), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)vout, start, cap, st, ovf, mid, spl);
        else
            hipLaunchKernelGGL(k_bucket_sort<0>, dim3(NB), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)nullptr, start, cap, st, ovf, mid, spl);
        prof(s, KID_LEARN_BUCKET, 1);
        prof(s, KID_LEARN_MID, 0);
        uint2* tasks = reinterpret_cast<uint2*>(ws + L.off_task);
        if (vb) {
            hipLaunchKernelGGL(k_bucket_mid<8>, dim3(MID_GRID), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)vout, start, st, mid, scr_k, scr_v, tasks);
            hipLaunchKernelGGL(k_bucket_sub<8>, dim3(MID_GRID), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)vout, st, tasks, scr_k, scr_v);
        } else {
            hipLaunchKernelGGL(k_bucket_mid<0>, dim3(MID_GRID), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)nullptr, start, st, mid, scr_k, scr_v, tasks);
            hipLaunchKernelGGL(k_bucket_sub<0>, dim3(MID_GRID), dim3(BS_NT), 0, s, (uint64_t*)kout,
                               (uint64_t*)nullptr, st, tasks, scr_k, scr_v);
        }
        prof(s, KID_LEARN_MID, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
    }
    State hs;
    if ((e = hipMemcpyAsync(&hs, st, sizeof(State), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
    rep->train_loss = hs.loss;
    rep->buckets_overflowed = hs.ovf_buckets;
    rep->keys_overflowed = (int64_t)hs.ovf_keys;
    rep->device_error = hs.err;
    rep->err_word = &st->err;
    rep->feature_mode = hs.mode;

    // too many keys, or too many separate buckets, beyond what one workgroup
    // sorts: the whole array goes through the LSD rounds instead
    bool whole = (double)hs.big_keys > opt.fallback_frac * (double)n ||
                 (int64_t)hs.big_buckets > (int64_t)opt.max_fallback_buckets;
    // 7. overflowed buckets by the LSD rounds, in place
    if (!whole && hs.big_buckets > 0) {
        const uint32_t nb = hs.big_buckets < NB ? hs.big_buckets : NB;
        std::vector<uint32_t> list(nb), st_h(NB + 1);
        if ((e = hipMemcpy(list.data(), ovf, 4 * (size_t)nb, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e);
        if ((e = hipMemcpy(st_h.data(), start, 4 * ((size_t)NB + 1), hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e);
        for (uint32_t b : list) {
            const size_t a = st_h[b], z = st_h[b + 1];
            LsdPlan bp;
            if (!lsd_plan(z - a, 8, vb, 8, &bp)) return RS_ERR_UNSUPPORTED;
            uint64_t* kp = static_cast<uint64_t*>(kout) + a;
            uint64_t* vp = vb ? static_cast<uint64_t*>(vout) + a : nullptr;
            if ((rc = lsd_run(bp, kp, kp, vp, vp, big, s)) != RS_OK) return rc;
            if ((rc = or_status(big, bp, st, s)) != RS_OK) return rc;
        }
    }
    if (!whole && g_inject.fault == RS_LEARNED_FAULT_SWAP) {
        if (vb)
            hipLaunchKernelGGL(k_fault_swap<8>, dim3(1), dim3(64), 0, s, (uint64_t*)kout, (uint64_t*)vout, (uint64_t)n);
        else
            hipLaunchKernelGGL(k_fault_swap<0>, dim3(1), dim3(64), 0, s, (uint64_t*)kout, (uint64_t*)nullptr,
                               (uint64_t)n);
        if ((rc = launch_status()) != RS_OK) return rc;
    }
    if (!whole) {
        prof(s, KID_LEARN_CHECK, 0);
        hipLaunchKernelGGL(k_check_sorted, dim3(4096), dim3(256), 0, s, (const uint64_t*)kout, (uint64_t)n, st);
        prof(s, KID_LEARN_CHECK, 1);
        if ((rc = launch_status()) != RS_OK) return rc;
        uint32_t unsorted = 0;
        if ((e = hipMemcpyAsync(&unsorted, &st->unsorted, 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
        rep->unsorted = unsorted;
        whole = unsorted != 0;
    }
    if (whole) {
        rep->fallback = 1;
        if ((rc = lsd_run(L.fb_plan, kin, kout, vb ? vin : nullptr, vb ? vout : nullptr, big, s)) != RS_OK)
            return rc;
        if ((rc = or_status(big, L.fb_plan, st, s)) != RS_OK) return rc;
    }
    return RS_OK;
}

// ---- test entry points ---------------------------------------------------------------

rs_status mlp_forward(const float* params, const float* x, float* y, size_t m, hipStream_t s) {
    if (!m) return RS_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, params, x, y,
                       (uint64_t)m);
    return launch_status();
}

rs_status mlp_loss_grad(const float* params, const float* x, const float* t, size_t m, float* grad,
                        hipStream_t s) {
    if (!m || m > 0x7FFFFFFFu) return RS_ERR_INVALID;
    rs_status rc = fill_u32(grad, GBUF, 0u, s);
    if (rc != RS_OK) return rc;
    const TrainCfg cfg{0.f, 0.9f, 0.999f, 1e-8f, (uint32_t)m, 1};
    hipLaunchKernelGGL(k_grad, dim3(64), dim3(TR_NT), 0, s, x, t, params, grad, cfg, 0);
    return launch_status();
}

rs_status mlp_adam_step(float* params, float* m1, float* m2, const float* grad, int step, float lr, float beta1,
                        float beta2, float eps, hipStream_t s) {
    const TrainCfg cfg{lr, beta1, beta2, eps, 1u, 0};
    hipLaunchKernelGGL(k_adam, dim3((GBUF + 255) / 256), dim3(256), 0, s, params, m1, m2, const_cast<float*>(grad),
                       cfg, step, 1u, (State*)nullptr, 0);
    return launch_status();
}

rs_status learned_inject_weights(const float* params, size_t count) {
    if (!params) {
        g_inject.weights = false;
        g_inject.params.clear();
        return RS_OK;
    }
    if (count != (size_t)NP) return RS_ERR_INVALID;
    g_inject.params.assign(params, params + NP);
    g_inject.weights = true;
    return RS_OK;
}

rs_status learned_debug_ids(uint16_t* direct, uint16_t* assigned) {
    if ((direct == nullptr) != (assigned == nullptr)) return RS_ERR_INVALID;
    g_inject.direct = direct;
    g_inject.assigned = assigned;
    return RS_OK;
}

rs_status learned_inject_fault(int kind, const uint64_t* spl, size_t count) {
    if (kind == RS_LEARNED_FAULT_SPLITTERS) {
        if (!spl || count != (size_t)NB - 1) return RS_ERR_INVALID;
        g_inject.spl.assign(spl, spl + (NB - 1));
    } else if (kind == RS_LEARNED_FAULT_NONE || kind == RS_LEARNED_FAULT_SWAP) {
        g_inject.spl.clear();
    } else {
        return RS_ERR_INVALID;
    }
    g_inject.fault = kind;
    return RS_OK;
}

}  // namespace rs
