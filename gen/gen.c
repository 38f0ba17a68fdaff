/* gen.c -- seeded synthetic inputs (see gen.h).  No sorting arithmetic. */
#include "gen.h"

#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gen_splitmix64(uint64_t seed, uint64_t i) { return mix64(seed + (i + 1) * GOLDEN); }

/* j-th draw of the private sub-stream of element i */
static inline uint64_t sub(uint64_t seed, uint64_t i, uint64_t j) {
    return gen_splitmix64(gen_splitmix64(seed, i), j);
}

/* uniform double on [0, 1) with 53 random bits */
static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

void gen_uniform_u32(uint64_t seed, uint32_t* out, size_t n) {
    gen_uniform_u32_range(seed, out, 0, n);
}

void gen_uniform_u32_range(uint64_t seed, uint32_t* out, size_t start, size_t n) {
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)n; i++)
        out[i] = (uint32_t)(gen_splitmix64(seed, (uint64_t)start + (uint64_t)i) >> 32);
}

void gen_uniform_u64(uint64_t seed, uint64_t* out, size_t n) {
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)n; i++) out[i] = gen_splitmix64(seed, (uint64_t)i);
}

/* ---- Zipf by rejection-inversion ---------------------------------------- */
/* H(x) = integral of x^-s = (x^(1-s) - 1)/(1-s), written with expm1/log1p
 * so it stays accurate when s is close to 1. */
static double zH(double x, double s) {
    double q = 1.0 - s, lx = log(x);
    return fabs(q * lx) > 1e-8 ? expm1(q * lx) / q : lx * (1.0 + 0.5 * q * lx);
}
static double zHinv(double u, double s) {
    double q = 1.0 - s, t = u * q;
    if (t < -1.0) t = -1.0;
    return fabs(t) > 1e-8 ? exp(log1p(t) / q) : exp(u * (1.0 - 0.5 * t));
}
static double zh(double x, double s) { return exp(-s * log(x)); }

void gen_zipf_u64(uint64_t seed, uint64_t* out, size_t n, double s, double N) {
    double hx1 = zH(1.5, s) - 1.0;
    double hN = zH(N + 0.5, s);
    double sq = 2.0 - zHinv(zH(2.5, s) - zh(2.0, s), s);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)n; i++) {
        uint64_t k = 1;
        for (uint64_t j = 0;; j++) {
            double u = hN + u01(sub(seed, (uint64_t)i, j)) * (hx1 - hN);
            double x = zHinv(u, s);
            double kf = floor(x + 0.5);
            if (kf < 1.0) kf = 1.0;
            if (kf > N) kf = N;
            if (kf - x <= sq || u >= zH(kf + 0.5, s) - zh(kf, s)) {
                k = (uint64_t)kf;
                break;
            }
        }
        out[i] = k - 1;
    }
}

/* ---- Gaussian draws ------------------------------------------------------ */
static double box_muller(uint64_t seed, uint64_t i, uint64_t j) {
    double u1 = 1.0 - u01(sub(seed, i, j));      /* (0, 1] */
    double u2 = u01(sub(seed, i, j + 1));        /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

void gen_lognormal_u64(uint64_t seed, uint64_t* out, size_t n) {
    const double cap = 1.0 - 0x1.0p-53;
    const double e16 = exp(16.0);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)n; i++) {
        double y = exp(2.0 * box_muller(seed, (uint64_t)i, 0)) / e16;
        if (y > cap) y = cap;
        out[i] = (uint64_t)floor(y * 0x1.0p63);
    }
}

void gen_gauss_mix_u64(uint64_t seed, uint64_t* out, size_t n, int comps, int sigma_log2) {
    uint64_t means[256];
    if (comps < 1) comps = 1;
    if (comps > 256) comps = 256;
    for (int c = 0; c < comps; c++) means[c] = gen_splitmix64(seed ^ 0x4D45414E53ULL, (uint64_t)c) >> 1;
    const double sd = ldexp(1.0, sigma_log2);
    const int64_t top = INT64_MAX;
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)n; i++) {
        int c = (int)(sub(seed, (uint64_t)i, 0) % (uint64_t)comps);
        long long dz = llround(sd * box_muller(seed, (uint64_t)i, 1));
        int64_t m = (int64_t)means[c], v;
        if (dz > 0 && m > top - dz) v = top;
        else if (dz < 0 && m < -dz) v = 0;
        else v = m + dz;
        out[i] = (uint64_t)v;
    }
}

void gen_loguniform_lengths(uint64_t seed, int64_t* out, size_t S, double lo_log2,
                            double hi_log2) {
    for (size_t s = 0; s < S; s++) {
        double u = u01(gen_splitmix64(seed, s));
        out[s] = (int64_t)floor(exp2(lo_log2 + (hi_log2 - lo_log2) * u));
    }
}

void gen_sample_indices(uint64_t seed, uint64_t* out, size_t m, uint64_t n) {
    for (size_t i = 0; i < m; i++) out[i] = n ? gen_splitmix64(seed, i) % n : 0;
}
