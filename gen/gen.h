/*
 * gen.h -- seeded synthetic inputs shared by the oracle tests, the GPU tests
 * and the benchmark.  Holds no sorting arithmetic.
 *
 * Every generator is counter-based: element i depends only on (seed, i), so
 * the host (OpenMP) and device versions give identical bits for any
 * partition of the work.
 *
 * The base stream is SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): the i-th output of a
 * generator seeded with `seed` is mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)
 * with mix64 the published variant-13 finaliser.
 */
#ifndef RS_GEN_H
#define RS_GEN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* i-th SplitMix64 output for `seed`. */
uint64_t gen_splitmix64(uint64_t seed, uint64_t i);

/* Uniform keys on the full range.  u32 keys take the high 32 bits. */
void gen_uniform_u32(uint64_t seed, uint32_t* out, size_t n);
void gen_uniform_u64(uint64_t seed, uint64_t* out, size_t n);
/* Uniform u32 keys for the index range [start, start + n). */
void gen_uniform_u32_range(uint64_t seed, uint32_t* out, size_t start, size_t n);

/* Zipf(s) ranks k in [1, N] by rejection-inversion (Hormann and Derflinger,
 * "Rejection-inversion to generate variates from monotone discrete
 * distributions", 1996); key = k - 1. */
void gen_zipf_u64(uint64_t seed, uint64_t* out, size_t n, double s, double N);

/* Lognormal mu = 0, sigma = 2 scaled to [0, 2^63): Y = exp(2 Z),
 * key = floor(min(Y / e^16, 1 - 2^-53) * 2^63).  Z by Box-Muller. */
void gen_lognormal_u64(uint64_t seed, uint64_t* out, size_t n);

/* Mixture of `comps` equally weighted Gaussians with means uniform on
 * [0, 2^63) and standard deviation 2^sigma_log2; key = mean + llround(
 * 2^sigma_log2 * Z) clamped to [0, 2^63 - 1] in integer arithmetic. */
void gen_gauss_mix_u64(uint64_t seed, uint64_t* out, size_t n, int comps, int sigma_log2);

/* Segment lengths L = floor(2^(lo + (hi - lo) u)), u uniform on [0, 1). */
void gen_loguniform_lengths(uint64_t seed, int64_t* out, size_t S, double lo_log2,
                            double hi_log2);

/* Sample indices in [0, n) drawn with replacement (index = mix % n). */
void gen_sample_indices(uint64_t seed, uint64_t* out, size_t m, uint64_t n);

#ifdef __cplusplus
}
#endif
#endif
