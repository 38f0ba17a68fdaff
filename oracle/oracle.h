/*
 * oracle.h -- plain serial C reference for the integer sorts of
 * Gerbessiotis, "Integer sorting on multicores: some (experiments and)
 * observations" (arXiv 1708.09495).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library: it is written from the
 * paper's definitions, slowly and obviously, so that a reader can check it
 * against the paper by eye.
 *
 * Conventions shared by every function here:
 *   - keys are unsigned integers of key_bytes = 4 or 8 bytes, sorted
 *     ascending (the paper says "32-bit integers" and never signed or
 *     descending; unsigned ascending is the reading taken);
 *   - values (payloads) are val_bytes = 0, 4 or 8 bytes and move with their
 *     key; every sort that takes values is stable (ties keep input order);
 *   - every array is a plain host array owned by the caller;
 *   - functions return 0 on success and a negative number on a bad argument
 *     or failed allocation.
 */
#ifndef RS_ORACLE_H
#define RS_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Structure counters, compared by the tests with the paper's closed forms:
 * rounds of count-sort (Section 3, 32/lg r rounds for 32-bit keys), bitonic
 * stages (lg p (lg p + 1)/2, Section 2 and Eq. Tb), odd-even transposition
 * rounds (p, Section 2 and Eq. To) and merge-split operations. */
typedef struct {
    int64_t rounds;       /* count-sort rounds run by the radix sort        */
    int64_t stages;       /* bitonic stages / odd-even transposition rounds */
    int64_t merge_splits; /* merge-split (or compare-exchange) operations   */
    int64_t local_sorts;  /* local run sorts before a network starts        */
} o_counters;

/* ---- radix sort: Section 3, "Serial radix-r radix-sort" ---------------- */

/* One stable count-sort round on the digit (key >> shift) & (2^bits - 1):
 * count the digits (first read), take the exclusive prefix of the count
 * array, then walk the input in increasing index order writing each key (and
 * value) to the next free slot of its digit (second read and the write).
 * hist, if not NULL, receives the 2^bits digit counts. */
int o_count_round(const uint64_t* keys_in, uint64_t* keys_out,
                  const uint64_t* vals_in, uint64_t* vals_out,
                  size_t n, int shift, int bits, uint64_t* hist);

/* LSD radix sort with radix 2^radix_bits: ceil(8*key_bytes/radix_bits)
 * count-sort rounds from the least significant digit up; the last round
 * takes the remaining high bits.  hists, if not NULL, receives
 * rounds * 2^radix_bits counts (round-major).  vals_in/vals_out may be NULL
 * when val_bytes == 0.  radix_bits in [1, 16]. */
int o_lsd(const void* keys_in, void* keys_out, const void* vals_in,
          void* vals_out, size_t n, int key_bytes, int val_bytes,
          int radix_bits, uint64_t* hists, o_counters* cnt);

/* Number of count-sort rounds the LSD sort runs: ceil(key_bits/radix_bits). */
int o_lsd_rounds(int key_bytes, int radix_bits);

/* ---- merge-split and the two block networks: Section 2 ----------------- */

/* Merge-split of two sorted runs A and B of N keys each: the N smallest keys
 * of A u B go to lo, the N largest to hi, both sorted ascending.  Ties are
 * taken from A first.  lo/hi must not alias A/B. */
int o_merge_split(const uint64_t* A, const uint64_t* B, size_t N,
                  uint64_t* lo, uint64_t* hi);

/* Block bitonic sort (BTN) on p runs, p a power of two >= 1.  Each of the p
 * runs holds N = ceil(n/p) keys (the tail is padded with the largest key
 * value), every run is sorted first (by the LSD radix sort above, radix
 * 2^8), then Batcher's bitonic network on p wires runs with each comparator
 * replaced by a merge-split: lg p (lg p + 1)/2 stages.  The first n keys of
 * the padded result are written to out. */
int o_bitonic_block(const void* in, void* out, size_t n, int key_bytes,
                    size_t p, o_counters* cnt);

/* Block odd-even transposition sort (OET) on p >= 1 runs of N = ceil(n/p)
 * keys (padded as above), each sorted first; then p rounds; round t
 * merge-splits every neighbour pair (i, i+1) with i = t + first_parity
 * (mod 2), the lower-indexed run keeping the smaller half. */
int o_oet_block(const void* in, void* out, size_t n, int key_bytes, size_t p,
                int first_parity, o_counters* cnt);

/* Textbook networks on single keys (the p = n special cases). */
/* Batcher bitonic sorter with compare-exchange on next_pow2(n) wires. */
int o_bitonic(const void* in, void* out, size_t n, int key_bytes,
              o_counters* cnt);
/* Odd-even transposition: n rounds; in round t every position i with
 * i = t + first_parity (mod 2) compares with i+1 and swaps if the former key
 * is strictly greater. */
int o_oet(const void* in, void* out, size_t n, int key_bytes, int first_parity,
          o_counters* cnt);

/* ---- batched segmented sort (extension) -------------------------------- */

/* Sorts each segment [offsets[s], offsets[s+1]) independently with o_lsd at
 * radix 2^radix_bits (keys only).  offsets has S+1 non-decreasing entries,
 * offsets[0] = 0. */
int o_segmented(const void* in, void* out, const int64_t* offsets, size_t S,
                int key_bytes, int radix_bits);

/* ---- checks ------------------------------------------------------------- */

/* 1 if keys[0..n) is non-decreasing, else 0. */
int o_is_sorted(const void* keys, size_t n, int key_bytes);

/* Checks that (keys_out, idx_out) is THE stable sort of keys_in, using
 * idx_out[i] = original index of the i-th output (idx_bytes = 4 or 8):
 *   1. keys_out non-decreasing;
 *   2. idx_out a permutation of 0..n-1;
 *   3. keys_out[i] == keys_in[idx_out[i]];
 *   4. idx_out strictly increasing inside every run of equal keys.
 * Returns 0 if all hold, else the number (1..4) of the first one broken. */
int o_check_stable_kv(const void* keys_in, const void* keys_out,
                      const void* idx_out, size_t n, int key_bytes,
                      int idx_bytes);

/* ---- learned CDF (extension): monotone MLP 1 -> H -> H -> 1 ------------- */

#define O_MLP_H 32
/* Raw parameter vector, in this order:
 *   v1[H]   (layer-1 weights, w1 = softplus(v1))
 *   b1[H]
 *   v2[H*H] (layer-2 weights, row-major [out][in], w2 = softplus(v2))
 *   b2[H]
 *   v3[H]   (output weights, w3 = softplus(v3))
 *   b3[1]
 * h1 = tanh(w1 x + b1); h2 = tanh(w2 h1 + b2); y = sigmoid(w3 . h2 + b3). */
#define O_MLP_NPARAM (O_MLP_H + O_MLP_H + O_MLP_H * O_MLP_H + O_MLP_H + O_MLP_H + 1)

/* Forward pass in double precision. */
double o_mlp_forward_f64(const double* params, double x);

/* Mean squared error over m samples and its gradient with respect to the raw
 * parameters (through the softplus).  Returns the loss; grad may be NULL. */
double o_mlp_loss_grad_f64(const double* params, const double* xs,
                           const double* ts, size_t m, double* grad);

/* One Adam step (Kingma and Ba 2015) on the raw parameters, step number
 * t >= 1, bias-corrected, in double precision. */
void o_adam_step_f64(double* params, const double* grad, double* mom1,
                     double* mom2, size_t np, int64_t t, double lr,
                     double beta1, double beta2, double eps);

/* Forward pass in single precision with a fixed order of operations: used
 * only to report how often the GPU's bucket ids agree with a host
 * evaluation (no parity claim rests on it). */
float o_mlp_forward_f32(const float* params, float x);

/* Mid-rank targets of a sorted sample s[0..m): t_i = (#{s < s_i} +
 * #{s <= s_i}) / (2m). */
int o_midrank_targets(const uint64_t* sorted, size_t m, double* t);

#ifdef __cplusplus
}
#endif
#endif
