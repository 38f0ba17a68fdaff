/*
 * oracle.c -- plain serial C reference (TEST INFRASTRUCTURE ONLY).
 *
 * Written from the paper's definitions: Section 3 ("Serial radix-r
 * radix-sort", Eq. Ts) for the count-sort rounds, Section 2 (the BTN and OET
 * paragraphs) for merge-split, the block bitonic network and the block
 * odd-even transposition sort.  Every key is widened to uint64_t and every
 * value to uint64_t internally so one code path serves all widths.  Nothing
 * here is blocked, fused or reordered beyond the definitions.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* width conversion helpers                                                 */

static uint64_t* widen(const void* a, size_t n, int bytes) {
    uint64_t* w = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!w) return NULL;
    for (size_t i = 0; i < n; i++)
        w[i] = (bytes == 4) ? ((const uint32_t*)a)[i] : ((const uint64_t*)a)[i];
    return w;
}

static void narrow(const uint64_t* w, void* a, size_t n, int bytes) {
    for (size_t i = 0; i < n; i++) {
        if (bytes == 4) ((uint32_t*)a)[i] = (uint32_t)w[i];
        else ((uint64_t*)a)[i] = w[i];
    }
}

static uint64_t key_max(int key_bytes) {
    return key_bytes == 4 ? (uint64_t)UINT32_MAX : UINT64_MAX;
}

/* ------------------------------------------------------------------------ */
/* Section 3: one round of count-sort                                       */

int o_count_round(const uint64_t* keys_in, uint64_t* keys_out,
                  const uint64_t* vals_in, uint64_t* vals_out,
                  size_t n, int shift, int bits, uint64_t* hist) {
    if (bits < 1 || bits > 16 || shift < 0 || shift > 63) return -1;
    size_t r = (size_t)1 << bits;
    uint64_t mask = ((uint64_t)1 << bits) - 1;
    uint64_t* count = (uint64_t*)calloc(r, sizeof(uint64_t));
    if (!count) return -2;
    /* count process: first read of the input */
    for (size_t i = 0; i < n; i++) count[(keys_in[i] >> shift) & mask]++;
    if (hist) memcpy(hist, count, r * sizeof(uint64_t));
    /* exclusive prefix of the count array */
    uint64_t running = 0;
    for (size_t d = 0; d < r; d++) {
        uint64_t c = count[d];
        count[d] = running;
        running += c;
    }
    /* output: second read, in input order, so equal digits keep their order */
    for (size_t i = 0; i < n; i++) {
        uint64_t d = (keys_in[i] >> shift) & mask;
        uint64_t pos = count[d]++;
        keys_out[pos] = keys_in[i];
        if (vals_in) vals_out[pos] = vals_in[i];
    }
    free(count);
    return 0;
}

int o_lsd_rounds(int key_bytes, int radix_bits) {
    int w = 8 * key_bytes;
    return (w + radix_bits - 1) / radix_bits;
}

/* LSD radix sort on widened arrays, in place in k (and v). */
static int lsd_wide(uint64_t* k, uint64_t* v, size_t n, int key_bits,
                    int radix_bits, uint64_t* hists, o_counters* cnt) {
    int rounds = (key_bits + radix_bits - 1) / radix_bits;
    size_t r = (size_t)1 << radix_bits;
    uint64_t* k2 = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* v2 = v ? (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t)) : NULL;
    if (!k2 || (v && !v2)) { free(k2); free(v2); return -2; }
    for (int j = 0; j < rounds; j++) {
        int shift = j * radix_bits;
        int bits = key_bits - shift < radix_bits ? key_bits - shift : radix_bits;
        uint64_t* h = NULL;
        if (hists) {
            h = hists + (size_t)j * r;
            memset(h, 0, r * sizeof(uint64_t));
        }
        int rc = o_count_round(k, k2, v, v2, n, shift, bits, h);
        if (rc) { free(k2); free(v2); return rc; }
        memcpy(k, k2, n * sizeof(uint64_t));
        if (v) memcpy(v, v2, n * sizeof(uint64_t));
        if (cnt) cnt->rounds++;
    }
    free(k2);
    free(v2);
    return 0;
}

int o_lsd(const void* keys_in, void* keys_out, const void* vals_in,
          void* vals_out, size_t n, int key_bytes, int val_bytes,
          int radix_bits, uint64_t* hists, o_counters* cnt) {
    if ((key_bytes != 4 && key_bytes != 8) ||
        (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) ||
        radix_bits < 1 || radix_bits > 16)
        return -1;
    if (val_bytes && (!vals_in || !vals_out)) return -1;
    uint64_t* k = widen(keys_in, n, key_bytes);
    uint64_t* v = val_bytes ? widen(vals_in, n, val_bytes) : NULL;
    if (!k || (val_bytes && !v)) { free(k); free(v); return -2; }
    int rc = lsd_wide(k, v, n, 8 * key_bytes, radix_bits, hists, cnt);
    if (!rc) {
        narrow(k, keys_out, n, key_bytes);
        if (v) narrow(v, vals_out, n, val_bytes);
    }
    free(k);
    free(v);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 2: merge-split, the comparator of the block networks             */

int o_merge_split(const uint64_t* A, const uint64_t* B, size_t N,
                  uint64_t* lo, uint64_t* hi) {
    size_t i = 0, j = 0;
    for (size_t o = 0; o < 2 * N; o++) {
        uint64_t x;
        if (j >= N || (i < N && A[i] <= B[j])) x = A[i++];
        else x = B[j++];
        if (o < N) lo[o] = x;
        else hi[o - N] = x;
    }
    return 0;
}

static int is_pow2(size_t x) { return x && !(x & (x - 1)); }

/* Pad to p runs of N keys with the largest key, sort every run. */
static uint64_t* make_runs(const void* in, size_t n, int key_bytes, size_t p,
                           size_t* N_out, o_counters* cnt) {
    size_t N = (n + p - 1) / p;
    uint64_t* a = (uint64_t*)malloc(((p * N) > 0 ? p * N : 1) * sizeof(uint64_t));
    if (!a) return NULL;
    for (size_t i = 0; i < p * N; i++) {
        if (i < n) a[i] = key_bytes == 4 ? ((const uint32_t*)in)[i] : ((const uint64_t*)in)[i];
        else a[i] = key_max(key_bytes);
    }
    /* the paper sorts each run with the serial radix-2^8 sort before the
       network starts */
    for (size_t r = 0; r < p; r++) {
        if (lsd_wide(a + r * N, NULL, N, 8 * key_bytes, 8, NULL, NULL)) {
            free(a);
            return NULL;
        }
        if (cnt) cnt->local_sorts++;
    }
    *N_out = N;
    return a;
}

/* merge-split of runs i < l; asc: run i keeps the smaller half. */
static int ms_runs(uint64_t* a, size_t N, size_t i, size_t l, int asc,
                   uint64_t* lo, uint64_t* hi) {
    o_merge_split(a + i * N, a + l * N, N, lo, hi);
    memcpy(a + i * N, asc ? lo : hi, N * sizeof(uint64_t));
    memcpy(a + l * N, asc ? hi : lo, N * sizeof(uint64_t));
    return 0;
}

int o_bitonic_block(const void* in, void* out, size_t n, int key_bytes,
                    size_t p, o_counters* cnt) {
    if ((key_bytes != 4 && key_bytes != 8) || !is_pow2(p)) return -1;
    if (n == 0) return 0;
    size_t N;
    uint64_t* a = make_runs(in, n, key_bytes, p, &N, cnt);
    if (!a) return -2;
    uint64_t* lo = (uint64_t*)malloc(N * sizeof(uint64_t));
    uint64_t* hi = (uint64_t*)malloc(N * sizeof(uint64_t));
    if (!lo || !hi) { free(a); free(lo); free(hi); return -2; }
    /* Batcher's bitonic sorter on p wires: for each merge size k and each
       distance j, wire i meets wire i^j; the pair sorts ascending when bit k
       of i is clear.  lg p (lg p + 1)/2 stages in all. */
    for (size_t k = 2; k <= p; k <<= 1) {
        for (size_t j = k >> 1; j >= 1; j >>= 1) {
            for (size_t i = 0; i < p; i++) {
                size_t l = i ^ j;
                if (l > i) {
                    ms_runs(a, N, i, l, (i & k) == 0, lo, hi);
                    if (cnt) cnt->merge_splits++;
                }
            }
            if (cnt) cnt->stages++;
        }
    }
    narrow(a, out, n, key_bytes);
    free(a); free(lo); free(hi);
    return 0;
}

int o_oet_block(const void* in, void* out, size_t n, int key_bytes, size_t p,
                int first_parity, o_counters* cnt) {
    if ((key_bytes != 4 && key_bytes != 8) || p < 1) return -1;
    if (n == 0) return 0;
    size_t N;
    uint64_t* a = make_runs(in, n, key_bytes, p, &N, cnt);
    if (!a) return -2;
    uint64_t* lo = (uint64_t*)malloc(N * sizeof(uint64_t));
    uint64_t* hi = (uint64_t*)malloc(N * sizeof(uint64_t));
    if (!lo || !hi) { free(a); free(lo); free(hi); return -2; }
    for (size_t t = 0; t < p; t++) {
        for (size_t i = (t + (size_t)first_parity) % 2; i + 1 < p; i += 2) {
            ms_runs(a, N, i, i + 1, 1, lo, hi);
            if (cnt) cnt->merge_splits++;
        }
        if (cnt) cnt->stages++;
    }
    narrow(a, out, n, key_bytes);
    free(a); free(lo); free(hi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* textbook networks on single keys                                         */

int o_bitonic(const void* in, void* out, size_t n, int key_bytes,
              o_counters* cnt) {
    if (key_bytes != 4 && key_bytes != 8) return -1;
    if (n == 0) return 0;
    size_t m = 1;
    while (m < n) m <<= 1;
    uint64_t* a = (uint64_t*)malloc(m * sizeof(uint64_t));
    if (!a) return -2;
    for (size_t i = 0; i < m; i++)
        a[i] = i < n ? (key_bytes == 4 ? ((const uint32_t*)in)[i] : ((const uint64_t*)in)[i])
                     : key_max(key_bytes);
    for (size_t k = 2; k <= m; k <<= 1) {
        for (size_t j = k >> 1; j >= 1; j >>= 1) {
            for (size_t i = 0; i < m; i++) {
                size_t l = i ^ j;
                if (l > i) {
                    int asc = (i & k) == 0;
                    if ((asc && a[i] > a[l]) || (!asc && a[i] < a[l])) {
                        uint64_t t = a[i]; a[i] = a[l]; a[l] = t;
                    }
                    if (cnt) cnt->merge_splits++;
                }
            }
            if (cnt) cnt->stages++;
        }
    }
    narrow(a, out, n, key_bytes);
    free(a);
    return 0;
}

int o_oet(const void* in, void* out, size_t n, int key_bytes, int first_parity,
          o_counters* cnt) {
    if (key_bytes != 4 && key_bytes != 8) return -1;
    uint64_t* a = widen(in, n, key_bytes);
    if (!a) return -2;
    for (size_t t = 0; t < n; t++) {
        for (size_t i = (t + (size_t)first_parity) % 2; i + 1 < n; i += 2) {
            if (a[i] > a[i + 1]) { uint64_t x = a[i]; a[i] = a[i + 1]; a[i + 1] = x; }
            if (cnt) cnt->merge_splits++;
        }
        if (cnt) cnt->stages++;
    }
    narrow(a, out, n, key_bytes);
    free(a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* segmented                                                                */

int o_segmented(const void* in, void* out, const int64_t* offsets, size_t S,
                int key_bytes, int radix_bits) {
    if ((key_bytes != 4 && key_bytes != 8) || offsets[0] != 0) return -1;
    for (size_t s = 0; s < S; s++) {
        int64_t b = offsets[s], e = offsets[s + 1];
        if (e < b) return -1;
        const char* src = (const char*)in + (size_t)b * key_bytes;
        char* dst = (char*)out + (size_t)b * key_bytes;
        int rc = o_lsd(src, dst, NULL, NULL, (size_t)(e - b), key_bytes, 0,
                       radix_bits, NULL, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* checks                                                                   */

static uint64_t at(const void* a, size_t i, int bytes) {
    return bytes == 4 ? ((const uint32_t*)a)[i] : ((const uint64_t*)a)[i];
}

int o_is_sorted(const void* keys, size_t n, int key_bytes) {
    for (size_t i = 1; i < n; i++)
        if (at(keys, i - 1, key_bytes) > at(keys, i, key_bytes)) return 0;
    return 1;
}

int o_check_stable_kv(const void* keys_in, const void* keys_out,
                      const void* idx_out, size_t n, int key_bytes,
                      int idx_bytes) {
    if (!o_is_sorted(keys_out, n, key_bytes)) return 1;
    unsigned char* seen = (unsigned char*)calloc(n ? n : 1, 1);
    if (!seen) return -2;
    for (size_t i = 0; i < n; i++) {
        uint64_t x = at(idx_out, i, idx_bytes);
        if (x >= n || seen[x]) { free(seen); return 2; }
        seen[x] = 1;
    }
    free(seen);
    for (size_t i = 0; i < n; i++)
        if (at(keys_out, i, key_bytes) != at(keys_in, at(idx_out, i, idx_bytes), key_bytes))
            return 3;
    for (size_t i = 1; i < n; i++)
        if (at(keys_out, i, key_bytes) == at(keys_out, i - 1, key_bytes) &&
            at(idx_out, i, idx_bytes) <= at(idx_out, i - 1, idx_bytes))
            return 4;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* learned CDF: monotone MLP                                                */

#define H O_MLP_H
#define P_V1 0
#define P_B1 (P_V1 + H)
#define P_V2 (P_B1 + H)
#define P_B2 (P_V2 + H * H)
#define P_V3 (P_B2 + H)
#define P_B3 (P_V3 + H)

static double softplus(double v) { return v > 30.0 ? v : log1p(exp(v)); }
static double dsoftplus(double v) { return 1.0 / (1.0 + exp(-v)); }
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

typedef struct {
    double a1[H], h1[H], a2[H], h2[H], z, y;
} fwd_cache;

static void forward(const double* q, double x, fwd_cache* c) {
    for (int i = 0; i < H; i++) {
        c->a1[i] = softplus(q[P_V1 + i]) * x + q[P_B1 + i];
        c->h1[i] = tanh(c->a1[i]);
    }
    for (int o = 0; o < H; o++) {
        double s = q[P_B2 + o];
        for (int i = 0; i < H; i++) s += softplus(q[P_V2 + o * H + i]) * c->h1[i];
        c->a2[o] = s;
        c->h2[o] = tanh(s);
    }
    double z = q[P_B3];
    for (int i = 0; i < H; i++) z += softplus(q[P_V3 + i]) * c->h2[i];
    c->z = z;
    c->y = sigmoid(z);
}

double o_mlp_forward_f64(const double* params, double x) {
    fwd_cache c;
    forward(params, x, &c);
    return c.y;
}

double o_mlp_loss_grad_f64(const double* q, const double* xs, const double* ts,
                           size_t m, double* grad) {
    if (grad) memset(grad, 0, O_MLP_NPARAM * sizeof(double));
    double loss = 0.0;
    fwd_cache c;
    for (size_t s = 0; s < m; s++) {
        forward(q, xs[s], &c);
        double e = c.y - ts[s];
        loss += e * e;
        if (!grad) continue;
        /* dL/dy for the mean of squared errors */
        double dy = 2.0 * e / (double)m;
        double dz = dy * c.y * (1.0 - c.y);
        grad[P_B3] += dz;
        double dh2[H], da2[H], dh1[H];
        for (int i = 0; i < H; i++) {
            grad[P_V3 + i] += dz * c.h2[i] * dsoftplus(q[P_V3 + i]);
            dh2[i] = dz * softplus(q[P_V3 + i]);
        }
        for (int o = 0; o < H; o++) {
            da2[o] = dh2[o] * (1.0 - c.h2[o] * c.h2[o]);
            grad[P_B2 + o] += da2[o];
        }
        for (int i = 0; i < H; i++) dh1[i] = 0.0;
        for (int o = 0; o < H; o++) {
            for (int i = 0; i < H; i++) {
                double v = q[P_V2 + o * H + i];
                grad[P_V2 + o * H + i] += da2[o] * c.h1[i] * dsoftplus(v);
                dh1[i] += da2[o] * softplus(v);
            }
        }
        for (int i = 0; i < H; i++) {
            double da1 = dh1[i] * (1.0 - c.h1[i] * c.h1[i]);
            grad[P_B1 + i] += da1;
            grad[P_V1 + i] += da1 * xs[s] * dsoftplus(q[P_V1 + i]);
        }
    }
    return loss / (double)(m ? m : 1);
}

void o_adam_step_f64(double* params, const double* grad, double* mom1,
                     double* mom2, size_t np, int64_t t, double lr,
                     double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (size_t i = 0; i < np; i++) {
        mom1[i] = beta1 * mom1[i] + (1.0 - beta1) * grad[i];
        mom2[i] = beta2 * mom2[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = mom1[i] / c1;
        double vh = mom2[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

static float softplusf_(float v) { return v > 20.0f ? v : log1pf(expf(v)); }

float o_mlp_forward_f32(const float* q, float x) {
    float h1[H], h2[H];
    for (int i = 0; i < H; i++) h1[i] = tanhf(fmaf(softplusf_(q[P_V1 + i]), x, q[P_B1 + i]));
    for (int o = 0; o < H; o++) {
        float s = q[P_B2 + o];
        for (int i = 0; i < H; i++) s = fmaf(softplusf_(q[P_V2 + o * H + i]), h1[i], s);
        h2[o] = tanhf(s);
    }
    float z = q[P_B3];
    for (int i = 0; i < H; i++) z = fmaf(softplusf_(q[P_V3 + i]), h2[i], z);
    return 1.0f / (1.0f + expf(-z));
}

int o_midrank_targets(const uint64_t* s, size_t m, double* t) {
    /* for a sorted sample, #{s < s_i} is the index of the first copy of s_i
       and #{s <= s_i} is one past the index of its last copy */
    size_t i = 0;
    while (i < m) {
        size_t j = i;
        while (j + 1 < m && s[j + 1] == s[i]) j++;
        double v = ((double)i + (double)(j + 1)) / (2.0 * (double)m);
        for (size_t k = i; k <= j; k++) t[k] = v;
        i = j + 1;
    }
    return 0;
}
