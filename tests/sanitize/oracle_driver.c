/* Exercises the oracle under AddressSanitizer / UndefinedBehaviorSanitizer
 * (built by tests/test_sanitizers.py): every sort on random small inputs,
 * checked against qsort; exits non-zero on a mismatch (a sanitizer report
 * aborts the process by itself). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static uint64_t state = 0x1708ull;
static uint64_t next(void) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int cmp32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : x > y;
}
static int cmp64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

int main(void) {
    int bad = 0;
    for (int trial = 0; trial < 200; ++trial) {
        size_t n = (size_t)(next() % 700);
        const int kb = (trial & 1) ? 8 : 4;
        const uint64_t range = (trial % 3 == 0) ? 5 : ~0ull;
        void* in = malloc(n * kb + 1);
        void* out = malloc(n * kb + 1);
        void* ref = malloc(n * kb + 1);
        uint64_t* vals = malloc(n * 8 + 8);
        uint64_t* vout = malloc(n * 8 + 8);
        for (size_t i = 0; i < n; ++i) {
            const uint64_t v = range == ~0ull ? next() : next() % range;
            if (kb == 4) ((uint32_t*)in)[i] = (uint32_t)v;
            else ((uint64_t*)in)[i] = v;
            vals[i] = i;
        }
        memcpy(ref, in, n * kb);
        qsort(ref, n, kb, kb == 4 ? cmp32 : cmp64);
        const int bits = 1 + (int)(next() % 16);
        o_counters c;
        if (o_lsd(in, out, vals, vout, n, kb, 8, bits, NULL, &c) != 0 || memcmp(out, ref, n * kb)) bad |= 1;
        if (n && o_check_stable_kv(in, out, vout, n, kb, 8) != 0) bad |= 2;
        const size_t p = (size_t)1 << (next() % 6);
        if (o_bitonic_block(in, out, n, kb, p, &c) != 0 || memcmp(out, ref, n * kb)) bad |= 4;
        if (o_oet_block(in, out, n, kb, 1 + next() % 9, (int)(next() & 1), &c) != 0 || memcmp(out, ref, n * kb))
            bad |= 8;
        if (n <= 64) {
            if (o_bitonic(in, out, n, kb, &c) != 0 || memcmp(out, ref, n * kb)) bad |= 16;
            if (o_oet(in, out, n, kb, 0, &c) != 0 || memcmp(out, ref, n * kb)) bad |= 32;
        }
        if (kb == 4) {
            int64_t off[4] = {0, (int64_t)(n / 3), (int64_t)(n / 2), (int64_t)n};
            if (o_segmented(in, out, off, 3, 4, 8) != 0) bad |= 64;
            for (int s = 0; s < 3; ++s) {
                const size_t a = (size_t)off[s], z = (size_t)off[s + 1];
                memcpy((uint32_t*)ref + a, (uint32_t*)in + a, (z - a) * 4);
                qsort((uint32_t*)ref + a, z - a, 4, cmp32);
            }
            if (memcmp(out, ref, n * 4)) bad |= 64;
        }
        free(in);
        free(out);
        free(ref);
        free(vals);
        free(vout);
    }
    double q[O_MLP_NPARAM], g[O_MLP_NPARAM], m1[O_MLP_NPARAM] = {0}, m2[O_MLP_NPARAM] = {0};
    double xs[37], ts[37];
    for (int i = 0; i < O_MLP_NPARAM; ++i) q[i] = (double)(next() % 2001) / 1000.0 - 1.0;
    for (int i = 0; i < 37; ++i) {
        xs[i] = (double)(next() % 1001) / 1000.0;
        ts[i] = (double)(next() % 1001) / 1000.0;
    }
    const double loss = o_mlp_loss_grad_f64(q, xs, ts, 37, g);
    o_adam_step_f64(q, g, m1, m2, O_MLP_NPARAM, 1, 1e-2, 0.9, 0.999, 1e-8);
    float qf[O_MLP_NPARAM];
    for (int i = 0; i < O_MLP_NPARAM; ++i) qf[i] = (float)q[i];
    const float y = o_mlp_forward_f32(qf, 0.5f);
    uint64_t srt[50];
    double tg[50];
    for (int i = 0; i < 50; ++i) srt[i] = (uint64_t)(i / 3);
    if (o_midrank_targets(srt, 50, tg) != 0) bad |= 128;
    if (!(loss >= 0.0) || !(y >= 0.f && y <= 1.f)) bad |= 256;
    if (bad) fprintf(stderr, "oracle driver: failures 0x%x\n", bad);
    else printf("oracle driver: ok\n");
    return bad ? 1 : 0;
}
