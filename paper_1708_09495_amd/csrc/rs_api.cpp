// rs_api.cpp -- the extern "C" entry points of librs (declared in
// include/rs.h): argument checks, planning, workspace checks and dispatch to
// the kernels' launchers.  Nothing here waits on the device except
// rs_get_stats.
#include <cmath>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "../../include/rs_learned.h"
#include "rs_internal.hpp"

namespace rs {
namespace {

struct CallState {
    rs_stats stats{};
    hipStream_t stream = nullptr;
    const uint32_t* status = nullptr;   // device status word of the last call
    const uint32_t* skipped = nullptr;  // device mask of skipped rounds (or none)
    bool pending = false;               // stats still need the device's word
};
thread_local CallState g_call;

void begin_call(int algo) {
    (void)hipGetLastError();  // drop an error left by an earlier, unrelated call
    memset(&g_call.stats, 0, sizeof(g_call.stats));
    g_call.stats.algo = algo;
    g_call.stream = nullptr;
    g_call.status = nullptr;
    g_call.skipped = nullptr;
    g_call.pending = false;
}

rs_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return RS_OK;
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0)
        return RS_ERR_WORKSPACE;
    return RS_OK;
}

int default_bits(int bits) { return bits == 0 ? 8 : bits; }

// Keys (and optionally values) through the LSD rounds.
rs_status sort_wide(const void* kin, void* kout, const void* vin, void* vout, size_t n, int kb,
                    int vb, int bits, void* ws, size_t ws_bytes, hipStream_t st) {
    WidePlan p;
    if (!wide_plan(n, kb, vb, bits, &p)) return RS_ERR_UNSUPPORTED;
    begin_call(RS_ALGO_LSD);
    g_call.stats.radix_bits = bits;
    g_call.stats.passes = p.passes;
    g_call.stats.tile_keys = (int64_t)p.tile_keys;
    if (n == 0) return RS_OK;
    rs_status rc = check_ws(ws, ws_bytes, p.total);
    if (rc != RS_OK) return rc;
    rc = wide_run(p, kin, kout, vin, vout, ws, st);
    if (rc == RS_OK) {
        g_call.stream = st;
        g_call.status = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(ws) + p.off_status);
        g_call.pending = true;
    }
    return rc;
}

// skip: rounds whose digit is the same for every key are skipped (decided on
// the device from the all-round histogram).
rs_status sort_lsd(const void* kin, void* kout, const void* vin, void* vout, size_t n, int kb,
                   int vb, int bits, void* ws, size_t ws_bytes, hipStream_t st, bool skip = false,
                   int items = 0) {
    if (bits >= 12) return sort_wide(kin, kout, vin, vout, n, kb, vb, bits, ws, ws_bytes, st);
    LsdPlan p;
    if (!lsd_plan(n, kb, vb, bits, &p, 0, items)) return RS_ERR_UNSUPPORTED;
    p.skip = skip && n < (1ull << 32) && p.passes <= 32;
    begin_call(RS_ALGO_LSD);
    g_call.stats.radix_bits = bits;
    g_call.stats.passes = p.passes;
    g_call.stats.tile_keys = p.tile;
    if (n == 0) return RS_OK;
    rs_status rc = check_ws(ws, ws_bytes, p.total);
    if (rc != RS_OK) return rc;
    rc = lsd_run(p, kin, kout, vin, vout, ws, st);
    if (rc == RS_OK) {
        g_call.stream = st;
        g_call.status = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(ws) + p.off_status);
        if (p.skip)
            g_call.skipped = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(ws) + p.off_status +
                                                               ROUTE_OFFSET);
        g_call.pending = true;
    }
    return rc;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);

// uint64 keys (optional uint64 values) through learned-CDF buckets; small or
// in-place sorts take the LSD rounds (the learned path needs the input
// intact for its fallback).
rs_status sort_learned(const void* kin, void* kout, const void* vin, void* vout, size_t n, int vb,
                       void* ws, size_t ws_bytes, hipStream_t st) {
    if (vb != 0 && vb != 8) return RS_ERR_UNSUPPORTED;
    if (n < (1u << 16) || n >= (1ull << 32) || kin == kout || (vb && vin == vout)) {
        rs_status rc = sort_lsd(kin, kout, vin, vout, n, 8, vb, 8, ws, ws_bytes, st);
        g_call.stats.algo = RS_ALGO_LEARNED;
        g_call.stats.fallback = 1;
        return rc;
    }
    begin_call(RS_ALGO_LEARNED);
    g_call.stats.radix_bits = 8;
    LearnReport rep;
    rs_status rc = learned_run(kin, kout, vin, vout, n, vb, ws, ws_bytes, st, &rep);
    g_call.stats.fallback = rep.fallback;
    g_call.stats.buckets_overflowed = rep.buckets_overflowed;
    g_call.stats.keys_overflowed = rep.keys_overflowed;
    g_call.stats.train_loss = rep.train_loss;
    g_call.stats.device_error = rep.device_error;
    g_call.stats.passes = rep.fallback ? 8 : 2;
    if (rc == RS_OK && rep.err_word) {
        // rs_get_stats reads the word once the stream is done: it also holds
        // the status of the LSD sorts enqueued after the host's last look
        g_call.stream = st;
        g_call.status = rep.err_word;
        g_call.pending = true;
    }
    return rc;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

int64_t network_stages(int algo, int p) {
    int lg = 0;
    while ((1 << lg) < p) ++lg;
    return algo == RS_ALGO_BTN ? (int64_t)lg * (lg + 1) / 2 : (algo == RS_ALGO_OET ? p : 0);
}

// `count` small arrays through BTN / OET / LDS radix.
rs_status sort_small(const uint32_t* in, uint32_t* out, size_t n, size_t count, int algo, int p,
                     hipStream_t st) {
    if (n > SMALL_CAP_U32) return RS_ERR_UNSUPPORTED;
    if (algo == RS_ALGO_AUTO) {
        int c = 0;
        while ((1u << c) < n) ++c;
        algo = tune_table().algo[c];
        if (p == 0 && algo != RS_ALGO_LDS_RADIX) p = tune_table().p[c];
        if (algo != RS_ALGO_LDS_RADIX && !small_valid_p((uint32_t)n, p)) p = 0;
    }
    if (algo == RS_ALGO_BTN || algo == RS_ALGO_OET) {
        if (p == 0) p = small_default_p(algo, (uint32_t)n);
        if (!small_valid_p((uint32_t)n, p)) return RS_ERR_INVALID;
    } else if (algo == RS_ALGO_LDS_RADIX) {
        p = 0;
    } else {
        return RS_ERR_UNSUPPORTED;
    }
    begin_call(algo);
    g_call.stats.runs_p = p;
    g_call.stats.network_stages = network_stages(algo, p);
    if (algo == RS_ALGO_LDS_RADIX) {
        g_call.stats.radix_bits = 8;
        g_call.stats.passes = 4;
    }
    return small_run(algo, in, out, (uint32_t)n, count, p, st);
}

rs_status sort_blocks(const uint32_t* in, uint32_t* out, size_t n, int algo, uint32_t p, void* ws,
                      size_t ws_bytes, hipStream_t st) {
    BlockPlan bp;
    if (!block_plan(n, algo, p, &bp)) return RS_ERR_UNSUPPORTED;
    begin_call(algo);
    g_call.stats.runs_p = (int32_t)p;
    g_call.stats.network_stages = block_stages(algo, p);
    g_call.stats.radix_bits = 8;
    g_call.stats.passes = 4;
    rs_status rc = check_ws(ws, ws_bytes, bp.total);
    if (rc != RS_OK) return rc;
    rc = block_run(bp, algo, in, out, n, tune_table(), ws, st);
    if (rc == RS_OK) {
        g_call.stream = st;
        g_call.status = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(ws) + bp.off_seg +
                                                          bp.seg.off_status);
        g_call.pending = true;
    }
    return rc;
}

rs_status sort_keys_common(const void* kin, void* kout, const void* vin, void* vout, size_t n,
                           int kb, int vb, int bits, rs_algo algo, void* ws, size_t ws_bytes,
                           void* stream) {
    if (kb != 4 && kb != 8) return RS_ERR_INVALID;
    if (vb != 0 && vb != 4 && vb != 8) return RS_ERR_INVALID;
    if (bits < 0 || bits > 16) return RS_ERR_INVALID;
    if (n > 0 && (!kin || !kout)) return RS_ERR_INVALID;
    if (vb && n > 0 && (!vin || !vout)) return RS_ERR_INVALID;
    if (n > 0 && kin != kout && overlaps(kin, n * kb, kout, n * kb)) return RS_ERR_INVALID;
    if (vb && n > 0 && vin != vout && overlaps(vin, n * vb, vout, n * vb)) return RS_ERR_INVALID;
    // keys and values are either both sorted in place or both not: the
    // rounds pick their buffers from the keys alone
    if (vb && n > 0 && (kin == kout) != (vin == vout)) return RS_ERR_INVALID;
    if ((uint64_t)n >= LSD_MAX_N) return RS_ERR_UNSUPPORTED;
    int items = 0;
    lsd_tuned(n, kb, vb, bits, &bits, &items);
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (algo) {
        case RS_ALGO_AUTO:
            return sort_lsd(kin, kout, vin, vout, n, kb, vb, bits, ws, ws_bytes, st, true, items);
        case RS_ALGO_LSD:
            return sort_lsd(kin, kout, vin, vout, n, kb, vb, bits, ws, ws_bytes, st, false, items);
        case RS_ALGO_LEARNED:
            if (kb != 8) return RS_ERR_UNSUPPORTED;
            return sort_learned(kin, kout, vin, vout, n, vb, ws, ws_bytes, st);
        case RS_ALGO_BTN:
        case RS_ALGO_OET:
        case RS_ALGO_LDS_RADIX:
            if (kb != 4 || vb != 0) return RS_ERR_UNSUPPORTED;
            if (algo != RS_ALGO_LDS_RADIX && n > SMALL_CAP_U32)
                return sort_blocks(static_cast<const uint32_t*>(kin), static_cast<uint32_t*>(kout), n, algo,
                                   block_default_p(n, algo), ws, ws_bytes, st);
            return sort_small(static_cast<const uint32_t*>(kin), static_cast<uint32_t*>(kout), n, 1,
                              algo, 0, st);
        default:
            return RS_ERR_UNSUPPORTED;
    }
}

}  // namespace

rs_status hip_fail(hipError_t e) {
    g_call.stats.hip_error = (int32_t)e;
    return RS_ERR_HIP;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_sort_u32(const uint32_t* in, uint32_t* out, size_t n, int radix_bits, rs_algo algo,
                      void* ws, size_t ws_bytes, void* stream) {
    return sort_keys_common(in, out, nullptr, nullptr, n, 4, 0, radix_bits, algo, ws, ws_bytes,
                            stream);
}

rs_status rs_sort_u64(const uint64_t* in, uint64_t* out, size_t n, int radix_bits, rs_algo algo,
                      void* ws, size_t ws_bytes, void* stream) {
    return sort_keys_common(in, out, nullptr, nullptr, n, 8, 0, radix_bits, algo, ws, ws_bytes,
                            stream);
}

rs_status rs_sort_kv(const void* keys_in, const void* vals_in, void* keys_out, void* vals_out,
                     size_t n, int key_bytes, int val_bytes, int radix_bits, rs_algo algo,
                     void* ws, size_t ws_bytes, void* stream) {
    if (val_bytes != 4 && val_bytes != 8) return RS_ERR_INVALID;
    return sort_keys_common(keys_in, keys_out, vals_in, vals_out, n, key_bytes, val_bytes,
                            radix_bits, algo, ws, ws_bytes, stream);
}

rs_status rs_sort_blocks_u32(const uint32_t* in, uint32_t* out, size_t n, rs_algo algo, int p, void* ws,
                             size_t ws_bytes, void* stream) {
    if (n > 0 && (!in || !out)) return RS_ERR_INVALID;
    if (n > 0 && in != out && overlaps(in, n * 4, out, n * 4)) return RS_ERR_INVALID;
    if (algo != RS_ALGO_BTN && algo != RS_ALGO_OET) return RS_ERR_UNSUPPORTED;
    if (p < 0 || p == 1 || p > 4096) return RS_ERR_INVALID;
    if (algo == RS_ALGO_BTN && p > 0 && (p & (p - 1))) return RS_ERR_INVALID;
    if (n == 0) {
        begin_call(algo);
        return RS_OK;
    }
    const uint32_t pp = p ? (uint32_t)p : block_default_p(n, algo);
    return sort_blocks(in, out, n, algo, pp, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

rs_status rs_blocks_set_model(const rs_block_model* m) {
    if (!m) return RS_ERR_INVALID;
    const bool ok = std::isfinite(m->local_ns_per_key) && std::isfinite(m->stage_ps_per_key) &&
                    std::isfinite(m->stage_fixed_us) && m->local_ns_per_key > 0.0 &&
                    m->stage_ps_per_key >= 0.0 && m->stage_fixed_us >= 0.0 && m->resident_runs >= 1;
    if (!ok) return RS_ERR_INVALID;
    block_model_set(*m);
    return RS_OK;
}

rs_status rs_blocks_get_model(rs_block_model* out) {
    if (!out) return RS_ERR_INVALID;
    *out = block_model();
    return RS_OK;
}

int32_t rs_blocks_default_p(size_t n, rs_algo algo) {
    if ((algo != RS_ALGO_BTN && algo != RS_ALGO_OET) || n == 0) return 0;
    return (int32_t)block_default_p(n, algo);
}

rs_status rs_sort_batch_u32(const uint32_t* in, uint32_t* out, size_t n, size_t count, rs_algo algo,
                            int p, void* ws, size_t ws_bytes, void* stream) {
    (void)ws;
    (void)ws_bytes;
    if (n > 0 && count > 0 && (!in || !out)) return RS_ERR_INVALID;
    if (count > 0x7FFFFFFFu) return RS_ERR_UNSUPPORTED;
    if (n > 0 && count > 0 && in != out && overlaps(in, n * count * 4, out, n * count * 4))
        return RS_ERR_INVALID;
    if (p < 0) return RS_ERR_INVALID;
    return sort_small(in, out, n, count, algo, p, static_cast<hipStream_t>(stream));
}

rs_status rs_sort_segmented(const uint32_t* in, uint32_t* out, const int64_t* offsets,
                            size_t num_segments, int64_t total_n, rs_algo algo, void* ws,
                            size_t ws_bytes, void* stream) {
    if (total_n < 0) return RS_ERR_INVALID;
    if (num_segments > 0 && !offsets) return RS_ERR_INVALID;
    if (total_n > 0 && (!in || !out)) return RS_ERR_INVALID;
    if (total_n > 0 && in != out && overlaps(in, (size_t)total_n * 4, out, (size_t)total_n * 4))
        return RS_ERR_INVALID;
    if (algo != RS_ALGO_AUTO && algo != RS_ALGO_BTN && algo != RS_ALGO_OET &&
        algo != RS_ALGO_LDS_RADIX && algo != RS_ALGO_LSD)
        return RS_ERR_UNSUPPORTED;
    SegPlan p;
    if (!seg_plan(num_segments, total_n, &p, algo != RS_ALGO_LSD)) return RS_ERR_UNSUPPORTED;
    begin_call(algo);
    g_call.stats.radix_bits = 8;
    g_call.stats.passes = 4;
    if (num_segments == 0) return RS_OK;
    rs_status rc = check_ws(ws, ws_bytes, p.total);
    if (rc != RS_OK) return rc;
    SegTable t = tune_table();
    if (algo != RS_ALGO_AUTO && algo != RS_ALGO_LSD)
        for (int c = 0; c < 64; ++c) {
            t.algo[c] = (int8_t)algo;
            const int npad = c < 15 ? (1 << c) : 16384;
            t.p[c] = (int16_t)small_default_p(algo, (uint32_t)npad);
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = seg_run(p, in, out, offsets, num_segments, total_n, t, ws, st);
    if (rc == RS_OK) {
        g_call.stream = st;
        g_call.status = reinterpret_cast<const uint32_t*>(static_cast<unsigned char*>(ws) + p.off_status);
        g_call.pending = true;
    }
    return rc;
}

size_t rs_workspace_bytes(int op, size_t n, int key_bytes, int val_bytes, int radix_bits,
                          rs_algo algo, size_t num_segments) {
    (void)algo;
    (void)num_segments;
    const int raw_bits = radix_bits;
    radix_bits = default_bits(radix_bits);
    if (op == RS_OP_SORT || op == RS_OP_SORT_KV) {
        if ((algo == RS_ALGO_BTN || algo == RS_ALGO_OET) && op == RS_OP_SORT && key_bytes == 4 &&
            n > SMALL_CAP_U32) {
            BlockPlan bp;
            return block_plan(n, algo, block_default_p(n, algo), &bp) ? bp.total : 0;
        }
        if (algo == RS_ALGO_BTN || algo == RS_ALGO_OET || algo == RS_ALGO_LDS_RADIX) return ALIGN;
        if (algo == RS_ALGO_LEARNED && key_bytes == 8) {
            const int vb = op == RS_OP_SORT ? 0 : val_bytes;
            LsdPlan p;
            if (!lsd_plan(n, 8, vb, 8, &p)) return 0;
            const size_t l = (n >= (1u << 16) && n < (1ull << 32)) ? learned_ws_bytes(n, vb) : 0;
            return l > p.total ? l : p.total;
        }
        const int vb = op == RS_OP_SORT ? 0 : val_bytes;
        int bits = 0, items = 0;
        lsd_tuned(n, key_bytes, vb, raw_bits, &bits, &items);
        if (bits >= 12) {
            WidePlan w;
            return wide_plan(n, key_bytes, vb, bits, &w) ? w.total : 0;
        }
        LsdPlan p;
        if (!lsd_plan(n, key_bytes, vb, bits, &p, 0, items)) return 0;
        return p.total;
    }
    if (op == RS_OP_BATCH) return ALIGN;
    if (op == RS_OP_TUNE) return (n >= 1 && n <= 65536) ? tune_ws_bytes((int)n) : 0;
    if (op == RS_OP_BLOCKS) {
        if (key_bytes != 4 || n == 0 || num_segments > 4096) return n == 0 ? ALIGN : 0;
        const uint32_t p = num_segments ? (uint32_t)num_segments : block_default_p(n, algo);
        BlockPlan bp;
        return block_plan(n, algo, p, &bp) ? bp.total : 0;
    }
    if (op == RS_OP_SEGMENTED) {
        SegPlan p;
        if ((int64_t)n < 0 || !seg_plan(num_segments, (int64_t)n, &p, algo != RS_ALGO_LSD)) return 0;
        return p.total;
    }
    return 0;
}

size_t rs_small_capacity(int key_bytes) {
    return key_bytes == 4 ? 16384 : (key_bytes == 8 ? 8192 : 0);
}

const char* rs_status_string(rs_status s) {
    // C callers may pass any int: read it as one rather than as the enum
    int v;
    memcpy(&v, &s, sizeof v);
    switch (v) {
        case RS_OK: return "ok";
        case RS_ERR_INVALID: return "invalid argument";
        case RS_ERR_UNSUPPORTED: return "unsupported request";
        case RS_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case RS_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

rs_status rs_get_stats(rs_stats* out) {
    if (!out) return RS_ERR_INVALID;
    if (g_call.pending) {
        uint32_t word = 0;
        hipError_t e = hipStreamSynchronize(g_call.stream);
        if (e == hipSuccess) e = hipMemcpy(&word, g_call.status, sizeof(word), hipMemcpyDeviceToHost);
        uint32_t mask = 0;
        if (e == hipSuccess && g_call.skipped)
            e = hipMemcpy(&mask, g_call.skipped, sizeof(mask), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e);
        g_call.stats.device_error = word;
        g_call.stats.passes_skipped = __builtin_popcount(mask);
        g_call.pending = false;
    }
    *out = g_call.stats;
    return RS_OK;
}

}  // extern "C"

// ---- learned path: options and network entry points --------------------------

extern "C" rs_status rs_learned_set_opts(const rs_learned_opts* o) {
    if (!o || o->train_steps < 0 || o->train_steps > 100000 || !(o->lr > 0.f) || o->bucket_cap < 2 ||
        o->feature_mode < -1 || o->feature_mode > 2 || o->fallback_frac < 0.0 || o->train_blocks < 1 ||
        o->train_blocks > 4096 || o->max_fallback_buckets < 0)
        return RS_ERR_INVALID;
    rs::LearnOpts& d = rs::learn_opts();
    d.train_steps = o->train_steps;
    d.lr = o->lr;
    d.use_network = o->use_network ? 1 : 0;
    d.bucket_cap = o->bucket_cap;
    d.feature_mode = o->feature_mode;
    d.fallback_frac = o->fallback_frac;
    d.train_blocks = o->train_blocks;
    d.max_fallback_buckets = o->max_fallback_buckets;
    return RS_OK;
}

extern "C" rs_status rs_learned_get_opts(rs_learned_opts* o) {
    if (!o) return RS_ERR_INVALID;
    const rs::LearnOpts& d = rs::learn_opts();
    o->train_steps = d.train_steps;
    o->lr = d.lr;
    o->use_network = d.use_network;
    o->bucket_cap = d.bucket_cap;
    o->feature_mode = d.feature_mode;
    o->fallback_frac = d.fallback_frac;
    o->train_blocks = d.train_blocks;
    o->max_fallback_buckets = d.max_fallback_buckets;
    return RS_OK;
}

extern "C" size_t rs_mlp_num_params(void) { return rs::MLP_NPARAM; }

extern "C" rs_status rs_mlp_forward(const float* params, const float* x, float* y, size_t m, void* stream) {
    if (m && (!params || !x || !y)) return RS_ERR_INVALID;
    (void)hipGetLastError();
    return rs::mlp_forward(params, x, y, m, static_cast<hipStream_t>(stream));
}

extern "C" rs_status rs_mlp_loss_grad(const float* params, const float* x, const float* t, size_t m,
                                      float* grad, void* stream) {
    if (!m || !params || !x || !t || !grad) return RS_ERR_INVALID;
    (void)hipGetLastError();
    return rs::mlp_loss_grad(params, x, t, m, grad, static_cast<hipStream_t>(stream));
}

extern "C" rs_status rs_mlp_adam_step(float* params, float* m1, float* m2, const float* grad, int32_t step,
                                      float lr, float beta1, float beta2, float eps, void* stream) {
    if (!params || !m1 || !m2 || !grad || step < 0) return RS_ERR_INVALID;
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return RS_ERR_INVALID;
    (void)hipGetLastError();
    return rs::mlp_adam_step(params, m1, m2, grad, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
}

extern "C" rs_status rs_mlp_set_weights(const float* params, size_t count) {
    return rs::learned_inject_weights(params, count);
}

extern "C" rs_status rs_learned_debug_fault(int kind, const uint64_t* splitters, size_t count) {
    return rs::learned_inject_fault(kind, splitters, count);
}

extern "C" rs_status rs_learned_debug_ids(uint16_t* direct, uint16_t* assigned) {
    return rs::learned_debug_ids(direct, assigned);
}

// ---- tuning table -----------------------------------------------------------

namespace rs {
namespace {
SegTable default_table() {
    SegTable d{};
    for (int c = 0; c < 64; ++c) {
        const uint32_t npad = c < 15 ? (1u << c) : 16384u;
        d.algo[c] = (int8_t)RS_ALGO_BTN;
        d.p[c] = (int16_t)small_default_p(RS_ALGO_BTN, npad);
    }
    return d;
}
rs_status load_table(const char* path, SegTable* t);
}  // namespace

// The process-wide table: defaults, then RS_TUNING_FILE if it names a table
// written for this device (same gfx architecture and compute unit count).
SegTable& tune_table() {
    static SegTable t = [] {
        SegTable d = default_table();
        if (const char* f = getenv("RS_TUNING_FILE"))
            if (*f) (void)load_table(f, &d);
        return d;
    }();
    return t;
}

void lsd_tuned(size_t n, int kb, int vb, int radix_bits, int* bits, int* items) {
    int c = 0;
    while (c < 63 && (1ull << c) < (unsigned long long)n) ++c;
    const SegTable& t = tune_table();
    const bool u32k = kb == 4 && vb == 0;
    int b = radix_bits;
    if (b == 0) b = (u32k && t.radix[c] > 0) ? t.radix[c] : 8;
    *bits = b;
    *items = (u32k && b <= 8) ? t.items[c] : 0;
}

namespace {
bool entry_ok(const rs_tune_entry& e) {
    const int c = e.size_log2;
    if (c < 0 || c >= TUNE_CLASSES) return false;
    if (c <= 14) {
        if (e.algo != RS_ALGO_BTN && e.algo != RS_ALGO_OET && e.algo != RS_ALGO_LDS_RADIX) return false;
        if (e.algo != RS_ALGO_LDS_RADIX && !small_valid_p(1u << c, e.p)) return false;
    } else if (e.algo != 0 || e.p != 0) {
        return false;  // no small-array choice above one workgroup's capacity
    }
    if (e.radix_bits < 0 || e.radix_bits > 16) return false;
    if (e.tile_items != 0 && e.tile_items != 8 && e.tile_items != 16 && e.tile_items != 28) return false;
    if (e.seg_tile_items != 0 && e.seg_tile_items != 8 && e.seg_tile_items != 16) return false;
    return true;
}

void put_entry(SegTable& t, const rs_tune_entry& e) {
    const int c = e.size_log2;
    if (c <= 14) {
        t.algo[c] = (int8_t)e.algo;
        t.p[c] = (int16_t)e.p;
    }
    t.radix[c] = (int8_t)e.radix_bits;
    t.items[c] = (int8_t)e.tile_items;
    t.seg_items[c] = (int8_t)e.seg_tile_items;
}

rs_tune_entry get_entry(const SegTable& t, int c) {
    rs_tune_entry e{};
    e.size_log2 = c;
    e.algo = c <= 14 ? t.algo[c] : 0;
    e.p = c <= 14 ? t.p[c] : 0;
    e.radix_bits = t.radix[c];
    e.tile_items = t.items[c];
    e.seg_tile_items = t.seg_items[c];
    return e;
}

// The current device's architecture name and compute unit count.
rs_status device_key(char* arch, size_t cap, int* cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e);
    snprintf(arch, cap, "%s", prop.gcnArchName);
    *cus = prop.multiProcessorCount;
    return RS_OK;
}

// ---- a small JSON reader for the tuning file: objects, arrays, strings
//      without escapes other than \" and \\, integers
struct JReader {
    const char* p;
    const char* end;
    bool ok = true;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool eat(char c) {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string* out) {
        ws();
        if (p >= end || *p != '"') return ok = false;
        ++p;
        out->clear();
        while (p < end && *p != '"') {
            if (*p == '\\' && p + 1 < end) ++p;
            out->push_back(*p++);
        }
        if (p >= end) return ok = false;
        ++p;
        return true;
    }
    bool num(long long* out) {
        ws();
        const char* q = p;
        if (q < end && *q == '-') ++q;
        if (q >= end || *q < '0' || *q > '9') return ok = false;
        long long v = 0;
        while (q < end && *q >= '0' && *q <= '9' && v < (1ll << 50)) v = v * 10 + (*q++ - '0');
        *out = (*p == '-') ? -v : v;
        p = q;
        return true;
    }
};

rs_status load_table(const char* path, SegTable* t) {
    FILE* f = fopen(path, "rb");
    if (!f) return RS_ERR_INVALID;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 20)) text.append(buf, got);
    fclose(f);
    JReader r{text.data(), text.data() + text.size()};
    std::string key, arch, fmt;
    long long cus = -1;
    SegTable nt = default_table();
    bool have_classes = false;
    if (!r.eat('{')) return RS_ERR_INVALID;
    while (r.ok && !r.eat('}')) {
        if (!r.str(&key) || !r.eat(':')) return RS_ERR_INVALID;
        if (key == "format") {
            if (!r.str(&fmt)) return RS_ERR_INVALID;
        } else if (key == "arch") {
            if (!r.str(&arch)) return RS_ERR_INVALID;
        } else if (key == "cus") {
            if (!r.num(&cus)) return RS_ERR_INVALID;
        } else if (key == "classes") {
            if (!r.eat('[')) return RS_ERR_INVALID;
            have_classes = true;
            while (r.ok && !r.eat(']')) {
                rs_tune_entry e{};
                if (!r.eat('{')) return RS_ERR_INVALID;
                while (r.ok && !r.eat('}')) {
                    long long v = 0;
                    if (!r.str(&key) || !r.eat(':') || !r.num(&v)) return RS_ERR_INVALID;
                    if (v < -(1ll << 30) || v > (1ll << 30)) return RS_ERR_INVALID;
                    if (key == "size_log2") e.size_log2 = (int32_t)v;
                    else if (key == "algo") e.algo = (int32_t)v;
                    else if (key == "p") e.p = (int32_t)v;
                    else if (key == "radix_bits") e.radix_bits = (int32_t)v;
                    else if (key == "tile_items") e.tile_items = (int32_t)v;
                    else if (key == "seg_tile_items") e.seg_tile_items = (int32_t)v;
                    else return RS_ERR_INVALID;
                    r.eat(',');
                }
                if (!entry_ok(e)) return RS_ERR_INVALID;
                put_entry(nt, e);
                r.eat(',');
            }
        } else {
            return RS_ERR_INVALID;
        }
        r.eat(',');
    }
    if (!r.ok || fmt != "rs-tuning-1" || arch.empty() || cus < 1 || !have_classes) return RS_ERR_INVALID;
    char darch[256];
    int dcus = 0;
    rs_status rc = device_key(darch, sizeof darch, &dcus);
    if (rc != RS_OK) return rc;
    if (arch != darch || cus != dcus) return RS_ERR_UNSUPPORTED;
    *t = nt;
    return RS_OK;
}
}  // namespace
}  // namespace rs

extern "C" rs_status rs_tune_set(const rs_tune_entry* e, int count) {
    if (count < 0 || (count > 0 && !e)) return RS_ERR_INVALID;
    for (int i = 0; i < count; ++i)
        if (!rs::entry_ok(e[i])) return RS_ERR_INVALID;
    rs::SegTable& t = rs::tune_table();
    for (int i = 0; i < count; ++i) rs::put_entry(t, e[i]);
    return RS_OK;
}

extern "C" int rs_tune_get(rs_tune_entry* out, int max) {
    if (!out || max <= 0) return 0;
    const rs::SegTable& t = rs::tune_table();
    int k = 0;
    for (int c = 0; c < rs::TUNE_CLASSES && k < max; ++c, ++k) out[k] = rs::get_entry(t, c);
    return k;
}

extern "C" rs_status rs_tune_save(const char* path) {
    if (!path || !*path) return RS_ERR_INVALID;
    char arch[256];
    int cus = 0;
    rs_status rc = rs::device_key(arch, sizeof arch, &cus);
    if (rc != RS_OK) return rc;
    for (const char* q = arch; *q; ++q)
        if (*q == '"' || *q == '\\') return RS_ERR_UNSUPPORTED;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return RS_ERR_INVALID;
    const rs::SegTable& t = rs::tune_table();
    bool ok = fprintf(f, "{\"format\": \"rs-tuning-1\", \"arch\": \"%s\", \"cus\": %d,\n \"classes\": [\n", arch,
                      cus) > 0;
    for (int c = 0; c < rs::TUNE_CLASSES && ok; ++c) {
        const rs_tune_entry e = rs::get_entry(t, c);
        ok = fprintf(f,
                     "  {\"size_log2\": %d, \"algo\": %d, \"p\": %d, \"radix_bits\": %d, \"tile_items\": %d, "
                     "\"seg_tile_items\": %d}%s\n",
                     e.size_log2, e.algo, e.p, e.radix_bits, e.tile_items, e.seg_tile_items,
                     c + 1 < rs::TUNE_CLASSES ? "," : "") > 0;
    }
    ok = ok && fprintf(f, " ]}\n") > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return RS_ERR_INVALID;
    }
    return RS_OK;
}

extern "C" rs_status rs_tune_load(const char* path) {
    if (!path || !*path) return RS_ERR_INVALID;
    rs::SegTable t;
    rs_status rc = rs::load_table(path, &t);
    if (rc == RS_OK) rs::tune_table() = t;
    return rc;
}

// ---- kernel timing --------------------------------------------------------
#include <mutex>
#include <vector>

namespace rs {
bool g_prof_on = false;
thread_local bool g_prof_muted = false;
namespace {
const char* const KNAMES[KID_COUNT_] = {
    "fill", "hist", "onesweep", "copy", "batch", "seg_plan", "seg",
    "learn_sample", "learn_train", "learn_split", "learn_assign", "learn_bucket", "learn_check",
    "wide_count", "wide_scatter", "learn_pass", "learn_mid", "block_merge", "stream_copy", "seg_round"};
struct Mark {
    int kid;
    hipEvent_t b, e;
};
std::mutex g_prof_mu;
std::vector<Mark> g_marks;
std::vector<hipEvent_t> g_free_events;
hipEvent_t take_event() {
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void prof_record(hipStream_t st, int kid, int phase) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (phase == 0) {
        Mark m{kid, take_event(), nullptr};
        if (m.b && hipEventRecord(m.b, st) != hipSuccess) {  // left out of the timings
            g_free_events.push_back(m.b);
            m.b = nullptr;
        }
        g_marks.push_back(m);
    } else {
        for (auto it = g_marks.rbegin(); it != g_marks.rend(); ++it) {
            if (it->kid == kid && it->e == nullptr) {
                it->e = take_event();
                if (it->e && hipEventRecord(it->e, st) != hipSuccess) {
                    g_free_events.push_back(it->e);
                    it->e = nullptr;
                }
                break;
            }
        }
    }
}
}  // namespace rs

extern "C" rs_status rs_stream_copy(const void* in, void* out, size_t bytes, void* stream) {
    if (bytes && (!in || !out)) return RS_ERR_INVALID;
    if (bytes && in != out && rs::overlaps(in, bytes, out, bytes)) return RS_ERR_INVALID;
    (void)hipGetLastError();
    return rs::stream_copy(in, out, bytes, static_cast<hipStream_t>(stream));
}

extern "C" rs_status rs_profile_enable(int on) {
    rs::g_prof_on = on != 0;
    return RS_OK;
}

extern "C" int rs_profile_read(rs_kernel_time* out, int max) {
    using namespace rs;
    std::lock_guard<std::mutex> g(g_prof_mu);
    double tot[KID_COUNT_] = {0};
    int64_t cnt[KID_COUNT_] = {0};
    int rc = 0;
    for (auto& m : g_marks) {
        if (m.b && m.e) {
            if (hipEventSynchronize(m.e) != hipSuccess) rc = -1;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, m.b, m.e) != hipSuccess) rc = -1;
            tot[m.kid] += ms;
            cnt[m.kid] += 1;
        }
        if (m.b) g_free_events.push_back(m.b);
        if (m.e) g_free_events.push_back(m.e);
    }
    g_marks.clear();
    if (rc) return -1;
    int k = 0;
    for (int i = 0; i < KID_COUNT_ && k < max; ++i) {
        if (!cnt[i]) continue;
        memset(out[k].name, 0, sizeof(out[k].name));
        strncpy(out[k].name, KNAMES[i], sizeof(out[k].name) - 1);
        out[k].launches = cnt[i];
        out[k].total_ms = tot[i];
        ++k;
    }
    return k;
}

// ---- sorting without allocation ----------------------------------------------
//
// rs_sort_u32_noalloc takes its scratch from `scratch`, a static device array
// of the library's code object: every device the library runs on holds its
// own copy until the process ends.  In host code the array's name is only a
// host-side stand-in; the device address comes from hipGetSymbolAddress,
// looked up once per device (with that device current) and kept.
namespace rs {
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(40) << 20;
constexpr size_t NOALLOC_MAX_KEYS = size_t(1) << 22;
constexpr int NOALLOC_MAX_DEVICES = 64;
static_assert(NOALLOC_SCRATCH_BYTES == (size_t)RS_NOALLOC_SCRATCH_BYTES &&
                  NOALLOC_MAX_KEYS == (size_t)RS_NOALLOC_MAX_KEYS,
              "the header states the same limits");
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
rs_status scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return RS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p || (reinterpret_cast<uintptr_t>(p) % ALIGN) != 0) return RS_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RS_OK;
}
}  // namespace
}  // namespace rs

extern "C" rs_status rs_sort_u32_noalloc(const uint32_t* in, uint32_t* out, size_t n, int radix_bits,
                                         rs_algo algo, void* stream) {
    using namespace rs;
    if (radix_bits < 0 || radix_bits > 16) return RS_ERR_INVALID;
    if (algo != RS_ALGO_LSD && algo != RS_ALGO_AUTO) return RS_ERR_UNSUPPORTED;
    if (n > NOALLOC_MAX_KEYS || radix_bits > 11) return RS_ERR_UNSUPPORTED;
    if (n > 0 && (!in || !out)) return RS_ERR_INVALID;
    if (n == 0) return sort_keys_common(in, out, nullptr, nullptr, 0, 4, 0, radix_bits, algo, nullptr, 0, stream);
    int bits = 0, items = 0;
    lsd_tuned(n, 4, 0, radix_bits, &bits, &items);
    LsdPlan plan;
    if (bits > 11 || !lsd_plan(n, 4, 0, bits, &plan, 0, items) || plan.total > NOALLOC_SCRATCH_BYTES)
        return RS_ERR_UNSUPPORTED;
    // the stream must belong to the current device, whose scratch is used
    if (stream) {
        int cur = -1, sdev = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess) e = hipStreamGetDevice(static_cast<hipStream_t>(stream), &sdev);
        if (e != hipSuccess) return hip_fail(e);
        if (sdev != cur) return RS_ERR_INVALID;
    }
    void* ws = nullptr;
    rs_status rc = scratch_of_current_device(&ws);
    if (rc != RS_OK) return rc;
    // no timing events either: creating one may allocate
    g_prof_muted = true;
    rc = sort_keys_common(in, out, nullptr, nullptr, n, 4, 0, radix_bits, algo, ws, NOALLOC_SCRATCH_BYTES,
                          stream);
    g_prof_muted = false;
    return rc;
}
