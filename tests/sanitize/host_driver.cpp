// Exercises the host side of librs under AddressSanitizer /
// UndefinedBehaviorSanitizer with no GPU (built by tests/test_sanitizers.py
// from the library's sources, host code instrumented): argument checks,
// workspace sizing over many shapes, the tuning table and its JSON reader
// on well-formed, truncated and corrupted files, the learned-path options
// and the block model.  Exits non-zero when a call returns something other
// than documented; a sanitizer report aborts the process by itself.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "../../include/rs.h"
#include "../../include/rs_learned.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "host driver: line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                \
        }                                                              \
    } while (0)

static std::string write_file(const char* dir, const std::string& text, int k) {
    std::string path = std::string(dir) + "/t" + std::to_string(k) + ".json";
    FILE* f = fopen(path.c_str(), "wb");
    if (f) {
        fwrite(text.data(), 1, text.size(), f);
        fclose(f);
    }
    return path;
}

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : "/tmp";
    void* a = reinterpret_cast<void*>(0x1000);
    void* b = reinterpret_cast<void*>(0x100000);
    // argument errors, before any device call
    EXPECT(rs_sort_u32(nullptr, (uint32_t*)b, 10, 8, RS_ALGO_LSD, nullptr, 0, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_u32((uint32_t*)a, (uint32_t*)b, 10, 17, RS_ALGO_LSD, nullptr, 0, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_u32((uint32_t*)a, (uint32_t*)a, (size_t)1 << 32, 8, RS_ALGO_LSD, nullptr, 0, nullptr) ==
           RS_ERR_UNSUPPORTED);
    EXPECT(rs_sort_kv(a, b, a, (char*)b + 64, 10, 8, 8, 8, RS_ALGO_LSD, nullptr, 0, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_kv(a, b, a, b, 10, 4, 2, 8, RS_ALGO_LSD, nullptr, 0, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_u32(nullptr, nullptr, 0, 8, RS_ALGO_LSD, nullptr, 0, nullptr) == RS_OK);
    EXPECT(rs_sort_blocks_u32((uint32_t*)a, (uint32_t*)b, 10, RS_ALGO_BTN, 3, nullptr, 0, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_u32_noalloc((uint32_t*)a, (uint32_t*)a, (1u << 22) + 1, 8, RS_ALGO_LSD, nullptr) ==
           RS_ERR_UNSUPPORTED);
    EXPECT(rs_stream_copy(a, (char*)a + 8, 64, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_sort_segmented((uint32_t*)a, (uint32_t*)b, (int64_t*)a, 3, -1, RS_ALGO_AUTO, nullptr, 0, nullptr) ==
           RS_ERR_INVALID);
    EXPECT(rs_sort_segmented((uint32_t*)a, (uint32_t*)b, (int64_t*)a, 3, 10, RS_ALGO_LEARNED, nullptr, 0, nullptr) ==
           RS_ERR_UNSUPPORTED);
    // the shared rounds' tables grow with the keys, not with the segment count
    EXPECT(rs_workspace_bytes(RS_OP_SEGMENTED, (size_t)1 << 24, 4, 0, 0, RS_ALGO_AUTO, (size_t)1 << 20) <
           ((size_t)8 << 24) + ((size_t)32 << 20));
    // workspace sizes over many shapes: non-zero, 256-byte multiples, growing with n
    for (int op = 0; op <= 5; ++op)
        for (int kb = 4; kb <= 8; kb += 4)
            for (int vb = 0; vb <= 8; vb += 4)
                for (int bits = 0; bits <= 17; ++bits)
                    for (int algo = 0; algo <= 6; ++algo)
                        for (size_t n : {(size_t)0, (size_t)1, (size_t)1000, (size_t)1 << 20, ((size_t)1 << 28) + 3}) {
                            const size_t w = rs_workspace_bytes(op, n, kb, vb, bits, (rs_algo)algo, n ? 7 : 0);
                            EXPECT(w % 256 == 0);
                        }
    EXPECT(rs_workspace_bytes(RS_OP_SORT, 1 << 20, 4, 0, 8, RS_ALGO_LSD, 0) <
           rs_workspace_bytes(RS_OP_SORT, 1 << 24, 4, 0, 8, RS_ALGO_LSD, 0));
    for (size_t n : {(size_t)100, (size_t)1 << 20, (size_t)1 << 30})
        for (int algo : {RS_ALGO_BTN, RS_ALGO_OET}) {
            const int p = rs_blocks_default_p(n, (rs_algo)algo);
            EXPECT(p >= 2 && p <= 4096);
        }
    // the tuning table
    rs_tune_entry t[64];
    const int k = rs_tune_get(t, 64);
    EXPECT(k == 33);
    rs_tune_entry e = {20, 0, 0, 11, 0, 8};
    EXPECT(rs_tune_set(&e, 1) == RS_OK);
    rs_tune_entry bad = {20, 2, 4, 8, 0, 0};
    EXPECT(rs_tune_set(&bad, 1) == RS_ERR_INVALID);
    EXPECT(rs_tune_set(t, k) == RS_OK);
    const std::string good =
        "{\"format\": \"rs-tuning-1\", \"arch\": \"gfx950\", \"cus\": 256, \"classes\": [{\"size_log2\": 20, "
        "\"algo\": 0, \"p\": 0, \"radix_bits\": 11, \"tile_items\": 0, \"seg_tile_items\": 8}]}";
    // every prefix of a well-formed file, and one byte changed at every place
    int files = 0;
    for (size_t cut = 0; cut < good.size(); ++cut) {
        const rs_status rc = rs_tune_load(write_file(dir, good.substr(0, cut), files++).c_str());
        EXPECT(rc == RS_ERR_INVALID);
    }
    for (size_t at = 0; at < good.size(); ++at)
        for (char ch : {'"', '{', '}', '[', ']', ':', ',', '\\', '9', '-', 'x', '\0'}) {
            std::string s = good;
            s[at] = ch;
            const rs_status rc = rs_tune_load(write_file(dir, s, files++).c_str());
            EXPECT(rc == RS_ERR_INVALID || rc == RS_ERR_HIP || rc == RS_ERR_UNSUPPORTED);
        }
    EXPECT(rs_tune_load(write_file(dir, good, files++).c_str()) == RS_ERR_HIP);  // no device here
    EXPECT(rs_tune_load((std::string(dir) + "/missing.json").c_str()) == RS_ERR_INVALID);
    EXPECT(rs_tune_load(nullptr) == RS_ERR_INVALID);
    // learned-path options and hooks
    rs_learned_opts o;
    EXPECT(rs_learned_get_opts(&o) == RS_OK);
    rs_learned_opts o2 = o;
    o2.bucket_cap = 1;
    EXPECT(rs_learned_set_opts(&o2) == RS_ERR_INVALID);
    EXPECT(rs_learned_set_opts(&o) == RS_OK);
    float w[1153] = {0};
    EXPECT(rs_mlp_set_weights(w, 1152) == RS_ERR_INVALID);
    EXPECT(rs_mlp_set_weights(w, 1153) == RS_OK);
    EXPECT(rs_mlp_set_weights(nullptr, 0) == RS_OK);
    EXPECT(rs_learned_debug_fault(RS_LEARNED_FAULT_SPLITTERS, nullptr, 0) == RS_ERR_INVALID);
    EXPECT(rs_learned_debug_fault(7, nullptr, 0) == RS_ERR_INVALID);
    EXPECT(rs_learned_debug_fault(RS_LEARNED_FAULT_NONE, nullptr, 0) == RS_OK);
    EXPECT(rs_learned_debug_ids(nullptr, (uint16_t*)b) == RS_ERR_INVALID);
    EXPECT(rs_learned_debug_ids((uint16_t*)a, nullptr) == RS_ERR_INVALID);
    EXPECT(rs_learned_debug_ids(nullptr, nullptr) == RS_OK);
    rs_tune_result tr[4];
    EXPECT(rs_tune_run_model(nullptr, 0, 0, nullptr, tr, 4) == -RS_ERR_INVALID);
    EXPECT(rs_tune_run_model(nullptr, 0, 16, nullptr, nullptr, 4) == -RS_ERR_INVALID);
    EXPECT(rs_tune_run_model(nullptr, 0, 16, nullptr, tr, 4) == -RS_ERR_WORKSPACE);
    rs_block_model m;
    EXPECT(rs_blocks_get_model(&m) == RS_OK);
    rs_block_model m2 = m;
    m2.local_ns_per_key = -1.0;
    EXPECT(rs_blocks_set_model(&m2) == RS_ERR_INVALID);
    EXPECT(rs_blocks_set_model(&m) == RS_OK);
    for (int s = -1; s <= 5; ++s) EXPECT(rs_status_string((rs_status)s) != nullptr);
    rs_stats st;
    EXPECT(rs_get_stats(&st) == RS_OK);
    if (failures) return 1;
    printf("host driver: ok (%d tuning files)\n", files);
    return 0;
}
