// Host-side checks of libhookcc, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py (no GPU needed):
//   1. the request server's arena allocator against a byte-map model of
//      first-fit allocation (every offset it returns must equal the model's,
//      and every request the model can place must succeed: release must
//      coalesce neighbouring free ranges);
//   2. the C ABI's argument validation and plan arithmetic: invalid
//      arguments of every entry point, and cc_workspace_bytes at extreme
//      sizes, where an overflow would otherwise go unnoticed.
// Prints "host checks ok" and exits 0 when every check passes.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../include/hookcc.h"
#include "../paper_1612_01178_amd/csrc/arena.hpp"

static int g_fail = 0;
#define CHECK(cond)                                                           \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "check failed, line %d: %s\n", __LINE__, #cond); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

// Lowest offset of `len` free units in `used`, or -1.
static long model_first_fit(const std::vector<char>& used, size_t len) {
    size_t run = 0;
    for (size_t i = 0; i < used.size(); ++i) {
        run = used[i] ? 0 : run + 1;
        if (run == len) return (long)(i + 1 - len);
    }
    return -1;
}

static void arena_against_model() {
    const size_t size = 4096;
    hookcc::Arena arena;
    arena.reset(size);
    std::vector<char> used(size, 0);
    std::vector<std::pair<size_t, size_t>> live;  // (offset, length)
    std::mt19937_64 rng(12345);
    size_t in_use = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t len = 1 + rng() % ((rng() % 8 == 0) ? 1024 : 48);
            const long want = model_first_fit(used, len);
            size_t off = ~size_t(0);
            const bool ok = arena.alloc(len, &off);
            CHECK(ok == (want >= 0));
            if (ok && want >= 0) {
                CHECK(off == (size_t)want);
                for (size_t i = off; i < off + len && i < size; ++i) {
                    CHECK(!used[i]);
                    used[i] = 1;
                }
                live.push_back({off, len});
                in_use += len;
            }
        } else {
            const size_t k = rng() % live.size();
            const auto blk = live[k];
            live[k] = live.back();
            live.pop_back();
            arena.release(blk.first, blk.second);
            for (size_t i = blk.first; i < blk.first + blk.second; ++i) used[i] = 0;
            in_use -= blk.second;
        }
        CHECK(arena.used() == in_use);
        if (g_fail > 20) return;
    }
    // everything released: one free range of the whole size again
    for (const auto& blk : live) arena.release(blk.first, blk.second);
    size_t off = 1;
    CHECK(arena.used() == 0);
    CHECK(arena.alloc(size, &off) && off == 0);
    // zero-byte requests take nothing
    hookcc::Arena empty;
    empty.reset(0);
    CHECK(empty.alloc(0, &off) && off == 0);
    CHECK(!empty.alloc(1, &off));
}

static void abi_validation() {
    int32_t d[8] = {0};
    int64_t d64[8] = {0};
    // cc_labels / cc_labels_ex / cc_labels_noalloc
    CHECK(cc_labels(-1, d, d, 1, d) == CC_ERR_ARG);
    CHECK(cc_labels(4, nullptr, d, 1, d) == CC_ERR_ARG);
    CHECK(cc_labels(4, d, nullptr, 1, d) == CC_ERR_ARG);
    CHECK(cc_labels(4, d, d, -1, d) == CC_ERR_ARG);
    CHECK(cc_labels(4, d, d, 1, nullptr) == CC_ERR_ARG);
    cc_options o;
    cc_options_init(&o);
    o.reserved[0] = 1;
    CHECK(cc_labels_ex(4, d, d, 1, d, &o, nullptr, 0, nullptr, nullptr) == CC_ERR_ARG);
    int32_t cc_options::*const fields[] = {&cc_options::hook,       &cc_options::filter,
                                          &cc_options::block,      &cc_options::edges_per_thread,
                                          &cc_options::hot_cache,  &cc_options::path_halving,
                                          &cc_options::symmetric,  &cc_options::graph,
                                          &cc_options::no_sync,    &cc_options::compact_threshold,
                                          &cc_options::host_loop,  &cc_options::profile,
                                          &cc_options::coherent_loads};
    const int32_t bad_values[] = {-7, 99, 100, 5, 9, 3, 2, 2, 2, 1001, 3, 2, 2};
    for (size_t i = 0; i < sizeof(fields) / sizeof(fields[0]); ++i) {
        cc_options_init(&o);
        o.*fields[i] = bad_values[i];
        CHECK(cc_labels_ex(4, d, d, 1, d, &o, nullptr, 0, nullptr, nullptr) == CC_ERR_ARG);
        CHECK(cc_workspace_bytes(4, 1, &o) == 0);
    }
    cc_options_init(&o);
    o.segments = -1;
    CHECK(cc_labels_ex(4, d, d, 1, d, &o, nullptr, 0, nullptr, nullptr) == CC_ERR_ARG);
    cc_options_init(&o);
    o.graph = 1;
    CHECK(cc_labels_noalloc(4, d, d, 1, d, &o, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_noalloc(-3, d, d, 1, d, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    // workspace sizes: plain arithmetic, also at extreme sizes
    CHECK(cc_workspace_bytes(-1, 1, nullptr) == 0);
    CHECK(cc_workspace_bytes(1, -1, nullptr) == 0);
    const int32_t ns[] = {0, 1, 7, 65536, 1 << 24, INT32_MAX};
    const int64_t ms[] = {0, 1, 3, 1 << 22, int64_t(1) << 31, int64_t(1) << 40, INT64_MAX / 64,
                          INT64_MAX};
    for (int32_t n : ns)
        for (int64_t m : ms)
            for (int hook : {CC_HOOK_AUTO, CC_HOOK_ATOMIC, CC_HOOK_PLAIN, CC_HOOK_HYBRID}) {
                cc_options_init(&o);
                o.hook = hook;
                const size_t w = cc_workspace_bytes(n, m, &o);
                CHECK(w == 0 || w >= 256);
            }
    // batches and graph lists
    int64_t vo[3] = {0, 4, 3}, eo[3] = {0, 1, 2};
    CHECK(cc_labels_batch(2, vo, eo, d, d, d) == CC_ERR_ARG);  // decreasing offsets
    int64_t vo1[2] = {1, 4}, eo1[2] = {0, 1};
    CHECK(cc_labels_batch(1, vo1, eo1, d, d, d) == CC_ERR_ARG);  // offsets start at 1
    int64_t vo2[2] = {0, int64_t(1) << 33}, eo2[2] = {0, 0};
    CHECK(cc_labels_batch(1, vo2, eo2, d, d, d) == CC_ERR_ARG);  // a graph of 2^33 vertices
    CHECK(cc_labels_batch(1, nullptr, eo1, d, d, d) == CC_ERR_ARG);
    CHECK(cc_labels_batch(-1, nullptr, nullptr, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_batch(0, nullptr, nullptr, nullptr, nullptr, nullptr) == CC_OK);
    int64_t vo3[2] = {0, 4}, eo3[2] = {0, 2};
    CHECK(cc_labels_batch(1, vo3, eo3, nullptr, d, d) == CC_ERR_ARG);  // null edges
    cc_options_init(&o);
    o.block = 100;
    CHECK(cc_labels_batch_ex(1, vo3, eo3, d, d, d, &o, nullptr, nullptr) == CC_ERR_ARG);
    // batches with device offsets: argument checks made before any launch
    CHECK(cc_labels_batch_device(-1, d64, d64, d, d, d, 8, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_batch_device(0, nullptr, nullptr, nullptr, nullptr, nullptr, 8, nullptr,
                                 nullptr, nullptr) == CC_OK);
    CHECK(cc_labels_batch_device(2, d64, d64, d, d, d, 0, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_batch_device(2, d64, d64, d, d, d, CC_BATCH_LDS_MAX_N + 1, nullptr, nullptr,
                                 nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_batch_device(2, nullptr, d64, d, d, d, 8, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_batch_device(2, d64, nullptr, d, d, d, 8, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    cc_options_init(&o);
    o.block = 96;
    CHECK(cc_labels_batch_device(2, d64, d64, d, d, d, 8, &o, nullptr, nullptr) == CC_ERR_ARG);
    cc_options_init(&o);
    o.no_sync = 1;
    CHECK(cc_labels_batch_device(2, d64, d64, d, d, d, 8, &o, nullptr, nullptr) == CC_ERR_ARG);
    cc_graph g[2];
    std::memset(g, 0, sizeof g);
    g[0].n = 4;
    g[0].m = 1;
    g[0].edges_u = d;
    g[0].edges_v = d;
    g[0].out_label = d;
    g[1] = g[0];
    g[1].reserved = 1;
    CHECK(cc_labels_list(2, g, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    g[1].reserved = 0;
    g[1].n = -1;
    CHECK(cc_labels_list(2, g, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    g[1].n = 4;
    g[1].edges_v = nullptr;
    CHECK(cc_labels_list(2, g, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_list(1, nullptr, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_list(-2, g, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    // CSR and streamed host edges
    CHECK(cc_labels_csr(4, nullptr, d, 1, d, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_csr(4, d64, nullptr, 1, d, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_csr(-4, d64, d, 1, d, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    cc_options_init(&o);
    o.hook = CC_HOOK_PLAIN;
    CHECK(cc_labels_csr(4, d64, d, 1, d, &o, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_host(4, d, d, 1, d, -5, nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_labels_host(4, d, d, 1, d, 0, &o, nullptr, nullptr) == CC_ERR_ARG);
    // probes
    CHECK(cc_probe(-1, d, d, 4, nullptr, 0, nullptr) == CC_ERR_ARG);
    CHECK(cc_probe(12, d, d, 4, d, 128, nullptr) == CC_ERR_ARG);
    CHECK(cc_probe(7, nullptr, nullptr, 0, nullptr, 0, nullptr) == CC_ERR_ARG);
    // server
    cc_server* srv = reinterpret_cast<cc_server*>(d);
    CHECK(cc_server_create(nullptr, nullptr) == CC_ERR_ARG);
    cc_server_config cfg;
    std::memset(&cfg, 0, sizeof cfg);
    cfg.reserved[3] = 1;
    CHECK(cc_server_create(&cfg, &srv) == CC_ERR_ARG && srv == nullptr);
    std::memset(&cfg, 0, sizeof cfg);
    cfg.workers = 17;
    CHECK(cc_server_create(&cfg, &srv) == CC_ERR_ARG);
    cfg.workers = 1;
    cfg.device_bytes = -5;
    CHECK(cc_server_create(&cfg, &srv) == CC_ERR_ARG);
    int64_t ticket = 0;
    CHECK(cc_server_submit(nullptr, 4, d, d, 1, d, 0, &ticket) == CC_ERR_ARG);
    CHECK(cc_server_wait(nullptr, 1, nullptr) == CC_ERR_ARG);
    CHECK(cc_server_poll(nullptr, 1, nullptr) == CC_ERR_ARG);
    CHECK(cc_server_stats(nullptr, nullptr, nullptr) == CC_ERR_ARG);
    CHECK(cc_server_destroy(nullptr) == CC_OK);
    // library state
    CHECK(cc_last_error() != nullptr);
    CHECK(std::strlen(cc_version()) > 0);
    cc_release();
    CHECK(cc_stream_status(nullptr) == CC_ERR_ARG);
}

int main() {
    arena_against_model();
    abi_validation();
    if (g_fail) {
        std::fprintf(stderr, "%d host checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks ok\n");
    return 0;
}
