// Host engine of libhookcc (the C ABI wrappers are in capi.cpp).
//
// The engine turns a call into a plan (hook variant, segment bounds, filter,
// tiling), takes device scratch from a per-(device, stream) cache, enqueues
// the kernel sequence on the caller's stream, and ends with one stream
// synchronisation plus a 256-byte read of the device control block (status
// bits and statistics).  No step of the solve runs on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"

namespace hookcc {

namespace {
thread_local std::string t_err;
}  // namespace

int32_t fail(int32_t code, const std::string& msg) {
    t_err = msg;
    return code;
}

const char* last_error() { return t_err.c_str(); }

namespace {

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? CC_ERR_NOMEM : CC_ERR_HIP,             \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Size class of a work amount w: 4 * floor(log2 w) + the two bits below the
// leading one (0..255; larger w, larger class).
int size_class(uint64_t w) {
    w |= 1;
    const int lg = 63 - __builtin_clzll(w);
    const int frac = lg >= 2 ? (int)((w >> (lg - 2)) & 3) : (int)((w << (2 - lg)) & 3);
    return lg * 4 + frac;
}

// ---------------------------------------------------------------------- plans
// round(m / n), at least 1, for m >= 0 and n > 0, without overflow.
int64_t round_ratio(int64_t m, int64_t n) {
    return std::max<int64_t>(1, m / n + ((m % n) * 2 >= n ? 1 : 0));
}

// First entry of segment i of S over m entries: floor(m * i / S) rounded down
// to a multiple of 4 (keeps 16-byte loads aligned); 128-bit product, so any
// m >= 0 works.
int64_t segment_start(int64_t m, int64_t i, int64_t S) {
    return (int64_t)(((__int128)m * i) / S) & ~int64_t(3);
}


struct Plan {
    int hook = CC_HOOK_ATOMIC;  // resolved variant: CC_HOOK_ATOMIC, CC_HOOK_PLAIN or CC_HOOK_HYBRID
    int segments = 1;
    int filter = CC_FILTER_OFF;
    int filter_after = 1;
    int block = 256;
    int ept = 8;
    int64_t max_rounds = 0;
    int rounds_per_check = 4;
    bool profile = false;
    int host_loop = CC_HOST_LOOP_OFF;
    bool coherent = false;
    bool hot = false;  // hot-word LDS cache of the giant bitmap
    int hot_slots = 32768;
    bool halve = true;  // path halving in the Atomic-Hook climb
    bool symmetric = false;  // caller promises both orientations of every pair
    bool graph = false;      // capture the launch sequence in a hipGraph and replay it
    bool no_sync = false;    // enqueue only; status read later by cc_stream_status
    uint32_t tau = 0xffffffffu;  // atomic-free Hook: frontier rewrite threshold (1/1000)
};

// Hook variants an input form supports: pair lists all of them; CSR input the
// Atomic-Hook and the hybrid plan (its atomic-free pass needs no frontier);
// the graph-list path the Atomic-Hook only.
enum PlanInput { kInputPairs, kInputCsr, kInputAtomicOnly };

int32_t make_plan(int32_t n, int64_t m, const cc_options* o, Plan& p,
                  PlanInput input = kInputPairs) {
    const bool allow_plain = input == kInputPairs;
    const bool allow_hybrid = input != kInputAtomicOnly;
    cc_options d;
    std::memset(&d, 0, sizeof d);
    d.filter = CC_FILTER_AUTO;
    const cc_options& op = o ? *o : d;
    if (op.reserved[0] != 0) return fail(CC_ERR_ARG, "cc_options.reserved must be zero");
    if (op.graph != 0 && op.graph != 1) return fail(CC_ERR_ARG, "cc_options.graph must be 0 or 1");
    p.graph = op.graph == 1;
    if (op.no_sync != 0 && op.no_sync != 1)
        return fail(CC_ERR_ARG, "cc_options.no_sync must be 0 or 1");
    p.no_sync = op.no_sync == 1;
    if (op.compact_threshold < 0 || op.compact_threshold > 1000)
        return fail(CC_ERR_ARG, "cc_options.compact_threshold must be in [0, 1000]");
    p.tau = op.compact_threshold ? (uint32_t)op.compact_threshold : 0xffffffffu;
    if (op.symmetric != 0 && op.symmetric != 1)
        return fail(CC_ERR_ARG, "cc_options.symmetric must be 0 or 1");
    p.symmetric = op.symmetric == 1;
    if (op.hot_cache < CC_HOT_AUTO || op.hot_cache > CC_HOT_VERTEX)
        return fail(CC_ERR_ARG, "unknown cc_options.hot_cache");
    // Hot cache: the vertex table where every id fits its tags (n <= 255 *
    // 81,920; R-MAT 24: 3.9 ms against 4.52 with 32,768 word slots), else the
    // word table.
    const bool vert = op.hot_cache == CC_HOT_VERTEX ||
                      (op.hot_cache == CC_HOT_AUTO && n <= (int64_t)kVertTagNone * kVertSets);
    p.hot_slots = op.hot_cache == CC_HOT_ON ? 16384 : vert ? kVertSlots : 32768;
    if (op.path_halving < CC_HALVE_AUTO || op.path_halving > CC_HALVE_OFF)
        return fail(CC_ERR_ARG, "unknown cc_options.path_halving");
    p.halve = op.path_halving != CC_HALVE_OFF;
    if (op.coherent_loads != 0 && op.coherent_loads != 1)
        return fail(CC_ERR_ARG, "cc_options.coherent_loads must be 0 or 1");
    p.coherent = op.coherent_loads == 1;
    if (op.hook != CC_HOOK_AUTO && op.hook != CC_HOOK_ATOMIC && op.hook != CC_HOOK_PLAIN &&
        op.hook != CC_HOOK_HYBRID)
        return fail(CC_ERR_ARG, "unknown cc_options.hook");
    if (op.segments < 0) return fail(CC_ERR_ARG, "cc_options.segments < 0");
    // Average-degree heuristic (Section 3.B, Fig. 4): s = 2|E|/|V|, read as
    // s = (entries passed) / n -- the average degree when the list holds both
    // orientations of every edge, half of it when each edge is listed once
    // (the library cannot tell the two apart).
    const int64_t s_paper = n > 0 ? std::min<int64_t>(int64_t(1) << 20, round_ratio(m, n)) : 1;
    // Automatic variant (measured on gfx950): on large dense lists (average
    // degree >= 8) the filtered Atomic-Hook wins (one pass over the entries,
    // most of them reduced to two bitmap tests; R-MAT 24 3.8 ms against 38 ms
    // for the atomic-free rounds); on large sparse lists the hybrid plan (the
    // window round, then Atomic-Hook over the compacted pairs; percolated
    // 4096^2 grid 0.38 ms against 1.07 Atomic-Hook and 0.99 atomic-free
    // rounds).  On small lists (< 2^22 entries) the per-kernel cost dominates
    // and the atomic-free rounds win (ER 2^16: 0.10 ms against 0.26 hybrid and
    // 0.14-0.28 Atomic-Hook); a no-sync call needs a fixed launch
    // sequence and takes the hybrid plan there.  CSR input has no atomic-free
    // rounds: its large sparse inputs take the hybrid plan (grid as CSR 0.73
    // ms against 1.47 Atomic-Hook), the rest the Atomic-Hook.
    const bool large = m >= (int64_t(1) << 22);
    const bool dense_large = large && n > 0 && m >= 8 * (int64_t)n;
    bool auto_filtered = false;
    if (op.hook == CC_HOOK_AUTO) {
        if (!allow_hybrid || (allow_plain && op.symmetric == 1) || dense_large) {
            p.hook = CC_HOOK_ATOMIC;
            auto_filtered = dense_large && op.filter != CC_FILTER_OFF;
        } else if (!allow_plain) {
            p.hook = large ? CC_HOOK_HYBRID : CC_HOOK_ATOMIC;
        } else if (large || op.no_sync == 1) {
            p.hook = CC_HOOK_HYBRID;
        } else {
            p.hook = CC_HOOK_PLAIN;
        }
    } else {
        p.hook = op.hook;
    }
    if ((!allow_plain && p.hook == CC_HOOK_PLAIN) || (!allow_hybrid && p.hook == CC_HOOK_HYBRID))
        return fail(CC_ERR_ARG, "the atomic-free Hook is not available here");
    int64_t s = op.segments;
    // The filtered plan hooks its first segment unfiltered, and that launch
    // is the costliest per entry (hub roots contended before any giant
    // exists): a first segment of ~n/16 entries (R-MAT 24: 3.80 ms against
    // 3.86 at n/8 and 3.98 at n/4).
    if (s == 0) s = auto_filtered ? 16 * s_paper : s_paper;
    const int64_t smax = std::max<int64_t>(1, m / 4 + (m % 4 != 0));
    s = std::max<int64_t>(1, std::min<int64_t>(s, smax));
    s = std::min<int64_t>(s, 1 << 20);
    p.segments = (int)s;
    if (op.filter < CC_FILTER_OFF || op.filter > CC_FILTER_AUTO)
        return fail(CC_ERR_ARG, "unknown cc_options.filter");
    if (op.filter_after < 0) return fail(CC_ERR_ARG, "cc_options.filter_after < 0");
    p.filter_after = op.filter_after ? op.filter_after : 1;
    if (p.hook != CC_HOOK_ATOMIC) {
        p.filter = CC_FILTER_OFF;
    } else if (op.hook == CC_HOOK_AUTO && op.filter == CC_FILTER_AUTO) {
        p.filter = auto_filtered ? CC_FILTER_GIANT : CC_FILTER_OFF;
    } else if (op.filter == CC_FILTER_AUTO) {
        // A giant component is near-certain at average degree >= 3.5, and the
        // sample + bitmap cost only pays off on large edge lists.
        p.filter = (p.segments >= 4 && m >= (int64_t(1) << 22)) ? CC_FILTER_GIANT : CC_FILTER_OFF;
    } else {
        p.filter = op.filter;
    }
    if (p.filter == CC_FILTER_GIANT && p.filter_after >= p.segments) p.filter = CC_FILTER_OFF;
    p.hot = p.filter == CC_FILTER_GIANT && op.hot_cache != CC_HOT_OFF && !p.coherent;
    if (op.block != 0) {
        if (op.block < 64 || op.block > 1024 || op.block % 64)
            return fail(CC_ERR_ARG, "cc_options.block must be a multiple of 64 in [64, 1024]");
        p.block = op.block;
    } else if (auto_filtered) {
        p.block = 512;  // first (unfiltered) segment: R-MAT 24 3.78 ms against 3.80 at 256
    }
    // Tile: 16 entries per thread for the plain Atomic-Hook (measured best on
    // sparse lists, e.g. the percolated grid), 8 where the filter runs.
    p.ept = (p.filter == CC_FILTER_GIANT || p.hook != CC_HOOK_ATOMIC) ? 8 : 16;
    // The hybrid plan's atomic-free round over the whole list runs best in
    // large tiles (percolated 4096^2 grid: 0.73 ms at 1024 threads x 16
    // entries against 0.83 ms at 256 x 8).
    if (p.hook == CC_HOOK_HYBRID) {
        p.ept = 16;
        if (op.block == 0) p.block = 1024;
    }
    if (op.edges_per_thread != 0) {
        if (op.edges_per_thread != 4 && op.edges_per_thread != 8 && op.edges_per_thread != 16)
            return fail(CC_ERR_ARG, "cc_options.edges_per_thread must be 4, 8 or 16");
        p.ept = op.edges_per_thread;
    }
    if (op.max_rounds < 0) return fail(CC_ERR_ARG, "cc_options.max_rounds < 0");
    p.max_rounds = op.max_rounds ? op.max_rounds : (int64_t)n + 1;
    if (op.rounds_per_check < 0) return fail(CC_ERR_ARG, "cc_options.rounds_per_check < 0");
    p.rounds_per_check = op.rounds_per_check ? op.rounds_per_check : 4;
    if (op.profile != 0 && op.profile != 1) return fail(CC_ERR_ARG, "cc_options.profile must be 0 or 1");
    p.profile = op.profile == 1;
    if (op.host_loop < CC_HOST_LOOP_OFF || op.host_loop > CC_HOST_LOOP_MULTIJUMP)
        return fail(CC_ERR_ARG, "unknown cc_options.host_loop");
    if (op.host_loop != CC_HOST_LOOP_OFF && op.hook != CC_HOOK_PLAIN)
        return fail(CC_ERR_ARG, "cc_options.host_loop needs hook = CC_HOOK_PLAIN");
    p.host_loop = op.host_loop;
    if (p.symmetric && p.hook != CC_HOOK_ATOMIC && !(input == kInputCsr && p.hook == CC_HOOK_HYBRID))
        return fail(CC_ERR_ARG, "cc_options.symmetric needs the Atomic-Hook");
    if ((p.hook == CC_HOOK_PLAIN || p.hook == CC_HOOK_HYBRID) && m >= (int64_t(1) << 32))
        return fail(CC_ERR_ARG, "atomic-free Hook supports m < 2^32 entries");
    if (p.no_sync && ((p.hook != CC_HOOK_ATOMIC && p.hook != CC_HOOK_HYBRID) || p.profile))
        return fail(CC_ERR_ARG,
                    "cc_options.no_sync needs the Atomic-Hook (the atomic-free Hook reads the "
                    "device convergence word from the host) and profile = 0");
    return CC_OK;
}

// Workspace: [Ctrl 256 B][giant bitmap][frontier 0][frontier 1]
struct Layout {
    size_t bits = 0, f0 = 0, f1 = 0, total = 0;
    size_t hot_counts = 0, hot_tags = 0, hot_vals = 0;
    int64_t cap = 0;
};

Layout layout(int32_t n, int64_t m, const Plan& p) {
    Layout L;
    size_t off = 256;
    if (p.hook == CC_HOOK_ATOMIC && p.filter == CC_FILTER_GIANT) {
        L.bits = off;
        off += align256(((size_t)n + 31) / 32 * 4);
        if (p.hot && p.hot_slots == kVertSlots) {  // selection scratch, byte table
            L.hot_counts = off;
            off += align256((size_t)kVertScratchWords * 4);
            L.hot_tags = L.hot_vals = off;  // tags, then member flags
            off += align256((size_t)kVertSlots * 2);
        } else if (p.hot) {
            L.hot_counts = off;
            off += align256(((size_t)n + 31) / 32 * 4);
            L.hot_tags = off;
            off += align256((size_t)kHotSlotsMax * 4);
            L.hot_vals = off;
            off += align256((size_t)kHotSlotsMax * 4);
        }
    }
    if (p.hook == CC_HOOK_PLAIN && p.host_loop == CC_HOST_LOOP_OFF) {
        L.cap = m;
        L.f0 = off;
        off += align256((size_t)m * 8);
        L.f1 = off;
        off += align256((size_t)m * 8);
    }
    if (p.hook == CC_HOOK_HYBRID) {  // one frontier: round 1 writes it, nothing rewrites it
        L.cap = m;
        L.f0 = L.f1 = off;
        off += align256((size_t)m * 8);
    }
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------- workspace cache
struct PoolEntry {
    std::mutex mu;  // held for the whole duration of a call using this entry
    void* dev = nullptr;
    size_t bytes = 0;
    Ctrl* host_ctrl = nullptr;  // pinned, host_ctrl_count control blocks
    int64_t host_ctrl_count = 0;
    void* host_stage = nullptr; // pinned staging for batch descriptors
    size_t stage_bytes = 0;
    hipStream_t copy_stream = nullptr;  // host-to-device staging of streamed solves
    hipEvent_t copied[2] = {nullptr, nullptr};
    int32_t* batch_status = nullptr;  // pinned: the LDS batch launch's status word
    hipEvent_t consumed[2] = {nullptr, nullptr};
    // status word of the last no-sync call (pinned) and the event after its copy
    int32_t* async_slot = nullptr;
    hipEvent_t async_done = nullptr;
    bool async_called = false;
    // captured launch sequences of recent calls, most recent last
    struct Captured {
        uint64_t key;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Captured> graphs;
};

// Waits for the work of earlier no-sync calls on this entry's stream (before
// a buffer or a graph that work may still use is freed).
void drain_async(PoolEntry* e) {
    if (e->async_called && e->async_done) (void)hipEventSynchronize(e->async_done);
}

void drop_graphs(PoolEntry* e) {
    if (!e->graphs.empty()) drain_async(e);
    for (auto& c : e->graphs) {
        (void)hipGraphExecDestroy(c.exec);
        (void)hipGraphDestroy(c.graph);
    }
    e->graphs.clear();
}

// FNV-1a over the bytes that determine a launch sequence.
struct KeyHash {
    uint64_t h = 1469598103934665603ULL;
    template <class T>
    KeyHash& add(const T& x) {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
        for (size_t i = 0; i < sizeof(T); ++i) h = (h ^ p[i]) * 1099511628211ULL;
        return *this;
    }
};

std::mutex g_pool_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<PoolEntry>> g_pool;

PoolEntry* pool_entry(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto& e = g_pool[{dev, s}];
    if (!e) e.reset(new PoolEntry());
    return e.get();
}

int32_t ensure_dev(PoolEntry* e, size_t bytes) {
    if (e->bytes >= bytes && e->dev) return CC_OK;
    drop_graphs(e);  // captured graphs point into the old buffer
    drain_async(e);
    if (e->dev) {
        HIPCHK(hipFree(e->dev));
        e->dev = nullptr;
        e->bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 1 << 20);
    HIPCHK(hipMalloc(&e->dev, want));
    e->bytes = want;
    return CC_OK;
}

int32_t ensure_host(PoolEntry* e, int64_t count = 1) {
    if (e->host_ctrl && e->host_ctrl_count >= count) return CC_OK;
    if (e->host_ctrl) {
        HIPCHK(hipHostFree(e->host_ctrl));
        e->host_ctrl = nullptr;
        e->host_ctrl_count = 0;
    }
    const int64_t want = std::max<int64_t>(count, 16);
    HIPCHK(hipHostMalloc((void**)&e->host_ctrl, sizeof(Ctrl) * want, hipHostMallocDefault));
    e->host_ctrl_count = want;
    return CC_OK;
}

int32_t ensure_stage(PoolEntry* e, size_t bytes) {
    if (e->stage_bytes >= bytes && e->host_stage) return CC_OK;
    drop_graphs(e);  // captured copies read from the old staging buffer
    if (e->host_stage) {
        HIPCHK(hipHostFree(e->host_stage));
        e->host_stage = nullptr;
        e->stage_bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 1 << 16);
    HIPCHK(hipHostMalloc(&e->host_stage, want, hipHostMallocDefault));
    e->stage_bytes = want;
    return CC_OK;
}

// ---------------------------------------------------------------------- profiling
struct Timer {
    bool on = false;
    hipStream_t s = nullptr;
    struct Ev {
        hipEvent_t a, b;
        int phase;
    };
    std::vector<Ev> evs;
    ~Timer() {
        for (auto& e : evs) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    }
    hipError_t begin(int phase) {
        if (!on) return hipSuccess;
        Ev e;
        e.phase = phase;
        hipError_t r = hipEventCreate(&e.a);
        if (r != hipSuccess) return r;
        r = hipEventCreate(&e.b);
        if (r != hipSuccess) return r;
        evs.push_back(e);
        return hipEventRecord(e.a, s);
    }
    hipError_t end() {
        if (!on) return hipSuccess;
        return hipEventRecord(evs.back().b, s);
    }
    void collect(cc_stats* st) {
        if (!on || !st) return;
        float t[3] = {0, 0, 0};
        for (auto& e : evs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) t[e.phase] += ms;
        }
        st->hook_ms = t[0];
        st->compress_ms = t[1];
        st->other_ms = t[2];
    }
};
enum { kPhaseHook = 0, kPhaseCompress = 1, kPhaseOther = 2 };

#define TIMED(phase, expr)                 \
    do {                                   \
        HIPCHK(tm.begin(phase));           \
        HIPCHK(expr);                      \
        HIPCHK(tm.end());                  \
    } while (0)

// Runs `enqueue` on s through a cached hipGraph keyed by `key`: the first
// call with a key captures the launch sequence, later calls replay it.  Up
// to 8 graphs are kept per pool entry.  Needs a stream other than the null
// stream (the legacy null stream cannot be captured).
template <class F>
int32_t run_graph(PoolEntry* pe, uint64_t key, hipStream_t s, F&& enqueue) {
    PoolEntry::Captured* hit = nullptr;
    for (auto& c : pe->graphs)
        if (c.key == key) hit = &c;
    if (!hit) {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int32_t rc = enqueue();
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc != CC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(CC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(CC_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        if (pe->graphs.size() >= 8) {
            drain_async(pe);
            (void)hipGraphExecDestroy(pe->graphs.front().exec);
            (void)hipGraphDestroy(pe->graphs.front().graph);
            pe->graphs.erase(pe->graphs.begin());
        }
        pe->graphs.push_back({key, g, x});
        hit = &pe->graphs.back();
    }
    HIPCHK(hipGraphLaunch(hit->exec, s));
    return CC_OK;
}

// ---------------------------------------------------------------------- single solve
int32_t finish(hipStream_t s, Ctrl* dctrl, Ctrl* hctrl, cc_stats* st) {
    HIPCHK(hipMemcpyAsync(hctrl, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st) st->host_syncs += 1;
    return CC_OK;
}

// No-sync end of a call: the status word is copied to the entry's pinned slot
// and an event recorded after it; cc_stream_status reads both later.
int32_t post_async(PoolEntry* e, hipStream_t s, const Ctrl* dctrl) {
    if (!e->async_slot) HIPCHK(hipHostMalloc((void**)&e->async_slot, 256, hipHostMallocDefault));
    if (!e->async_done) HIPCHK(hipEventCreateWithFlags(&e->async_done, hipEventDisableTiming));
    HIPCHK(hipMemcpyAsync(e->async_slot, &dctrl->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(e->async_done, s));
    e->async_called = true;
    return CC_OK;
}


// Enqueues the Atomic-Hook solve (Fig. 4) of one graph on s; no synchronisation.
// `ctrl` is the graph's control block, `bits` its giant bitmap (filter plans).
// Giant-filter buffers of one solve (null when the plan does not use them).
struct FilterBufs {
    uint32_t* bits = nullptr;
    uint32_t* hot_counts = nullptr;
    uint32_t* hot_tags = nullptr;
    uint32_t* hot_vals = nullptr;
    uint8_t* vtab = nullptr;  // vertex table (then hot_tags and hot_vals stay null)
};

FilterBufs filter_bufs(char* base, const Layout& L) {
    FilterBufs f;
    if (L.bits) f.bits = reinterpret_cast<uint32_t*>(base + L.bits);
    if (L.hot_counts && L.hot_tags == L.hot_vals) {
        f.hot_counts = reinterpret_cast<uint32_t*>(base + L.hot_counts);
        f.vtab = reinterpret_cast<uint8_t*>(base + L.hot_tags);
    } else if (L.hot_counts) {
        f.hot_counts = reinterpret_cast<uint32_t*>(base + L.hot_counts);
        f.hot_tags = reinterpret_cast<uint32_t*>(base + L.hot_tags);
        f.hot_vals = reinterpret_cast<uint32_t*>(base + L.hot_vals);
    }
    return f;
}

// Growth factor of the super-segments hooked after the giant filter is on:
// with the filter, later segments hook few edges, so they are taken in
// launches of 2, 8, 32, ... segments (from kSuperStart times the unfiltered
// prefix; each launch followed by a Multi-Jump and a bitmap refresh).
// Measured on R-MAT 24 (s = 512, from 1 segment): x2 3.81 ms, x4 3.76 ms,
// x8 3.88 ms -- fewer refreshes against a staler bitmap.
constexpr int64_t kSuperGrowth = 4;
// Segments of the first filtered launch, as a multiple of the unfiltered
// prefix (filter_after segments): R-MAT 24 (s = 512, launches of 2, 8, 32,
// 128 and 341 segments) 3.58 ms against 3.63 ms for 1, 3.64 for 4 and 3.61
// for 8; the same graph as CSR 4.74 against 4.76 ms for 1.
constexpr int64_t kSuperStart = 2;

int32_t enqueue_atomic(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                       const Plan& p, Ctrl* ctrl, const FilterBufs& fb, hipStream_t s, Timer& tm,
                       cc_stats* st) {
    uint32_t* bits = fb.bits;
    const bool hot = p.hot && fb.hot_tags != nullptr;
    const bool vhot = p.hot && fb.vtab != nullptr;
    const int S = p.segments;
    auto bound = [&](int64_t i) -> int64_t {
        if (i >= S) return m;
        return segment_start(m, i, S);
    };
    int hooks = 0, jumps = 0;
    TIMED(kPhaseOther, launch_init(pi, n, ctrl, s));
    if (p.filter != CC_FILTER_GIANT) {
        // Fig. 4: for each segment, Atomic-Hook the segment, then Multi-Jump all of V.
        for (int i = 0; i < S; ++i) {
            TIMED(kPhaseHook, launch_ahook(u, v, bound(i), bound(i + 1), pi, n, ctrl, nullptr,
                                           p.block, p.ept, p.coherent, p.halve, p.symmetric, s));
            TIMED(kPhaseCompress, launch_mj(pi, n, nullptr, p.coherent, s));
            ++hooks;
            ++jumps;
        }
    } else {
        const int fa = p.filter_after;
        for (int i = 0; i < fa; ++i) {
            TIMED(kPhaseHook, launch_ahook(u, v, bound(i), bound(i + 1), pi, n, ctrl, nullptr,
                                           p.block, p.ept, p.coherent, p.halve, p.symmetric, s));
            TIMED(kPhaseCompress, launch_mj(pi, n, nullptr, p.coherent, s));
            ++hooks;
            ++jumps;
        }
        TIMED(kPhaseOther, launch_sample_giant(u, m, pi, n, ctrl, 2048, s));
        TIMED(kPhaseOther, launch_bitmap(pi, n, ctrl, bits, s));
        if (hot) {
            TIMED(kPhaseOther, launch_hot_prepare(u, v, m, n, fb.hot_counts, fb.hot_tags,
                                                  p.hot_slots, s));
            TIMED(kPhaseOther, launch_hot_values(bits, fb.hot_tags, fb.hot_vals, ctrl,
                                                 p.hot_slots, s));
        }
        if (vhot) {
            TIMED(kPhaseOther, launch_hot_vprepare(u, v, m, n, fb.hot_counts, fb.vtab, s));
            TIMED(kPhaseOther, launch_hot_vvalues(bits, fb.vtab, ctrl, s));
        }
        // The rest of the list in super-segments that grow by kSuperGrowth,
        // each followed by a Compress and a bitmap refresh.
        int64_t g = fa, step = kSuperStart * fa;
        while (g < S) {
            const int64_t h = std::min<int64_t>(S, g + step);
            if (hot)
                TIMED(kPhaseHook, launch_ahook_hot(u, v, bound(g), bound(h), pi, n, ctrl, bits,
                                                   fb.hot_tags, fb.hot_vals, p.ept, p.hot_slots,
                                                   p.halve, p.symmetric, s));
            else if (vhot)
                TIMED(kPhaseHook, launch_ahook_hotv(u, v, bound(g), bound(h), pi, n, ctrl, bits,
                                                    fb.vtab, p.halve, p.symmetric, s));
            else
                TIMED(kPhaseHook, launch_ahook(u, v, bound(g), bound(h), pi, n, ctrl, bits,
                                               p.block, p.ept, p.coherent, p.halve, p.symmetric, s));
            if (h < S && !p.coherent) {
                // Compress, bitmap refresh and hot-word refresh in one pass
                TIMED(kPhaseCompress, launch_mj_bitmap(pi, n, ctrl, bits, hot ? fb.hot_tags : nullptr,
                                                       fb.hot_vals, p.hot_slots, fb.vtab, s));
            } else {
                TIMED(kPhaseCompress, launch_mj(pi, n, nullptr, p.coherent, s));
                if (h < S) TIMED(kPhaseOther, launch_bitmap(pi, n, ctrl, bits, s));
            }
            ++hooks;
            ++jumps;
            g = h;
            step *= kSuperGrowth;
        }
    }
    if (st) {
        st->hook_launches += hooks;
        st->compress_launches += jumps;
    }
    return CC_OK;
}

// The atomic-free Hook in blocks of K = rounds_per_check rounds, the host
// reading the control block after each block.  With `graph`, each block's
// launches (block b: rounds bK+1 .. bK+K; block 0 also the init) are
// captured once per (arrays, sizes, plan, b) and replayed.
// Hybrid plan: one atomic-free Hook round (Fig. 2) over all entries, in
// which each workgroup first joins its chunk of entries in an LDS window
// (launch_hook_window), and the compaction of the entries whose endpoints
// still have different parents into parent pairs; then one Atomic-Hook pass
// with path halving (Fig. 3) over those pairs and a final Multi-Jump (skipped
// on the device when no pair was active).  Trees only merge, so an entry
// dropped by the compaction stays satisfied; the pairs are vertices of the
// endpoints' trees, valid starting parents for the climb.  A fixed launch
// sequence: no host read until the end.
int32_t enqueue_hybrid(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                       const Plan& p, char* ws, const Layout& L, hipStream_t s, Timer& tm,
                       cc_stats* st) {
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    int2* F = reinterpret_cast<int2*>(ws + L.f0);
    const int grid_cap = device_cu_count() * 8;
    TIMED(kPhaseOther, launch_init(pi, n, ctrl, s));
    // the atomic-free round, each workgroup's chunk joined in an LDS window
    TIMED(kPhaseHook, launch_hook_window(u, v, m, pi, n, ctrl, s));
    // The compaction compares parents, not roots.  An entry whose endpoints
    // have equal parents is inside one tree and is dropped; one whose parents
    // differ is kept (also when they share a root), and the Atomic-Hook climbs
    // from that pair to the roots (every parent is a vertex of its endpoint's
    // tree, a valid start).  When the windows held most entries, nearly every
    // vertex already points at its chunk's local root and the extra pairs
    // are few, so no Multi-Jump runs first (4096^2 grid: it cost 58 us, the
    // pairs it saved far less); when more than a quarter of the entries were
    // hooked outside the windows (inputs without locality), the plain round's
    // chains would make most entries look active, and a Multi-Jump, gated on
    // the device by that count, makes the trees stars first.
    TIMED(kPhaseCompress, launch_mj1(pi, n, &ctrl->win_far, s, (uint32_t)(m / 4)));
    TIMED(kPhaseHook, launch_compact(1, u, v, m, F, F, L.cap, pi, n, ctrl, 0xffffffffu, p.block,
                                     p.ept, grid_cap, s));
    TIMED(kPhaseHook, launch_ahook_pairs(F, &ctrl->count[1], L.cap, pi, p.halve, grid_cap, s));
    TIMED(kPhaseCompress, launch_mj1(pi, n, &ctrl->count[1], s));
    if (st) {
        st->hook_launches += 3;
        st->compress_launches += 2;
    }
    return CC_OK;
}

int32_t solve_plain(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                    const Plan& p, char* ws, const Layout& L, hipStream_t s, PoolEntry* pe,
                    Ctrl* hctrl, bool use_graph, Timer& tm, cc_stats* st, int64_t* rounds_run) {
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    int2* F0 = reinterpret_cast<int2*>(ws + L.f0);
    int2* F1 = reinterpret_cast<int2*>(ws + L.f1);
    const int grid_cap = device_cu_count() * 8;
    const int K = p.rounds_per_check;
    auto enqueue_block = [&](int64_t b) -> int32_t {
        if (b == 0) TIMED(kPhaseOther, launch_init(pi, n, ctrl, s));
        for (int k = 0; k < K; ++k) {
            const int64_t r = b * K + k + 1;
            // sources and sizes are chosen on the device (round_src); the
            // grid covers the capacity and loops over what is there
            const int64_t work = (r == 1) ? m : L.cap;
            TIMED(kPhaseHook, launch_hook_plain((int)r, u, v, work, F0, F1, pi, n, ctrl, p.block,
                                                p.ept, grid_cap, s));
            if (r == 1)  // the round leaves chains
                TIMED(kPhaseCompress, launch_mj_deep(pi, n, s));
            else
                TIMED(kPhaseCompress, launch_mj1(pi, n, &ctrl->count[(r - 1) & 1], s));
            TIMED(kPhaseHook, launch_compact((int)r, u, v, work, F0, F1, L.cap, pi, n, ctrl,
                                             p.tau, p.block, p.ept, grid_cap, s));
        }
        return CC_OK;
    };
    int64_t r = 0;
    int hooks = 0, jumps = 0;
    for (int64_t b = 0;; ++b) {
        int32_t rc;
        if (use_graph) {
            KeyHash k;
            k.add(n).add(m).add(u).add(v).add(pi).add(ws).add(s).add(p.block).add(p.ept)
                .add(p.tau).add(K).add(b);
            rc = run_graph(pe, k.h, s, [&]() { return enqueue_block(b); });
        } else {
            rc = enqueue_block(b);
        }
        if (rc != CC_OK) return rc;
        r += K;
        hooks += 2 * K;
        jumps += K;
        rc = finish(s, ctrl, hctrl, st);
        if (rc != CC_OK) return rc;
        if (hctrl->status) break;  // reported by the caller
        if (hctrl->count[r & 1] == 0) break;
        if (r >= p.max_rounds) {
            *rounds_run = r;
            if (st) {
                st->hook_launches += hooks;
                st->compress_launches += jumps;
            }
            return fail(CC_ERR_NOCONVERGE, "atomic-free Hook did not converge within max_rounds");
        }
    }
    *rounds_run = r;
    if (st) {
        st->hook_launches += hooks;
        st->compress_launches += jumps;
    }
    return CC_OK;
}

// Fig. 1 exactly as the paper's baseline runs it: every Hook pass covers all
// entries, and the host reads a device "changed" flag after every launch
// (the CPU-GPU round trips that Section 1 sets out to remove).  Compress is
// either repeated single-level Jump launches (Fig. 2) or one Multi-Jump.
int32_t solve_host_loop(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                        const Plan& p, char* ws, hipStream_t s, Ctrl* hctrl, Timer& tm,
                        cc_stats* st) {
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    TIMED(kPhaseOther, launch_init(pi, n, ctrl, s));
    int64_t rounds = 0;
    int hooks = 0, jumps = 0;
    while (true) {
        ++rounds;
        HIPCHK(hipMemsetAsync(&ctrl->hook_changed, 0, 4, s));
        TIMED(kPhaseHook, launch_hook_flag(u, v, m, pi, n, ctrl, p.block, p.ept, s));
        ++hooks;
        int32_t rc = finish(s, ctrl, hctrl, st);
        if (rc != CC_OK) return rc;
        if (hctrl->status) break;
        const bool hooked = hctrl->hook_changed != 0;
        if (p.host_loop == CC_HOST_LOOP_MULTIJUMP) {
            TIMED(kPhaseCompress, launch_mj(pi, n, nullptr, p.coherent, s));
            ++jumps;
        } else {
            while (true) {
                HIPCHK(hipMemsetAsync(&ctrl->jump_changed, 0, 4, s));
                TIMED(kPhaseCompress, launch_jump(pi, n, ctrl, s));
                ++jumps;
                rc = finish(s, ctrl, hctrl, st);
                if (rc != CC_OK) return rc;
                if (!hctrl->jump_changed) break;
            }
        }
        if (!hooked) break;
        if (rounds >= p.max_rounds) {
            if (st) {
                st->rounds = (int32_t)rounds;
                st->hook_launches += hooks;
                st->compress_launches += jumps;
            }
            return fail(CC_ERR_NOCONVERGE, "Hook did not converge within max_rounds");
        }
    }
    int32_t rc = finish(s, ctrl, hctrl, st);
    if (rc != CC_OK) return rc;
    if (st) {
        st->rounds = (int32_t)rounds;
        st->hook_launches += hooks;
        st->compress_launches += jumps;
    }
    return CC_OK;
}

int32_t check_args(int32_t n, const int32_t* u, const int32_t* v, int64_t m, const int32_t* out) {
    if (n < 0) return fail(CC_ERR_ARG, "n < 0");
    if (m < 0) return fail(CC_ERR_ARG, "m < 0");
    if (m > 0 && (!u || !v)) return fail(CC_ERR_ARG, "null edge array with m > 0");
    if (n > 0 && !out) return fail(CC_ERR_ARG, "null out_label with n > 0");
    return CC_OK;
}


// Enqueues the solve of one graph with plan p on s into the workspace ws
// (laid out by L) and waits for it; `hctrl` receives the control block.
// `pe` (nullable) supplies the captured launch sequences of p.graph and the
// status slot of p.no_sync; without it neither is used (the caller has
// rejected both).
int32_t run_solve(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* out,
                  const Plan& p, const Layout& L, char* ws, Ctrl* hctrl, PoolEntry* pe,
                  hipStream_t s, cc_stats* st) {
    int32_t rc = CC_OK;
    Timer tm;
    tm.on = p.profile;
    tm.s = s;
    int64_t rounds = 0;
    const bool use_graph = p.graph && s != nullptr && !p.profile && pe != nullptr;
    if (p.hook == CC_HOOK_ATOMIC || p.hook == CC_HOOK_HYBRID) {
        // fixed launch sequences: no host read until the end
        auto enqueue = [&](cc_stats* sx) {
            if (p.hook == CC_HOOK_HYBRID)
                return enqueue_hybrid(n, u, v, m, out, p, ws, L, s, tm, sx);
            return enqueue_atomic(n, u, v, m, out, p, reinterpret_cast<Ctrl*>(ws),
                                  filter_bufs(ws, L), s, tm, sx);
        };
        if (use_graph) {
            KeyHash k;
            k.add(n).add(m).add(u).add(v).add(out).add(ws).add(s).add(p.hook).add(p.segments)
                .add(p.filter).add(p.filter_after).add(p.block).add(p.ept).add(p.coherent)
                .add(p.hot).add(p.hot_slots).add(p.halve).add(p.symmetric);
            rc = run_graph(pe, k.h, s, [&]() { return enqueue(st); });
        } else {
            rc = enqueue(st);
        }
        if (rc == CC_OK && p.no_sync && pe) {
            rc = post_async(pe, s, reinterpret_cast<const Ctrl*>(ws));
            if (st) st->giant_label = -1;  // not known without a synchronisation
            return rc;
        }
        if (rc == CC_OK) rc = finish(s, reinterpret_cast<Ctrl*>(ws), hctrl, st);
    } else if (p.host_loop != CC_HOST_LOOP_OFF) {
        rc = solve_host_loop(n, u, v, m, out, p, ws, s, hctrl, tm, st);
    } else {
        rc = solve_plain(n, u, v, m, out, p, ws, L, s, pe, hctrl, use_graph, tm, st, &rounds);
    }
    if (rc != CC_OK && rc != CC_ERR_NOCONVERGE) return rc;
    const Ctrl& c = *hctrl;
    tm.collect(st);
    if (st) {
        st->filter_used = (p.filter == CC_FILTER_GIANT && c.filter_on) ? 1 : 0;
        st->giant_label = st->filter_used ? c.giant : -1;
        if (p.hook == CC_HOOK_PLAIN && p.host_loop == CC_HOST_LOOP_OFF) {
            st->rounds = c.rounds;
            st->active_edges = c.active_round1;
        }
    }
    if (c.status & kStatusRange) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n)");
    if (c.status & kStatusOverflow) return fail(CC_ERR_NOMEM, "frontier capacity exceeded");
    return rc;
}

void init_stats(cc_stats* st, const Plan& p) {
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    st->hook = p.hook;
    st->segments = p.hook == CC_HOOK_ATOMIC ? p.segments : 0;
    st->giant_label = -1;
}

}  // namespace

int32_t labels_impl(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* out,
                    const cc_options* opts, void* workspace, size_t ws_bytes, hipStream_t s,
                    cc_stats* st) {
    int32_t rc = check_args(n, u, v, m, out);
    if (rc != CC_OK) return rc;
    Plan p;
    rc = make_plan(n, m, opts, p);
    if (rc != CC_OK) return rc;
    init_stats(st, p);
    if (n == 0) {
        if (m > 0) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n) (n == 0)");
        return CC_OK;
    }
    const Layout L = layout(n, m, p);
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    rc = ensure_host(pe);
    if (rc != CC_OK) return rc;
    char* ws;
    if (workspace) {
        if (ws_bytes < L.total) return fail(CC_ERR_NOMEM, "workspace smaller than cc_workspace_bytes()");
        if ((uintptr_t)workspace & 255) return fail(CC_ERR_ARG, "workspace must be 256-byte aligned");
        ws = static_cast<char*>(workspace);
    } else {
        rc = ensure_dev(pe, L.total);
        if (rc != CC_OK) return rc;
        ws = static_cast<char*>(pe->dev);
    }
    return run_solve(n, u, v, m, out, p, L, ws, pe->host_ctrl, pe, s, st);
}

// ---------------------------------------------------------------------- no-allocation solve
// cc_labels_noalloc: the solve of cc_labels_ex with its workspace taken from
// a fixed device array instead of the pool or the caller, for callers that
// must not allocate.  One array per device (each GPU the library runs on
// holds its own copy until the process ends); host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
namespace {

static __device__ __align__(256) char scratch[CC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];   // one call at a time per device
char* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, guarded as above

}  // namespace

int32_t labels_noalloc_impl(int32_t n, const int32_t* u, const int32_t* v, int64_t m,
                            int32_t* out, const cc_options* opts, hipStream_t s, cc_stats* st) {
    int32_t rc = check_args(n, u, v, m, out);
    if (rc != CC_OK) return rc;
    if (opts && (opts->graph != 0 || opts->no_sync != 0 || opts->profile != 0))
        return fail(CC_ERR_ARG, "cc_labels_noalloc: graph, no_sync and profile must be 0");
    Plan p;
    rc = make_plan(n, m, opts, p);
    if (rc != CC_OK) return rc;
    Layout L = layout(n, m, p);
    if (L.total > (size_t)CC_NOALLOC_SCRATCH_BYTES && (!opts || opts->hook == CC_HOOK_AUTO)) {
        // the automatic choice falls back to plans whose workspace fits: the
        // Atomic-Hook (no frontier), then without the giant filter (256 bytes)
        cc_options o;
        if (opts) o = *opts;
        else cc_options_init(&o);
        o.hook = CC_HOOK_ATOMIC;
        rc = make_plan(n, m, &o, p);
        if (rc != CC_OK) return rc;
        L = layout(n, m, p);
        if (L.total > (size_t)CC_NOALLOC_SCRATCH_BYTES) {
            o.filter = CC_FILTER_OFF;
            rc = make_plan(n, m, &o, p);
            if (rc != CC_OK) return rc;
            L = layout(n, m, p);
        }
    }
    if (L.total > (size_t)CC_NOALLOC_SCRATCH_BYTES)
        return fail(CC_ERR_NOMEM, "cc_labels_noalloc: the plan needs " + std::to_string(L.total) +
                                      " bytes of workspace; the fixed buffer holds " +
                                      std::to_string((size_t)CC_NOALLOC_SCRATCH_BYTES) +
                                      " (use cc_labels_ex, or the automatic hook)");
    init_stats(st, p);
    if (n == 0) {
        if (m > 0) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n) (n == 0)");
        return CC_OK;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CC_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255))
            return fail(CC_ERR_HIP, "cc_labels_noalloc: unusable address of the fixed buffer");
        g_scratch_ptr[dev] = static_cast<char*>(ptr);
    }
    // every kernel of the solve writes the workspace words it reads (the
    // control block is reset by the init kernel), so the previous call's
    // contents need no clearing
    Ctrl hctrl;
    return run_solve(n, u, v, m, out, p, L, g_scratch_ptr[dev], &hctrl, nullptr, s, st);
}

// ---------------------------------------------------------------------- streamed solve
// Edges in host memory, larger than one wants to (or can) hold in HBM.  The
// Atomic-Hook reads every entry exactly once, so the list is cut into chunks
// that are copied host-to-device on a copy stream into two staging buffers
// (double buffering: chunk i+1 is copied while chunk i is hooked) and hooked
// on the caller's stream, each chunk followed by a Multi-Jump (Fig. 4 with one
// segment per chunk).  With the giant filter, the first chunk's Compress is
// followed by the sample and the bitmap, which later chunks use and which is
// rebuilt after each chunk's Compress.  Only pi, the bitmap and the staging
// buffers (2 x 2 x chunk x 4 bytes) occupy device memory.
int32_t stream_impl(int32_t n, const int32_t* hu, const int32_t* hv, int64_t m, int32_t* out,
                    int64_t chunk, const cc_options* opts, hipStream_t s, cc_stats* st) {
    int32_t rc = check_args(n, hu, hv, m, out);
    if (rc != CC_OK) return rc;
    if (chunk < 0) return fail(CC_ERR_ARG, "chunk_entries < 0");
    if (chunk == 0) chunk = int64_t(1) << 24;
    chunk = std::max<int64_t>(4, chunk & ~int64_t(3));
    if (opts && opts->hook == CC_HOOK_PLAIN)
        return fail(CC_ERR_ARG, "streamed solves use the Atomic-Hook (each entry is read once)");
    if (opts && opts->no_sync)
        return fail(CC_ERR_ARG, "cc_options.no_sync is for cc_labels_ex and cc_labels_csr only");
    Plan p;
    rc = make_plan(n, m, opts, p, kInputAtomicOnly);
    if (rc != CC_OK) return rc;
    // Giant filter: as asked, or (auto) for dense lists that span several chunks.
    const int32_t fopt = opts ? opts->filter : CC_FILTER_AUTO;
    const bool filter = fopt == CC_FILTER_GIANT ||
                        (fopt == CC_FILTER_AUTO && m >= 8 * (int64_t)n && m > chunk);
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->hook = CC_HOOK_ATOMIC;
        st->giant_label = -1;
    }
    if (n == 0) {
        if (m > 0) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n) (n == 0)");
        return CC_OK;
    }
    const int64_t chunks = std::max<int64_t>(1, (m + chunk - 1) / chunk);
    const size_t bits_bytes = filter ? align256(((size_t)n + 31) / 32 * 4) : 0;
    const size_t stage = align256((size_t)chunk * 4);
    const size_t total = 256 + bits_bytes + 4 * stage;
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    rc = ensure_host(pe);
    if (rc != CC_OK) return rc;
    rc = ensure_dev(pe, total);
    if (rc != CC_OK) return rc;
    if (!pe->copy_stream) HIPCHK(hipStreamCreateWithFlags(&pe->copy_stream, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        if (!pe->copied[i]) HIPCHK(hipEventCreateWithFlags(&pe->copied[i], hipEventDisableTiming));
        if (!pe->consumed[i]) HIPCHK(hipEventCreateWithFlags(&pe->consumed[i], hipEventDisableTiming));
    }
    char* ws = static_cast<char*>(pe->dev);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    uint32_t* bits = filter ? reinterpret_cast<uint32_t*>(ws + 256) : nullptr;
    int32_t* su[2] = {reinterpret_cast<int32_t*>(ws + 256 + bits_bytes),
                      reinterpret_cast<int32_t*>(ws + 256 + bits_bytes + stage)};
    int32_t* sv[2] = {reinterpret_cast<int32_t*>(ws + 256 + bits_bytes + 2 * stage),
                      reinterpret_cast<int32_t*>(ws + 256 + bits_bytes + 3 * stage)};
    hipStream_t cs = pe->copy_stream;
    HIPCHK(launch_init(out, n, ctrl, s));
    // The copy stream must not overwrite a staging buffer before the solve
    // stream is done with it, nor start before init is queued (ordering only).
    HIPCHK(hipEventRecord(pe->consumed[0], s));
    HIPCHK(hipEventRecord(pe->consumed[1], s));
    int hooks = 0, jumps = 0;
    for (int64_t i = 0; i < chunks; ++i) {
        const int b = (int)(i & 1);
        const int64_t e0 = i * chunk, len = std::min<int64_t>(chunk, m - e0);
        HIPCHK(hipStreamWaitEvent(cs, pe->consumed[b], 0));
        if (len > 0) {
            HIPCHK(hipMemcpyAsync(su[b], hu + e0, (size_t)len * 4, hipMemcpyHostToDevice, cs));
            HIPCHK(hipMemcpyAsync(sv[b], hv + e0, (size_t)len * 4, hipMemcpyHostToDevice, cs));
        }
        HIPCHK(hipEventRecord(pe->copied[b], cs));
        HIPCHK(hipStreamWaitEvent(s, pe->copied[b], 0));
        const bool filtered = filter && i > 0;
        HIPCHK(launch_ahook(su[b], sv[b], 0, len, out, n, ctrl, filtered ? bits : nullptr, p.block,
                            p.ept, p.coherent, p.halve, p.symmetric, s));
        HIPCHK(launch_mj(out, n, nullptr, p.coherent, s));
        ++hooks;
        ++jumps;
        if (filter && i == 0) HIPCHK(launch_sample_giant(su[b], len, out, n, ctrl, 2048, s));
        if (filter && i + 1 < chunks) HIPCHK(launch_bitmap(out, n, ctrl, bits, s));
        HIPCHK(hipEventRecord(pe->consumed[b], s));
    }
    rc = finish(s, ctrl, pe->host_ctrl, st);
    if (rc != CC_OK) return rc;
    if (st) {
        st->segments = (int32_t)chunks;
        st->hook_launches = hooks;
        st->compress_launches = jumps;
        st->filter_used = (filter && pe->host_ctrl->filter_on) ? 1 : 0;
        st->giant_label = st->filter_used ? pe->host_ctrl->giant : -1;
    }
    if (pe->host_ctrl->status & kStatusRange) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n)");
    return CC_OK;
}

// ---------------------------------------------------------------------- CSR input
// Same plan as a pair list of m entries (segments of the col[] array, each
// followed by a Multi-Jump; with the giant filter the growing super-segments
// of enqueue_atomic); the first endpoint of an entry is its row.  The hybrid
// plan is the pair-list one: an atomic-free Hook pass over all entries, a
// Multi-Jump, the still-active entries compacted to root pairs, then the
// Atomic-Hook (with path halving) over those pairs and a Multi-Jump; the
// first pass joins nearly everything with plain stores, and the Atomic-Hook
// restores the links it overwrote (grid as CSR 0.73 ms; 0.77 ms with an
// Atomic-Hook pass over all entries instead of the compaction).
int32_t csr_impl(int32_t n, const int64_t* row_ptr, const int32_t* col, int64_t m, int32_t* out,
                 const cc_options* opts, hipStream_t s, cc_stats* st) {
    if (n < 0 || m < 0) return fail(CC_ERR_ARG, "n < 0 or m < 0");
    if (!row_ptr) return fail(CC_ERR_ARG, "null row_ptr");
    if (m > 0 && !col) return fail(CC_ERR_ARG, "null col with m > 0");
    if (n > 0 && !out) return fail(CC_ERR_ARG, "null out_label with n > 0");
    if (opts && opts->hook == CC_HOOK_PLAIN)
        return fail(CC_ERR_ARG, "CSR input uses the Atomic-Hook or the hybrid plan");
    Plan p;
    int32_t rc = make_plan(n, m, opts, p, kInputCsr);
    if (rc != CC_OK) return rc;
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->hook = p.hook;
        st->segments = p.hook == CC_HOOK_ATOMIC ? p.segments : 0;
        st->giant_label = -1;
    }
    if (n == 0) {
        if (m > 0) return fail(CC_ERR_RANGE, "entries in a graph with no vertices");
        return CC_OK;
    }
    const bool filter = p.filter == CC_FILTER_GIANT;
    const size_t bits_bytes = filter ? align256(((size_t)n + 31) / 32 * 4) : 0;
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    rc = ensure_host(pe);
    if (rc != CC_OK) return rc;
    // the hybrid plan's frontier of root pairs (8 B x m)
    const size_t frontier_bytes = p.hook == CC_HOOK_HYBRID ? align256((size_t)m * 8) : 0;
    rc = ensure_dev(pe, 256 + bits_bytes + frontier_bytes);
    if (rc != CC_OK) return rc;
    char* ws = static_cast<char*>(pe->dev);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    uint32_t* bits = filter ? reinterpret_cast<uint32_t*>(ws + 256) : nullptr;
    int2* F = frontier_bytes ? reinterpret_cast<int2*>(ws + 256 + bits_bytes) : nullptr;
    const int S = p.segments;
    auto bound = [&](int64_t i) -> int64_t { return i >= S ? m : segment_start(m, i, S); };
    Timer tm;
    tm.on = p.profile;
    tm.s = s;
    int hooks = 0, jumps = 0;
    TIMED(kPhaseOther, launch_init(out, n, ctrl, s));
    TIMED(kPhaseOther, launch_csr_check(row_ptr, n, m, ctrl, s));
    if (p.hook == CC_HOOK_HYBRID) {
        TIMED(kPhaseHook, launch_ahook_csr(row_ptr, col, n, 0, m, out, ctrl, nullptr, p.symmetric,
                                           false, /*plain=*/true, s));
        TIMED(kPhaseCompress, launch_mj_deep(out, n, s));  // the pass leaves chains
        // the entries still active, as root pairs, then the Atomic-Hook over
        // those pairs (as the pair-list hybrid plan)
        TIMED(kPhaseHook, launch_compact_csr(row_ptr, col, n, m, out, F, &ctrl->count[1],
                                             p.symmetric, s));
        TIMED(kPhaseHook, launch_ahook_pairs(F, &ctrl->count[1], m, out, p.halve,
                                             device_cu_count() * 8, s));
        TIMED(kPhaseCompress, launch_mj1(out, n, &ctrl->count[1], s));
        hooks = 3;
        jumps = 2;
    } else if (!filter) {
        for (int i = 0; i < S; ++i) {
            TIMED(kPhaseHook, launch_ahook_csr(row_ptr, col, n, bound(i), bound(i + 1), out, ctrl,
                                               nullptr, p.symmetric, p.halve, false, s));
            TIMED(kPhaseCompress, launch_mj(out, n, nullptr, false, s));
            ++hooks;
            ++jumps;
        }
    } else {
        const int fa = p.filter_after;
        for (int i = 0; i < fa; ++i) {
            TIMED(kPhaseHook, launch_ahook_csr(row_ptr, col, n, bound(i), bound(i + 1), out, ctrl,
                                               nullptr, p.symmetric, p.halve, false, s));
            TIMED(kPhaseCompress, launch_mj(out, n, nullptr, false, s));
            ++hooks;
            ++jumps;
        }
        // endpoints sampled from col[] (the second endpoints of the entries)
        TIMED(kPhaseOther, launch_sample_giant(col, m, out, n, ctrl, 2048, s));
        TIMED(kPhaseOther, launch_bitmap(out, n, ctrl, bits, s));
        int64_t g = fa, step = kSuperStart * fa;
        while (g < S) {
            const int64_t h = std::min<int64_t>(S, g + step);
            TIMED(kPhaseHook, launch_ahook_csr(row_ptr, col, n, bound(g), bound(h), out, ctrl, bits,
                                               p.symmetric, p.halve, false, s));
            TIMED(kPhaseCompress, launch_mj(out, n, nullptr, false, s));
            ++hooks;
            ++jumps;
            if (h < S) TIMED(kPhaseOther, launch_bitmap(out, n, ctrl, bits, s));
            g = h;
            step *= kSuperGrowth;
        }
    }
    if (p.no_sync) {
        if (st) {
            st->hook_launches = hooks;
            st->compress_launches = jumps;
        }
        return post_async(pe, s, ctrl);
    }
    rc = finish(s, ctrl, pe->host_ctrl, st);
    if (rc != CC_OK) return rc;
    tm.collect(st);
    if (st) {
        st->hook_launches = hooks;
        st->compress_launches = jumps;
        st->filter_used = (filter && pe->host_ctrl->filter_on) ? 1 : 0;
        st->giant_label = st->filter_used ? pe->host_ctrl->giant : -1;
    }
    if (pe->host_ctrl->status & kStatusRange)
        return fail(CC_ERR_RANGE, "column id outside [0, n) or malformed row_ptr");
    return CC_OK;
}

size_t workspace_bytes_impl(int32_t n, int64_t m, const cc_options* opts) {
    if (n < 0 || m < 0) return 0;
    Plan p;
    if (make_plan(n, m, opts, p) != CC_OK) return 0;
    return layout(n, m, p).total;
}

// ---------------------------------------------------------------------- graph lists
// Segments of an LDS-solved graph: min(cap, round(m / n)) (at least 1), or
// round(m / n) for cap 0; small caps by comparison, without a division.
int32_t lds_segments(int64_t m, int64_t n, int32_t cap) {
    if (cap > 0 && cap <= 16 && m < (int64_t(1) << 61)) {
        int32_t k = cap;  // round(m / n) >= k  <=>  2m >= (2k - 1) n
        while (k > 1 && 2 * m < (2 * (int64_t)k - 1) * n) --k;
        return k;
    }
    const int32_t r = (int32_t)std::min<int64_t>(int64_t(1) << 20, round_ratio(m, n));
    return cap > 0 ? std::min(r, cap) : r;
}

// The graph-list solve over any graph accessor: graph_at(g) returns graph g
// as a cc_graph (the caller's array, or one computed from batch offsets, so a
// batch never materialises a list).  Small graphs (n <= CC_BATCH_LDS_MAX_N)
// go to one persistent LDS launch whose workgroups take them largest first;
// every larger graph gets the device-memory Atomic-Hook solve with its own
// control block.  Everything is enqueued on `s`; the call ends with one
// synchronisation, after which the LDS launch's pinned status word and the
// large graphs' control blocks (copied back) are read.
template <class GraphAt>
int32_t list_core(int32_t count, GraphAt&& graph_at, const cc_options* opts, hipStream_t s,
                  cc_stats* st, void* workspace, size_t ws_bytes, size_t* ws_needed) {
    if (ws_needed) *ws_needed = 0;
    if (count < 0) return fail(CC_ERR_ARG, "graph count < 0");
    if (opts && opts->no_sync)
        return fail(CC_ERR_ARG, "cc_options.no_sync is for cc_labels_ex and cc_labels_csr only");
    // Per-graph segment count of the LDS solver: min(S, round(m/n)) for a
    // cap S > 0.  Default (S = 0): 2 with path halving in the LDS climb (the
    // default; measured best, batch of 10,000 ER graphs 1.54 ms against 1.78
    // for the paper's schedule without halving), the paper's round(m/n)
    // (no cap) with halving off.
    const int32_t ph = opts ? opts->path_halving : CC_HALVE_AUTO;
    if (ph < CC_HALVE_AUTO || ph > CC_HALVE_OFF) return fail(CC_ERR_ARG, "unknown cc_options.path_halving");
    const bool lds_halve = ph != CC_HALVE_OFF;
    int32_t seg_cap = opts ? opts->segments : 0;
    if (seg_cap < 0) return fail(CC_ERR_ARG, "cc_options.segments < 0");
    // workgroup size of the LDS solver (0 = 1024)
    const int32_t lds_block = (opts && opts->block) ? opts->block : 1024;
    if (lds_block < 64 || lds_block > 1024 || lds_block % 64)
        return fail(CC_ERR_ARG, "cc_options.block must be a multiple of 64 in [64, 1024]");
    if (seg_cap == 0 && lds_halve) seg_cap = 2;
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->giant_label = -1;
    }
    if (count == 0) return CC_OK;
    // host scratch kept per thread: a call allocates nothing once warm
    static thread_local std::vector<int32_t> small, large, sorted;
    static thread_local std::vector<uint8_t> cls;
    small.clear();
    large.clear();
    small.reserve((size_t)count);
    cls.resize((size_t)count);
    int64_t start[257] = {0};
    int64_t maxn_small = 0;
    for (int32_t g = 0; g < count; ++g) {
        const cc_graph G = graph_at(g);
        if (G.reserved != 0) return fail(CC_ERR_ARG, "cc_graph.reserved must be zero");
        if (G.n < 0 || G.m < 0) return fail(CC_ERR_ARG, "graph with n < 0 or m < 0");
        if (G.m > 0 && (!G.edges_u || !G.edges_v)) return fail(CC_ERR_ARG, "null edge array");
        if (G.n > 0 && !G.out_label) return fail(CC_ERR_ARG, "null out_label");
        if (G.n == 0) {
            if (G.m > 0) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n) (empty graph)");
            continue;
        }
        if (G.n <= CC_BATCH_LDS_MAX_N) {
            const uint8_t c = (uint8_t)(255 - size_class((uint64_t)G.m + (uint64_t)G.n));
            cls[small.size()] = c;
            ++start[c + 1];
            small.push_back(g);
            maxn_small = std::max<int64_t>(maxn_small, G.n);
        } else {
            large.push_back(g);
        }
    }
    // Largest first (longest-processing-time order): the queue's tail holds
    // the small graphs, which even out the workgroups' finishing times.  An
    // O(count) counting sort on a size class (four classes per power of two
    // of m + n) gives that order; a comparison sort of 10,000 graphs costs
    // about a millisecond of host time, more than a third of the solve.
    {
        const size_t k = small.size();
        for (int c = 0; c < 256; ++c) start[c + 1] += start[c];
        sorted.resize(k);
        for (size_t i = 0; i < k; ++i) sorted[start[cls[i]]++] = small[i];
        small.swap(sorted);
    }
    const int32_t ns = (int32_t)small.size();
    const int32_t nl = (int32_t)large.size();
    std::vector<Plan> plans(nl);
    std::vector<size_t> region_off(nl, 0);
    std::vector<Layout> layouts(nl);
    // Workspace: the LDS launch's control block, its descriptors right after
    // (one copy from the staging buffer uploads both and clears the block),
    // then the large graphs' control blocks and their regions.
    const size_t desc_off = sizeof(Ctrl);
    const size_t desc_bytes = align256((size_t)ns * sizeof(GraphDesc));
    const size_t lctrl_off = desc_off + desc_bytes;
    size_t off = lctrl_off + align256((size_t)nl * sizeof(Ctrl));
    for (int32_t i = 0; i < nl; ++i) {
        const cc_graph G = graph_at(large[i]);
        int32_t rc = make_plan(G.n, G.m, nullptr, plans[i], kInputAtomicOnly);
        if (rc != CC_OK) return rc;
        layouts[i] = layout(G.n, G.m, plans[i]);  // its control block is lctrls[i] instead
        region_off[i] = off;
        off += align256(layouts[i].total);
    }
    if (ws_needed) {  // size query only
        *ws_needed = off;
        return CC_OK;
    }
    if (workspace) {
        if (ws_bytes < off) return fail(CC_ERR_NOMEM, "graph-list workspace too small");
        if ((uintptr_t)workspace & 255) return fail(CC_ERR_ARG, "workspace must be 256-byte aligned");
    }
    if (ns > 0) HIPCHK(prepare_batch_lds());
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    int32_t rc = ensure_host(pe, std::max(1, nl));
    if (rc != CC_OK) return rc;
    if (!pe->batch_status)
        HIPCHK(hipHostMalloc((void**)&pe->batch_status, 256, hipHostMallocDefault));
    if (!workspace) {
        rc = ensure_dev(pe, off);
        if (rc != CC_OK) return rc;
    }
    if (ns > 0) {
        rc = ensure_stage(pe, desc_off + desc_bytes);
        if (rc != CC_OK) return rc;
    }
    char* ws = workspace ? static_cast<char*>(workspace) : static_cast<char*>(pe->dev);
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);                 // the LDS launch's
    Ctrl* lctrls = reinterpret_cast<Ctrl*>(ws + lctrl_off);   // the large graphs'
    // The LDS launch reports a bad endpoint in a pinned host word, so a call
    // without large graphs needs no copy back before its synchronisation.
    *pe->batch_status = 0;
    if (ns > 0) {
        std::memset(pe->host_stage, 0, desc_off);  // the cleared control block
        GraphDesc* hd = reinterpret_cast<GraphDesc*>(static_cast<char*>(pe->host_stage) + desc_off);
        for (int32_t i = 0; i < ns; ++i) {
            const cc_graph G = graph_at(small[i]);
            GraphDesc& d = hd[i];
            d.u = G.edges_u;
            d.v = G.edges_v;
            d.out = G.out_label;
            d.m = G.m;
            d.n = G.n;
            // average-degree segmentation per graph (Section 3.B), capped
            d.segments = lds_segments(G.m, G.n, seg_cap);
        }
    }
    // The launch sequence: clear the LDS solver's control block, upload the
    // descriptors, one persistent LDS launch, then every large graph's solve.
    Timer tm;
    auto enqueue = [&]() -> int32_t {
        if (ns > 0) {
            HIPCHK(hipMemcpyAsync(ws, pe->host_stage, desc_off + desc_bytes, hipMemcpyHostToDevice, s));
            HIPCHK(launch_batch_lds(reinterpret_cast<GraphDesc*>(ws + desc_off), ns,
                                    (int32_t)maxn_small, &ctrl->queue_head, pe->batch_status,
                                    lds_halve, device_cu_count(), s, lds_block));
        }
        for (int32_t i = 0; i < nl; ++i) {
            const cc_graph G = graph_at(large[i]);
            int32_t r2 = enqueue_atomic(G.n, G.edges_u, G.edges_v, G.m, G.out_label, plans[i],
                                        &lctrls[i], filter_bufs(ws + region_off[i], layouts[i]),
                                        s, tm, nullptr);
            if (r2 != CC_OK) return r2;
        }
        return CC_OK;
    };
    const bool use_graph = opts && opts->graph == 1 && s != nullptr;
    if (use_graph) {
        KeyHash k;
        // The LDS graphs' descriptors are not part of the key: the captured
        // copy node re-reads the pinned staging buffer, rewritten above, at
        // every replay.  Only what the capture bakes in is: sizes, pointers,
        // the LDS launch shape, and each large graph's arrays and plan.
        k.add(count).add(ws).add(s).add(pe->host_stage).add(seg_cap).add(lds_halve)
            .add(maxn_small).add(ns).add(nl).add(lds_block);
        for (int32_t i = 0; i < nl; ++i) {
            const cc_graph G = graph_at(large[i]);
            k.add(G.edges_u).add(G.edges_v).add(G.out_label).add(G.m).add(G.n);
        }
        rc = run_graph(pe, k.h, s, enqueue);
    } else {
        rc = enqueue();
    }
    if (rc != CC_OK) return rc;
    if (st) st->hook_launches += (ns > 0 ? 1 : 0);
    if (nl > 0)
        HIPCHK(hipMemcpyAsync(pe->host_ctrl, lctrls, sizeof(Ctrl) * nl, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st) st->host_syncs += 1;
    bool bad = (*(volatile int32_t*)pe->batch_status & kStatusRange) != 0;
    for (int32_t i = 0; i < nl; ++i) bad |= (pe->host_ctrl[i].status & kStatusRange) != 0;
    if (bad) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n_g)");
    return CC_OK;
}

int32_t list_impl(int32_t count, const cc_graph* graphs, const cc_options* opts, hipStream_t s,
                  cc_stats* st, void* workspace, size_t ws_bytes, size_t* ws_needed) {
    if (count > 0 && !graphs) {
        if (ws_needed) *ws_needed = 0;
        return fail(CC_ERR_ARG, "null graph list");
    }
    return list_core(count, [graphs](int32_t g) { return graphs[g]; }, opts, s, st, workspace,
                     ws_bytes, ws_needed);
}

int32_t batch_lds_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int64_t* hvo,
                       const int64_t* heo, const int32_t* u, const int32_t* v, int32_t* out,
                       int32_t max_n, const cc_options* opts, hipStream_t s, cc_stats* st);

int32_t batch_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int32_t* u,
                   const int32_t* v, int32_t* out, const cc_options* opts, hipStream_t s,
                   cc_stats* st) {
    if (B < 0) return fail(CC_ERR_ARG, "num_graphs < 0");
    if (opts && opts->no_sync)
        return fail(CC_ERR_ARG, "cc_options.no_sync is for cc_labels_ex and cc_labels_csr only");
    if (B == 0) {
        if (st) {
            std::memset(st, 0, sizeof *st);
            st->giant_label = -1;
        }
        return CC_OK;
    }
    if (!vo || !eo) return fail(CC_ERR_ARG, "null offsets");
    if (vo[0] != 0 || eo[0] != 0) return fail(CC_ERR_ARG, "offsets must start at 0");
    int64_t max_n = 0;
    for (int32_t g = 0; g < B; ++g) {
        const int64_t nv = vo[g + 1] - vo[g], ne = eo[g + 1] - eo[g];
        if (nv < 0 || ne < 0) return fail(CC_ERR_ARG, "offsets must be non-decreasing");
        if (nv > INT32_MAX) return fail(CC_ERR_ARG, "graph with 2^31 or more vertices");
        max_n = std::max(max_n, nv);
    }
    if (eo[B] > 0 && (!u || !v)) return fail(CC_ERR_ARG, "null edge array");
    if (vo[B] > 0 && !out) return fail(CC_ERR_ARG, "null out_label");
    // Every graph LDS-sized: the offsets are copied to the device as they are
    // and the graphs ordered and described there (the device-offset path),
    // which costs less host time than building the descriptors here.
    if (max_n <= CC_BATCH_LDS_MAX_N)
        return batch_lds_impl(B, nullptr, nullptr, vo, eo, u, v, out,
                              (int32_t)std::max<int64_t>(1, max_n), opts, s, st);
    // graph g straight from the offsets: no list of B graphs is built
    auto graph_at = [=](int32_t g) {
        cc_graph G;
        const int64_t ne = eo[g + 1] - eo[g];
        G.edges_u = ne ? u + eo[g] : nullptr;
        G.edges_v = ne ? v + eo[g] : nullptr;
        G.out_label = out ? out + vo[g] : nullptr;
        G.m = ne;
        G.n = (int32_t)(vo[g + 1] - vo[g]);
        G.reserved = 0;
        return G;
    };
    return list_core(B, graph_at, opts, s, st, nullptr, 0, nullptr);
}

// Device offsets: the preparation workgroup builds the descriptors and the
// largest-first order on the device (no host pass over the graphs), then the
// persistent LDS launch solves them; one synchronisation.
// The LDS batch with offsets in device memory (vo, eo), or in host memory
// (hvo, heo non-null: copied through the pinned staging buffer into the
// workspace first, one copy per call).
int32_t batch_lds_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int64_t* hvo,
                       const int64_t* heo, const int32_t* u, const int32_t* v, int32_t* out,
                       int32_t max_n, const cc_options* opts, hipStream_t s, cc_stats* st) {
    if (B < 0) return fail(CC_ERR_ARG, "num_graphs < 0");
    if (opts && opts->no_sync)
        return fail(CC_ERR_ARG, "cc_options.no_sync is for cc_labels_ex and cc_labels_csr only");
    const int32_t ph = opts ? opts->path_halving : CC_HALVE_AUTO;
    if (ph < CC_HALVE_AUTO || ph > CC_HALVE_OFF) return fail(CC_ERR_ARG, "unknown cc_options.path_halving");
    const bool lds_halve = ph != CC_HALVE_OFF;
    int32_t seg_cap = opts ? opts->segments : 0;
    if (seg_cap < 0) return fail(CC_ERR_ARG, "cc_options.segments < 0");
    if (seg_cap == 0 && lds_halve) seg_cap = 2;
    const int32_t lds_block = (opts && opts->block) ? opts->block : 1024;
    if (lds_block < 64 || lds_block > 1024 || lds_block % 64)
        return fail(CC_ERR_ARG, "cc_options.block must be a multiple of 64 in [64, 1024]");
    if (max_n < 1 || max_n > CC_BATCH_LDS_MAX_N)
        return fail(CC_ERR_ARG, "max_n must be in [1, CC_BATCH_LDS_MAX_N]");
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->giant_label = -1;
    }
    if (B == 0) return CC_OK;
    // null edge or label arrays are allowed for graphs without entries /
    // vertices; the preparation launch checks that on the device
    const bool staged = hvo && heo;
    if (!staged && (!vo || !eo)) return fail(CC_ERR_ARG, "null offsets");
    if ((size_t)B > (SIZE_MAX - sizeof(Ctrl)) / sizeof(GraphDesc)) return fail(CC_ERR_ARG, "too many graphs");
    const size_t desc_off = sizeof(Ctrl);
    const size_t rows_off = desc_off + align256((size_t)B * sizeof(GraphDesc));
    const size_t off_bytes = align256(((size_t)B + 1) * 8);  // one offset array
    const size_t offs_off = rows_off + align256((((size_t)B + 1023) / 1024 + 1) * 256 * 4);
    const size_t total = offs_off + (staged ? 2 * off_bytes : 0);
    HIPCHK(prepare_batch_lds());
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    int32_t rc = ensure_dev(pe, total);
    if (rc != CC_OK) return rc;
    if (staged) {
        rc = ensure_stage(pe, 2 * off_bytes);
        if (rc != CC_OK) return rc;
        std::memcpy(pe->host_stage, hvo, ((size_t)B + 1) * 8);
        std::memcpy(static_cast<char*>(pe->host_stage) + off_bytes, heo, ((size_t)B + 1) * 8);
    }
    if (!pe->batch_status)
        HIPCHK(hipHostMalloc((void**)&pe->batch_status, 256, hipHostMallocDefault));
    pe->batch_status[0] = pe->batch_status[1] = pe->batch_status[2] = 0;
    char* ws = static_cast<char*>(pe->dev);
    if (staged) {
        vo = reinterpret_cast<const int64_t*>(ws + offs_off);
        eo = reinterpret_cast<const int64_t*>(ws + offs_off + off_bytes);
    }
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws);
    GraphDesc* descs = reinterpret_cast<GraphDesc*>(ws + desc_off);
    int32_t* rows = reinterpret_cast<int32_t*>(ws + rows_off);
    auto enqueue = [&]() -> int32_t {
        if (staged)
            HIPCHK(hipMemcpyAsync(ws + offs_off, pe->host_stage, 2 * off_bytes,
                                  hipMemcpyHostToDevice, s));
        HIPCHK(launch_batch_prep(vo, eo, B, u, v, out, max_n, seg_cap, descs, rows, ctrl,
                                 pe->batch_status, s));
        HIPCHK(launch_batch_lds(descs, B, max_n, &ctrl->queue_head, pe->batch_status, lds_halve,
                                device_cu_count(), s, lds_block));
        return CC_OK;
    };
    if (opts && opts->graph == 1 && s != nullptr) {
        KeyHash k;
        // staged offsets: the captured copy re-reads the staging buffer,
        // rewritten above, at every replay
        k.add(uint64_t(0xba7c4de71ce)).add(B).add(vo).add(eo).add(u).add(v).add(out).add(max_n)
            .add(seg_cap).add(lds_halve).add(lds_block).add(ws).add(s).add(staged)
            .add(pe->host_stage);
        rc = run_graph(pe, k.h, s, enqueue);
    } else {
        rc = enqueue();
    }
    if (rc != CC_OK) return rc;
    if (st) st->hook_launches += 1;
    HIPCHK(hipStreamSynchronize(s));
    if (st) st->host_syncs += 1;
    const int32_t prep = *(volatile int32_t*)(pe->batch_status + 1) |
                         *(volatile int32_t*)(pe->batch_status + 2);
    const int32_t solve = *(volatile int32_t*)pe->batch_status;
    if (prep & kStatusBadGraph)
        return fail(CC_ERR_ARG, "batch offsets must start at 0, be non-decreasing and give "
                                "every graph at most max_n vertices");
    if ((prep | solve) & kStatusRange) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n_g)");
    return CC_OK;
}

int32_t batch_device_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int32_t* u,
                          const int32_t* v, int32_t* out, int32_t max_n, const cc_options* opts,
                          hipStream_t s, cc_stats* st) {
    return batch_lds_impl(B, vo, eo, nullptr, nullptr, u, v, out, max_n, opts, s, st);
}

// ---------------------------------------------------------------------- probes, release
int32_t probe_impl(int32_t mode, const int32_t* u, const int32_t* v, int64_t m, const void* table,
                   int32_t n, hipStream_t s) {
    if (m < 0 || mode < 0 || mode > 11) return fail(CC_ERR_ARG, "bad probe arguments");
    if (mode >= 7) {  // memory-model probe: table is int32[128], edges unused
        if (!table || n < 128) return fail(CC_ERR_ARG, "memory-model probe needs a 128-word table");
        HIPCHK(launch_probe_mm(mode, static_cast<int32_t*>(const_cast<void*>(table)), s));
        return CC_OK;
    }
    if (m > 0 && (!u || !v)) return fail(CC_ERR_ARG, "null edge array");
    if (mode > 0 && (!table || n <= 0)) return fail(CC_ERR_ARG, "probe table required");
    if (((uintptr_t)u & 15) || ((uintptr_t)v & 15))
        return fail(CC_ERR_ARG, "probe edge arrays must be 16-byte aligned");
    PoolEntry* pe = pool_entry(s);
    std::lock_guard<std::mutex> lk(pe->mu);
    int32_t rc = ensure_dev(pe, 256);
    if (rc != CC_OK) return rc;
    uint32_t* sink = static_cast<uint32_t*>(pe->dev);
    if (mode == 0)
        HIPCHK(launch_probe_stream(u, v, m, sink, s));
    else if (mode == 1)
        HIPCHK(launch_probe_gather(u, v, m, static_cast<const int32_t*>(table), n, sink, s));
    else if (mode >= 5)
        HIPCHK(launch_probe_cas(u, v, m, static_cast<int32_t*>(const_cast<void*>(table)), n,
                                mode == 6, sink, s));
    else
        HIPCHK(launch_probe_bitgather(u, v, m, static_cast<const uint32_t*>(table), n, mode - 2,
                                      sink, s));
    return CC_OK;
}

void release_impl() {
    std::lock_guard<std::mutex> g(g_pool_mu);
    for (auto& kv : g_pool) {
        PoolEntry* e = kv.second.get();
        std::lock_guard<std::mutex> lk(e->mu);
        drain_async(e);
        drop_graphs(e);
        if (e->async_done) (void)hipEventDestroy(e->async_done);
        if (e->async_slot) (void)hipHostFree(e->async_slot);
        e->async_done = nullptr;
        e->async_slot = nullptr;
        e->async_called = false;
        for (int i = 0; i < 2; ++i) {
            if (e->copied[i]) (void)hipEventDestroy(e->copied[i]);
            if (e->consumed[i]) (void)hipEventDestroy(e->consumed[i]);
            e->copied[i] = e->consumed[i] = nullptr;
        }
        if (e->copy_stream) (void)hipStreamDestroy(e->copy_stream);
        e->copy_stream = nullptr;
        if (e->dev) (void)hipFree(e->dev);
        if (e->host_ctrl) (void)hipHostFree(e->host_ctrl);
        if (e->host_stage) (void)hipHostFree(e->host_stage);
        if (e->batch_status) (void)hipHostFree(e->batch_status);
        e->batch_status = nullptr;
        e->dev = nullptr;
        e->host_ctrl = nullptr;
        e->host_stage = nullptr;
        e->bytes = e->stage_bytes = 0;
        e->host_ctrl_count = 0;
    }
    g_pool.clear();
}

int32_t stream_status_impl(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    PoolEntry* e = nullptr;
    {
        std::lock_guard<std::mutex> g(g_pool_mu);
        auto it = g_pool.find({dev, s});
        if (it != g_pool.end()) e = it->second.get();
    }
    if (!e) return fail(CC_ERR_ARG, "no no-sync call on this stream and device");
    std::lock_guard<std::mutex> lk(e->mu);
    if (!e->async_called) return fail(CC_ERR_ARG, "no no-sync call on this stream and device");
    const hipError_t q = hipEventQuery(e->async_done);
    if (q == hipErrorNotReady) return CC_PENDING;
    if (q != hipSuccess) return fail(CC_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    const int32_t status = *reinterpret_cast<volatile int32_t*>(e->async_slot);
    if (status & kStatusRange) return fail(CC_ERR_RANGE, "edge endpoint outside [0, n)");
    if (status & kStatusOverflow) return fail(CC_ERR_NOMEM, "frontier capacity exceeded");
    return CC_OK;
}

}  // namespace hookcc
