// Continuous-batching request server for connected-components queries.
//
// Admission by HBM footprint.  Every request is charged 8m bytes of edges,
// 4n bytes of labels and the device workspace its solve takes (a request
// above CC_BATCH_LDS_MAX_N vertices: its own Atomic-Hook workspace, sized by
// the graph-list solver; small requests: nothing beyond a fixed block per
// worker, set aside at creation) against a budget of `device_bytes`, whether
// its arrays live in host or device memory.  A request is admitted, in
// arrival order, only while the charges of all admitted requests fit the
// budget; the bytes the server itself puts on the device (copies of host
// edges and labels, workspaces) are carved from an arena of that size.
// Each of `workers` host threads owns one HIP stream; whenever a worker is
// free it forms a wave from the head of the queue: either the longest run of
// small requests that fits (up to max_batch requests / max_batch_edges
// entries), solved together by one persistent LDS launch, or a single large
// request, solved in device memory.  A large request never joins a wave of
// small ones, so small requests do not wait for it, and large requests run
// concurrently on different workers' streams.  The worker waits (on the
// device) for the point the submitter marked on its stream, copies host
// inputs to the device, solves the wave with one graph-list call into the
// arena's workspace, copies labels back, and releases the request's charge.
// Requests that arrive while other waves are on the GPU join the next free
// worker's wave, so waves overlap on the device.  Every request records
// submit, admit, launch, device-done and host-done times on one steady clock.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "engine.hpp"

namespace hookcc {
namespace {

double now_s() {
    using namespace std::chrono;
    static const steady_clock::time_point t0 = steady_clock::now();
    return duration<double>(steady_clock::now() - t0).count();
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct Request {
    int64_t id = 0;
    int32_t n = 0;
    int64_t m = 0;
    const int32_t* u = nullptr;
    const int32_t* v = nullptr;
    int32_t* out = nullptr;
    int32_t flags = 0;
    size_t charge = 0;     // footprint charged against the budget: 8m + 4n + workspace
    size_t ws_bytes = 0;   // device workspace of a large request's solve (0: small)
    size_t off = 0, bytes = 0;  // its arena block: host copies, then the workspace
    int32_t* du = nullptr;
    int32_t* dv = nullptr;
    int32_t* dout = nullptr;
    char* ws = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream (device arrays)
    cc_request_info info{};
    bool done = false;
};

}  // namespace
}  // namespace hookcc

struct cc_server {
    int device = 0;
    cc_server_config cfg{};
    char* arena_base = nullptr;
    size_t arena_size = 0;
    hookcc::Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<hookcc::Request*> pending;
    std::unordered_map<int64_t, std::unique_ptr<hookcc::Request>> reqs;
    std::vector<std::thread> workers;
    bool stop = false;
    size_t budget = 0;        // device_bytes
    size_t budget_used = 0;   // charges of admitted, unfinished requests + worker blocks
    size_t small_ws = 0;      // per-worker workspace block for waves of small requests
    std::vector<size_t> worker_ws_off;
    int32_t alive = 0;  // workers that started and have not exited
    int64_t next_id = 1;
    int32_t worker_error = CC_OK;
    std::string worker_msg;
};

namespace hookcc {
namespace {

size_t edge_bytes(const Request& r) { return 2 * a256((size_t)r.m * 4); }
size_t label_bytes(const Request& r) { return a256((size_t)r.n * 4); }

// Bytes of the request's arena block: the device copies of host arrays, then
// the workspace of a large request's solve.
size_t block_bytes(const Request& r) {
    size_t b = r.ws_bytes;
    if (r.flags & CC_REQ_HOST_EDGES) b += edge_bytes(r);
    if (r.flags & CC_REQ_HOST_LABELS) b += label_bytes(r);
    return b;
}

void place(cc_server* S, Request* r) {
    char* p = S->arena_base + r->off;
    if (r->flags & CC_REQ_HOST_EDGES) {
        r->du = reinterpret_cast<int32_t*>(p);
        p += a256((size_t)r->m * 4);
        r->dv = reinterpret_cast<int32_t*>(p);
        p += a256((size_t)r->m * 4);
    } else {
        r->du = const_cast<int32_t*>(r->u);
        r->dv = const_cast<int32_t*>(r->v);
    }
    if (r->flags & CC_REQ_HOST_LABELS) {
        r->dout = reinterpret_cast<int32_t*>(p);
        p += label_bytes(*r);
    } else {
        r->dout = r->out;
    }
    r->ws = r->ws_bytes ? p : nullptr;
}

int32_t run_wave(std::vector<Request*>& wave, hipStream_t s, char* small_ws, size_t small_bytes) {
    for (Request* r : wave) {
        if (r->ready) {
            hipError_t e = hipStreamWaitEvent(s, r->ready, 0);
            if (e != hipSuccess) return fail(CC_ERR_HIP, std::string("request ready wait: ") + hipGetErrorString(e));
        }
    }
    for (Request* r : wave) {
        if ((r->flags & CC_REQ_HOST_EDGES) && r->m > 0) {
            hipError_t e = hipMemcpyAsync(r->du, r->u, (size_t)r->m * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(r->dv, r->v, (size_t)r->m * 4, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return fail(CC_ERR_HIP, std::string("request upload: ") + hipGetErrorString(e));
        }
    }
    std::vector<cc_graph> list(wave.size());
    for (size_t i = 0; i < wave.size(); ++i) {
        Request* r = wave[i];
        list[i].edges_u = r->m ? r->du : nullptr;
        list[i].edges_v = r->m ? r->dv : nullptr;
        list[i].out_label = r->n ? r->dout : nullptr;
        list[i].m = r->m;
        list[i].n = r->n;
        list[i].reserved = 0;
    }
    // a large request is a wave of its own and brings its workspace; small
    // ones use the worker's block
    char* ws = wave.size() == 1 && wave[0]->ws ? wave[0]->ws : small_ws;
    const size_t wsb = wave.size() == 1 && wave[0]->ws ? wave[0]->ws_bytes : small_bytes;
    int32_t rc = list_impl((int32_t)list.size(), list.data(), nullptr, s, nullptr, ws, wsb);
    const double t = now_s();
    for (Request* r : wave) r->info.t_device_done = t;
    if (rc == CC_ERR_RANGE && wave.size() > 1) {
        // attribute the error: solve each request of the wave on its own
        for (size_t i = 0; i < wave.size(); ++i) {
            int32_t ri = list_impl(1, &list[i], nullptr, s, nullptr, ws, wsb);
            wave[i]->info.status = ri;
        }
        rc = CC_OK;
    } else {
        for (Request* r : wave) r->info.status = rc;
    }
    for (Request* r : wave) {
        if ((r->flags & CC_REQ_HOST_LABELS) && r->n > 0 && r->info.status == CC_OK) {
            hipError_t e = hipMemcpyAsync(r->out, r->dout, (size_t)r->n * 4, hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return fail(CC_ERR_HIP, std::string("label download: ") + hipGetErrorString(e));
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CC_ERR_HIP, std::string("wave sync: ") + hipGetErrorString(e));
    const double th = now_s();
    for (Request* r : wave) r->info.t_host_done = th;
    return rc;
}

void worker_main(cc_server* S, int32_t index) {
    hipStream_t s = nullptr;
    if (hipSetDevice(S->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        std::lock_guard<std::mutex> g(S->mu);
        S->worker_error = CC_ERR_HIP;
        S->worker_msg = "worker could not create its stream";
        S->alive -= 1;
        S->cv_done.notify_all();
        return;
    }
    char* small_ws = S->arena_base + S->worker_ws_off[index];
    std::vector<Request*> wave;
    while (true) {
        wave.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            while (true) {
                if (S->stop && S->pending.empty()) break;
                int64_t edges = 0;
                while (!S->pending.empty() && (int32_t)wave.size() < S->cfg.max_batch) {
                    Request* r = S->pending.front();
                    const bool large = r->n > CC_BATCH_LDS_MAX_N;
                    if (!wave.empty() && (large || edges + r->m > S->cfg.max_batch_edges)) break;
                    if (r->charge > S->budget - S->small_ws * S->cfg.workers) {
                        // can never fit, even with nothing else admitted
                        r->info.status = CC_ERR_NOMEM;
                        r->done = true;
                        S->pending.pop_front();
                        S->cv_done.notify_all();
                        continue;
                    }
                    if (S->budget_used + r->charge > S->budget) break;  // wait for releases
                    size_t off = 0;
                    r->bytes = block_bytes(*r);
                    if (!S->arena.alloc(r->bytes, &off)) break;
                    S->budget_used += r->charge;
                    r->off = off;
                    place(S, r);
                    r->info.t_admit = now_s();
                    wave.push_back(r);
                    edges += r->m;
                    S->pending.pop_front();
                    if (large) break;  // a large request is a wave of its own
                }
                if (!wave.empty()) break;
                S->cv_work.wait(lk);
            }
            if (wave.empty()) break;
        }
        const double tl = now_s();
        for (Request* r : wave) {
            r->info.t_launch = tl;
            r->info.batch_size = (int32_t)wave.size();
        }
        int32_t rc = run_wave(wave, s, small_ws, S->small_ws);
        {
            std::lock_guard<std::mutex> g(S->mu);
            for (Request* r : wave) {
                if (rc != CC_OK) r->info.status = rc;
                S->arena.release(r->off, r->bytes);
                S->budget_used -= r->charge;
                if (r->ready) {
                    (void)hipEventDestroy(r->ready);
                    r->ready = nullptr;
                }
                r->done = true;
            }
            if (rc != CC_OK && rc != CC_ERR_RANGE) {
                S->worker_error = rc;
                S->worker_msg = last_error();
            }
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
    (void)hipStreamDestroy(s);
    std::lock_guard<std::mutex> g(S->mu);
    S->alive -= 1;
    S->cv_done.notify_all();
}

}  // namespace
}  // namespace hookcc

using namespace hookcc;

extern "C" {

double cc_server_clock(void) { return now_s(); }

int32_t cc_server_create(const cc_server_config* cfg, cc_server** out) {
    if (!out) return fail(CC_ERR_ARG, "null server output");
    *out = nullptr;
    cc_server_config c;
    std::memset(&c, 0, sizeof c);
    if (cfg) c = *cfg;
    for (int i = 0; i < 8; ++i)
        if (c.reserved[i]) return fail(CC_ERR_ARG, "cc_server_config.reserved must be zero");
    if (c.device_bytes < 0 || c.workers < 0 || c.max_batch < 0 || c.max_batch_edges < 0)
        return fail(CC_ERR_ARG, "negative server setting");
    if (c.workers == 0) c.workers = 2;
    if (c.workers > 16) return fail(CC_ERR_ARG, "at most 16 workers");
    if (c.max_batch == 0) c.max_batch = 1024;
    if (c.max_batch_edges == 0) c.max_batch_edges = int64_t(1) << 28;
    std::unique_ptr<cc_server> S(new cc_server());
    if (hipGetDevice(&S->device) != hipSuccess) return fail(CC_ERR_HIP, "no current HIP device");
    if (c.device_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return fail(CC_ERR_HIP, "hipMemGetInfo failed");
        c.device_bytes = (int64_t)(fr / 4);
    }
    S->cfg = c;
    S->arena_size = a256((size_t)c.device_bytes);
    S->budget = S->arena_size;
    // each worker's workspace for a wave of up to max_batch small graphs
    {
        std::vector<cc_graph> probe((size_t)c.max_batch);
        static int32_t dummy;
        for (auto& G : probe) {
            std::memset(&G, 0, sizeof G);
            G.n = 1;
            G.out_label = &dummy;
        }
        int32_t rc = list_impl(c.max_batch, probe.data(), nullptr, nullptr, nullptr, nullptr, 0,
                               &S->small_ws);
        if (rc != CC_OK) return rc;
    }
    if (S->small_ws * (size_t)c.workers > S->arena_size)
        return fail(CC_ERR_NOMEM, "server: device_bytes below the workers' fixed workspace (" +
                                      std::to_string(S->small_ws * (size_t)c.workers) + " bytes)");
    if (S->arena_size) {
        hipError_t e = hipMalloc((void**)&S->arena_base, S->arena_size);
        if (e != hipSuccess) return fail(CC_ERR_NOMEM, std::string("server arena: ") + hipGetErrorString(e));
    }
    S->arena.reset(S->arena_size);
    for (int i = 0; i < c.workers; ++i) {
        size_t off = 0;
        if (!S->arena.alloc(S->small_ws, &off)) {
            (void)hipFree(S->arena_base);
            return fail(CC_ERR_NOMEM, "server: arena too small for the workers' workspace");
        }
        S->worker_ws_off.push_back(off);
        S->budget_used += S->small_ws;
    }
    cc_server* raw = S.release();
    raw->alive = c.workers;
    for (int i = 0; i < c.workers; ++i) raw->workers.emplace_back(worker_main, raw, i);
    *out = raw;
    return CC_OK;
}

int32_t cc_server_submit_on(cc_server* S, int32_t n, const int32_t* edges_u,
                            const int32_t* edges_v, int64_t m, int32_t* out_label, int32_t flags,
                            void* ready_stream, int64_t* ticket) {
    if (!S || !ticket) return fail(CC_ERR_ARG, "null server or ticket");
    if (n < 0 || m < 0) return fail(CC_ERR_ARG, "n < 0 or m < 0");
    if (m > 0 && (!edges_u || !edges_v)) return fail(CC_ERR_ARG, "null edge array");
    if (n > 0 && !out_label) return fail(CC_ERR_ARG, "null out_label");
    if (flags & ~(CC_REQ_HOST_EDGES | CC_REQ_HOST_LABELS)) return fail(CC_ERR_ARG, "unknown flags");
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->m = m;
    r->u = edges_u;
    r->v = edges_v;
    r->out = out_label;
    r->flags = flags;
    if (n > CC_BATCH_LDS_MAX_N) {
        // the workspace the graph-list solver takes for this graph alone
        cc_graph G;
        std::memset(&G, 0, sizeof G);
        G.edges_u = edges_u;
        G.edges_v = edges_v;
        G.out_label = out_label;
        G.m = m;
        G.n = n;
        int32_t rc = list_impl(1, &G, nullptr, nullptr, nullptr, nullptr, 0, &r->ws_bytes);
        if (rc != CC_OK) return rc;
    }
    r->charge = edge_bytes(*r) + label_bytes(*r) + r->ws_bytes;
    const bool device_arrays = (m > 0 && !(flags & CC_REQ_HOST_EDGES)) ||
                               (n > 0 && !(flags & CC_REQ_HOST_LABELS));
    if (device_arrays) {
        // the worker's stream waits for the work queued on the submitter's
        // stream so far (the producers of the edges, earlier users of out's memory)
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return fail(CC_ERR_HIP, "no current HIP device");
        if (prev != S->device && hipSetDevice(S->device) != hipSuccess)
            return fail(CC_ERR_HIP, "cannot select the server's device");
        hipError_t e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r->ready, static_cast<hipStream_t>(ready_stream));
        if (prev != S->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (r->ready) (void)hipEventDestroy(r->ready);
            return fail(CC_ERR_HIP, std::string("request ready event: ") + hipGetErrorString(e));
        }
    }
    r->info.status = 1;  // pending
    r->info.t_submit = now_s();
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
        if (r->ready) (void)hipEventDestroy(r->ready);
        return fail(CC_ERR_ARG, "server is shutting down");
    }
    r->id = S->next_id++;
    *ticket = r->id;
    S->pending.push_back(r.get());
    S->reqs[r->id] = std::move(r);
    S->cv_work.notify_one();
    return CC_OK;
}

int32_t cc_server_submit(cc_server* S, int32_t n, const int32_t* edges_u, const int32_t* edges_v,
                         int64_t m, int32_t* out_label, int32_t flags, int64_t* ticket) {
    return cc_server_submit_on(S, n, edges_u, edges_v, m, out_label, flags, nullptr, ticket);
}

static int32_t finish_ticket(cc_server* S, int64_t ticket, cc_request_info* info, bool block) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(CC_ERR_ARG, "unknown ticket");
    Request* r = it->second.get();
    if (!r->done && !block) return 1;
    while (!r->done) {
        if (S->alive <= 0) {
            r->info.status = CC_ERR_HIP;  // no worker left to serve it
            break;
        }
        S->cv_done.wait(lk);
    }
    if (info) *info = r->info;
    const int32_t st = r->info.status;
    S->reqs.erase(it);
    if (st != CC_OK) return fail(st, "request failed");
    return CC_OK;
}

int32_t cc_server_wait(cc_server* S, int64_t ticket, cc_request_info* info) {
    if (!S) return fail(CC_ERR_ARG, "null server");
    return finish_ticket(S, ticket, info, true);
}

int32_t cc_server_poll(cc_server* S, int64_t ticket, cc_request_info* info) {
    if (!S) return fail(CC_ERR_ARG, "null server");
    return finish_ticket(S, ticket, info, false);
}

int32_t cc_server_stats(cc_server* S, int64_t* pending, int64_t* arena_used) {
    if (!S) return fail(CC_ERR_ARG, "null server");
    std::lock_guard<std::mutex> g(S->mu);
    if (pending) *pending = (int64_t)S->pending.size();
    if (arena_used) *arena_used = (int64_t)S->budget_used;
    return CC_OK;
}

int32_t cc_server_destroy(cc_server* S) {
    if (!S) return CC_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    const int32_t rc = S->worker_error;
    const std::string msg = S->worker_msg;
    if (S->arena_base) (void)hipFree(S->arena_base);
    delete S;
    if (rc != CC_OK) return fail(rc, msg);
    return CC_OK;
}

}  // extern "C"
