// Batched solve of many small graphs in one persistent launch (CDNA4).
//
// Persistent workgroups (1024 threads, 16 waves, by default; as many per CU as
// the LDS of the launch's largest graph allows) take graphs from a device
// work queue (an atomic counter over descriptors ordered largest first, by
// the host or, for offsets in device memory, by the preparation launches
// below) and solve each one entirely in LDS: the graph's tree array pi lives in LDS as
// local ids, 32-bit for n <= 32768 and 16-bit up to 65536 (at most 128 KiB of
// the 160 KiB LDS), the edge entries are streamed once from HBM, and the
// labels are written once.
// Per graph the schedule is the paper's adaptive one (Fig. 4): for each of
// the graph's s edge segments, Atomic-Hook the segment, then Multi-Jump all
// its vertices, with a workgroup barrier between phases.
#include "kernels.hpp"

namespace hookcc {

constexpr int kBatchEPT = 8;  // edge entries per thread per step
// Fourth word of a raw buffer resource on gfx9-family GPUs (32-bit data
// format, no swizzle) and the non-temporal cache policy of a buffer load.
constexpr int32_t kBufferRsrcWord3 = 0x00020000;
constexpr int32_t kBufferNonTemporal = 2;

// 16-bit compare-and-swap in LDS, built on the 32-bit CAS of the containing
// word: succeeds iff slot `idx` holds `expected`; returns the value found.
// The other half-word may change concurrently; the loop then retries with
// the fresh word, so only a change of this half-word can make it fail.
__device__ __forceinline__ uint32_t lds_cas16(uint16_t* spi, uint32_t idx, uint32_t expected,
                                              uint32_t desired) {
    uint32_t* w = reinterpret_cast<uint32_t*>(spi) + (idx >> 1);
    const uint32_t sh = (idx & 1) * 16;
    uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    while (true) {
        const uint32_t cur = (old >> sh) & 0xffffu;
        if (cur != expected) return cur;
        const uint32_t nw = (old & ~(0xffffu << sh)) | (desired << sh);
        const uint32_t prev = atomicCAS(w, old, nw);
        if (prev == old) return expected;
        old = prev;
    }
}

// The graph's arrays come from a descriptor in memory, so the compiler cannot
// tell their address space; they are global memory, and saying so gives
// global (not flat) loads and stores.
typedef __attribute__((address_space(1))) const int32_t g_cint;
typedef __attribute__((address_space(1))) int32_t g_int;

// Slots of the tree array in LDS.  Graphs of at most kWideMaxN vertices keep
// 32-bit slots (4n bytes <= 128 KiB) and hook with the native 32-bit LDS
// compare-and-swap; larger ones keep 16-bit slots (2n bytes) and hook with
// lds_cas16 on the containing word.
constexpr uint32_t kWideMaxN = 32768;

// Relaxed workgroup-scope atomics, not volatile accesses: the compiler keeps
// every access (other threads change pi concurrently) and still sees that
// the pointer is in LDS, so these are ds_read / ds_write -- a volatile access
// through the pointer became a flat access, which also waits on the
// outstanding global loads of the software pipeline.
template <typename T>
__device__ __forceinline__ uint32_t lds_ld(T* spi, uint32_t idx) {
    return __hip_atomic_load(spi + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void lds_st(T* spi, uint32_t idx, uint32_t x) {
    __hip_atomic_store(spi + idx, (T)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Compare-and-swap of slot idx from `expected` to `desired`; returns the value
// found (== expected on success).
__device__ __forceinline__ uint32_t lds_cas(uint32_t* spi, uint32_t idx, uint32_t expected,
                                            uint32_t desired) {
    __hip_atomic_compare_exchange_strong(spi + idx, &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return expected;
}
__device__ __forceinline__ uint32_t lds_cas(uint16_t* spi, uint32_t idx, uint32_t expected,
                                            uint32_t desired) {
    return lds_cas16(spi, idx, expected, desired);
}

// Atomic-Hook in LDS (Fig. 3, top), same steps as the device-memory kernel;
// with `halve`, a passed non-root H whose grandparent differs from its
// parent is re-pointed at the grandparent (path halving).  The re-point of a
// non-root never meets a successful CAS on its own slot (that needs a root),
// and with 16-bit slots it cannot be lost to, nor undo, a concurrent CAS on
// the other half of its 32-bit word: that CAS compares the whole word, so it
// fails and retries if the store landed between its read and its swap.  In
// LDS the store costs one write, and the shallower trees let a graph run
// with fewer segments (fewer Multi-Jump passes over its vertices).
template <typename T>
__device__ __forceinline__ void lds_atomic_hook(T* spi, uint32_t pu, uint32_t pv, bool halve) {
    // One exit, at the loop's head, and no branch inside (halve is uniform):
    // after a successful CAS both ends are set to L, which ends the loop; the
    // two loads and the store of that last pass are wasted but cheaper than
    // the exec-mask bookkeeping of a second exit.
    while (pu != pv) {
        const uint32_t H = pu > pv ? pu : pv;
        const uint32_t L = pu > pv ? pv : pu;
        const uint32_t found = lds_cas(spi, H, H, L);
        const uint32_t gu = lds_ld(spi, found);
        const uint32_t gv = lds_ld(spi, L);
        // H is no root now (it was none or the CAS made it a child of L), so
        // no CAS can succeed on its slot and every value stored there is one
        // of its ancestors: gu (found's parent, found itself, or L after a
        // successful CAS) is one, whichever halving store lands last.
        if (halve) lds_st(spi, H, gu);
        const bool hooked = found == H;
        pu = hooked ? L : gu;
        pv = hooked ? L : gv;
    }
}

// Entries [base, base + step) of the edge arrays, clipped at `end`: lane
// tid loads entries base + tid + j * blockDim.x into a[j], b[j] (0 past
// `end`).  Each array is read through a raw buffer resource whose size is
// the step's entries inside [base, end), so no load is issued past `end`;
// the byte offsets are per lane and the same at every step.
template <int EPT = kBatchEPT>
__device__ __forceinline__ void edge_step_loads(g_cint* du, g_cint* dv, int64_t base, int64_t end,
                                                int64_t step, int32_t* a, int32_t* b) {
    const int64_t rem = end - base < step ? end - base : step;
    const int32_t bytes = rem > 0 ? (int32_t)(rem * 4) : 0;
    const __amdgpu_buffer_rsrc_t ru =
        __builtin_amdgcn_make_buffer_rsrc((void*)(du + base), 0, bytes, kBufferRsrcWord3);
    const __amdgpu_buffer_rsrc_t rv =
        __builtin_amdgcn_make_buffer_rsrc((void*)(dv + base), 0, bytes, kBufferRsrcWord3);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int32_t off = (int32_t)((threadIdx.x + j * blockDim.x) * 4);
        a[j] = __builtin_amdgcn_raw_buffer_load_b32(ru, off, 0, kBufferNonTemporal);
        b[j] = __builtin_amdgcn_raw_buffer_load_b32(rv, off, 0, kBufferNonTemporal);
    }
}

// One graph by the whole workgroup (called by every thread): init, then per
// segment Atomic-Hook of its entries and Multi-Jump of its vertices; the last
// Multi-Jump writes the labels instead of storing the roots in LDS.  Sets
// `bad` on an endpoint outside [0, n).  Returns without a final barrier: the
// caller's next barrier separates the label reads from the next graph's init.
template <typename T>
__device__ __forceinline__ void solve_graph(T* spi, const GraphDesc& d, bool halve, bool& bad) {
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = blockDim.x;
    const uint32_t n = (uint32_t)d.n;
    g_cint* du = (g_cint*)d.u;
    g_cint* dv = (g_cint*)d.v;
    g_int* dout = (g_int*)d.out;
    const int32_t s = d.segments > 0 ? d.segments : 1;
    const int64_t step = (int64_t)nthr * kBatchEPT;
    int32_t a[kBatchEPT], b[kBatchEPT], na[kBatchEPT], nb[kBatchEPT];
    // the first segment's first loads go out before the init, so that their
    // latency overlaps it and its barrier
    edge_step_loads(du, dv, 0, d.m / s, step, a, b);
    for (uint32_t x = tid; x < n; x += nthr) lds_st(spi, x, x);
    __syncthreads();
    for (int32_t seg = 0; seg < s; ++seg) {
        const int64_t b0 = d.m * seg / s, b1 = d.m * (seg + 1) / s;
        // kBatchEPT entries per thread per step, all loads issued before
        // any hook, and the next step's loads issued before this step's
        // hooks (software pipelining), so the edge stream's latency
        // overlaps the LDS work.  The loads go through buffer resources
        // that cover exactly the step's entries: the per-lane byte offsets
        // are the same at every step, and a load past the segment's end
        // returns 0 without touching memory.  No branch surrounds a load or
        // a hook: such an entry, and one out of range, becomes the pair
        // (0, 0), whose hook does nothing -- divergent branches would cost
        // more scalar exec-mask instructions than the work they skip.
        if (b1 > b0) {
            int64_t base = b0;
            if (seg > 0) edge_step_loads(du, dv, base, b1, step, a, b);
            for (; base < b1; base += step) {
                edge_step_loads(du, dv, base + step, b1, step, na, nb);
#pragma unroll
                for (int j = 0; j < kBatchEPT; ++j) {
                    const bool ok = max((uint32_t)a[j], (uint32_t)b[j]) < n;
                    bad |= !ok;
                    const uint32_t x = ok ? (uint32_t)a[j] : 0u;
                    const uint32_t y = ok ? (uint32_t)b[j] : 0u;
                    lds_atomic_hook(spi, lds_ld(spi, x), lds_ld(spi, y), halve);
                }
#pragma unroll
                for (int j = 0; j < kBatchEPT; ++j) {
                    a[j] = na[j];
                    b[j] = nb[j];
                }
            }
        }
        __syncthreads();
        // Multi-Jump (Fig. 3, bottom) over the graph's vertices, low ids first.
        // Each vertex climbs to its root and stores it once (a root stores
        // itself); no hook runs in this phase, so only the stores of other
        // climbers race with it, and each stores an ancestor.  After the last
        // segment the root is the label: it goes to global memory only.
        // Two vertices per thread and pass, their climbs interleaved (a
        // finished climb stays on its root, whose parent is itself).
        const bool last = seg + 1 == s;
        for (uint32_t x = tid; x < n; x += 2 * nthr) {
            const uint32_t y = x + nthr;
            const bool has_y = y < n;
            uint32_t p1 = lds_ld(spi, x), p2 = lds_ld(spi, has_y ? y : x);
            uint32_t g1 = lds_ld(spi, p1), g2 = lds_ld(spi, p2);
            while (g1 != p1 || g2 != p2) {
                p1 = g1;
                p2 = g2;
                g1 = lds_ld(spi, p1);
                g2 = lds_ld(spi, p2);
            }
            if (last) {
                dout[x] = (int32_t)p1;
                if (has_y) dout[y] = (int32_t)p2;
            } else {
                lds_st(spi, x, p1);
                if (has_y) lds_st(spi, y, p2);
            }
        }
        if (!last) __syncthreads();
    }
}

template <bool HALVE>
__global__ __launch_bounds__(1024) void k_batch_lds(const GraphDesc* __restrict__ descs,
                                                    int32_t count, int32_t* queue_head,
                                                    int32_t* status) {
    constexpr bool halve = HALVE;  // a compile-time constant: no branch in the hook loop
    extern __shared__ uint16_t spi[];
    __shared__ int32_t next;
    bool bad = false;
    if (threadIdx.x == 0) next = atomicAdd(queue_head, 1);
    __syncthreads();
    int32_t idx = next;
    while (idx < count) {
        const GraphDesc d = descs[idx];
        // The next position is fetched while this graph is solved, so the
        // queue's latency is paid once per workgroup, not once per graph.
        // Thread 0 writes `next` again only after the barriers inside
        // solve_graph, which every thread passes after reading it.
        int32_t pre = 0;
        if (threadIdx.x == 0) pre = atomicAdd(queue_head, 1);
        if ((uint32_t)d.n <= kWideMaxN)
            solve_graph(reinterpret_cast<uint32_t*>(spi), d, halve, bad);
        else
            solve_graph(spi, d, halve, bad);
        if (threadIdx.x == 0) next = pre;
        __syncthreads();
        idx = next;
    }
    // status may be host memory: a plain store (every writer stores the same
    // bit) visible to the host once the launch has completed
    if (bad) __hip_atomic_store(status, kStatusRange, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---------------------------------------------------------------------------
// Preparation of a batch whose offsets are in device memory, in two launches
// of one thread per graph: every graph is checked and given its size class
// of m + n (four classes per power of two, the order the host-offset call
// builds); the graphs are placed largest class first (a counting sort) and
// their descriptors written for k_batch_lds.  A graph whose offsets are
// invalid (not starting at 0, decreasing, more than max_n vertices) or that
// has entries but no vertex gets an empty descriptor (nothing is read or
// written for it); status[1] / status[2] (host memory) then receive
// kStatusBadGraph / kStatusRange.  ctrl->queue_head is cleared for the
// solve.

__device__ __forceinline__ int batch_size_class(uint64_t w) {
    w |= 1;
    const int lg = 63 - __clzll((long long)w);
    const int frac = lg >= 2 ? (int)((w >> (lg - 2)) & 3) : (int)((w << (2 - lg)) & 3);
    return lg * 4 + frac;
}

// min(cap, round(m / n)), at least 1 (cap 0: round(m / n) up to 2^20)
__device__ __forceinline__ int32_t batch_segments(int64_t m, int64_t n, int32_t cap) {
    if (cap > 0 && cap <= 16 && m < (int64_t(1) << 61)) {
        int32_t k = cap;
        while (k > 1 && 2 * m < (2 * (int64_t)k - 1) * n) --k;
        return k;
    }
    int64_t r = m / n + ((m % n) * 2 >= n ? 1 : 0);
    r = r < 1 ? 1 : (r > (int64_t(1) << 20) ? (int64_t(1) << 20) : r);
    return cap > 0 && r > cap ? cap : (int32_t)r;
}

constexpr int kPrepGraphs = 1024;  // graphs per preparation workgroup, one per thread

struct PrepGraph {
    int64_t v0, n, e0, m;
    int32_t cls;   // position class: 0 = largest
    int32_t flag;  // 0, kStatusBadGraph or kStatusRange
};

__device__ __forceinline__ PrepGraph prep_graph(const int64_t* vo, const int64_t* eo, int32_t g,
                                                int32_t max_n, bool edges, bool labels) {
    PrepGraph p;
    p.v0 = vo[g];
    p.e0 = eo[g];
    p.n = vo[g + 1] - p.v0;
    p.m = eo[g + 1] - p.e0;
    p.flag = 0;
    // (edges / labels: whether those arrays were given; a null one may only
    // belong to graphs that have no entries / no vertices)
    if ((g == 0 && (p.v0 != 0 || p.e0 != 0)) || p.n < 0 || p.m < 0 || p.n > max_n ||
        (p.m > 0 && !edges) || (p.n > 0 && !labels))
        p.flag = kStatusBadGraph;
    else if (p.n == 0 && p.m > 0)
        p.flag = kStatusRange;
    if (p.flag) p.n = p.m = 0;
    p.cls = 255 - batch_size_class((uint64_t)p.m + (uint64_t)p.n);
    return p;
}

// Step 1 (one thread per graph, kPrepGraphs per workgroup): each workgroup
// counts its graphs per class into its row of `rows` (W x 256).
__global__ __launch_bounds__(1024) void k_batch_prep_count(const int64_t* __restrict__ vo,
                                                           const int64_t* __restrict__ eo,
                                                           int32_t B, int32_t max_n, bool edges,
                                                           bool labels, int32_t* __restrict__ rows,
                                                           Ctrl* ctrl) {
    __shared__ int32_t hist[256];
    const int32_t tid = threadIdx.x;
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    const int32_t g = blockIdx.x * kPrepGraphs + tid;
    if (g < B) atomicAdd(&hist[prep_graph(vo, eo, g, max_n, edges, labels).cls], 1);
    __syncthreads();
    if (tid < 256) rows[blockIdx.x * 256 + tid] = hist[tid];
    if (blockIdx.x == 0 && tid == 0) ctrl->queue_head = 0;
}

// Up to this many preparation workgroups, each placing workgroup sums the
// rows of all of them itself (W x 256 loads each); above it a scan launch
// turns the rows into prefix sums first, so that the work stays linear in B.
constexpr int32_t kPrepLoopMaxW = 32;

// Step 1b (only when W > kPrepLoopMaxW; one workgroup per class c): column c
// of `rows` becomes the exclusive prefix sums over the workgroups (row w: the
// graphs of class c in workgroups before w), and totals[c] its sum.  Thread t
// takes a run of consecutive rows.
__global__ __launch_bounds__(1024) void k_batch_prep_scan(int32_t* __restrict__ rows, int32_t W,
                                                          int32_t* __restrict__ totals) {
    __shared__ int32_t wsum[16];
    const int32_t c = blockIdx.x, tid = threadIdx.x;
    const int32_t lane = tid & 63, wave = tid >> 6;
    const int32_t per = (W + 1023) / 1024;
    const int32_t w0 = min(W, tid * per), w1 = min(W, w0 + per);
    int32_t sum = 0;
    for (int32_t w = w0; w < w1; ++w) sum += rows[(int64_t)w * 256 + c];
    int32_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t at = incl - sum, all = 0;
    for (int32_t i = 0; i < 16; ++i) {
        at += i < wave ? wsum[i] : 0;
        all += wsum[i];
    }
    for (int32_t w = w0; w < w1; ++w) {
        const int32_t r = rows[(int64_t)w * 256 + c];
        rows[(int64_t)w * 256 + c] = at;
        at += r;
    }
    if (tid == 0) totals[c] = all;
}

// Step 2: each workgroup finds where its graphs of each class go (all
// earlier classes of every workgroup, then this class of the earlier
// workgroups) and writes their descriptors there.  `totals` null: `rows`
// holds the per-workgroup counts; else the scanned rows and the totals.
__global__ __launch_bounds__(1024) void k_batch_prep_place(
    const int64_t* __restrict__ vo, const int64_t* __restrict__ eo, int32_t B, const int32_t* u,
    const int32_t* v, int32_t* out, int32_t max_n, int32_t seg_cap,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ totals, int32_t W,
    GraphDesc* __restrict__ descs, int32_t* status) {
    __shared__ int32_t base[256];
    __shared__ int32_t flags;
    const int32_t tid = threadIdx.x;
    int32_t total = 0, before = 0;
    if (tid < 256 && totals) {
        total = totals[tid];
        before = rows[(int64_t)blockIdx.x * 256 + tid];
    } else if (tid < 256) {
        for (int32_t w = 0; w < W; ++w) {
            const int32_t r = rows[w * 256 + tid];
            total += r;
            before += w < (int32_t)blockIdx.x ? r : 0;
        }
    }
    if (tid == 0) flags = 0;
    __shared__ int32_t tot[256];
    if (tid < 256) tot[tid] = total;
    __syncthreads();
    if (tid < 64) {
        // exclusive scan of the 256 class totals: 4 per lane, then across the wave
        const int32_t c0 = tot[4 * tid], c1 = tot[4 * tid + 1], c2 = tot[4 * tid + 2],
                      c3 = tot[4 * tid + 3];
        const int32_t sum = c0 + c1 + c2 + c3;
        int32_t inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t t = __shfl_up(inc, d, 64);
            if (tid >= d) inc += t;
        }
        const int32_t ex = inc - sum;
        tot[4 * tid] = ex;
        tot[4 * tid + 1] = ex + c0;
        tot[4 * tid + 2] = ex + c0 + c1;
        tot[4 * tid + 3] = ex + c0 + c1 + c2;
    }
    __syncthreads();
    if (tid < 256) base[tid] = tot[tid] + before;
    __syncthreads();
    const int32_t g = blockIdx.x * kPrepGraphs + tid;
    if (g < B) {
        const PrepGraph p = prep_graph(vo, eo, g, max_n, u && v, out != nullptr);
        const int32_t pos = atomicAdd(&base[p.cls], 1);
        GraphDesc d;
        d.u = u + p.e0;
        d.v = v + p.e0;
        d.out = out + p.v0;
        d.m = p.m;
        d.n = (int32_t)p.n;
        d.segments = p.n > 0 ? batch_segments(p.m, p.n, seg_cap) : 1;
        descs[pos] = d;
        if (p.flag) atomicOr(&flags, p.flag);
    }
    __syncthreads();
    // one word per kind of fault, so that plain stores of different
    // workgroups never overwrite each other's bits
    if (tid == 0 && (flags & kStatusBadGraph))
        __hip_atomic_store(status + 1, kStatusBadGraph, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (tid == 0 && (flags & kStatusRange))
        __hip_atomic_store(status + 2, kStatusRange, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_batch_prep(const int64_t* vo, const int64_t* eo, int32_t B, const int32_t* u,
                             const int32_t* v, int32_t* out, int32_t max_n, int32_t seg_cap,
                             GraphDesc* descs, int32_t* rows, Ctrl* ctrl, int32_t* status,
                             hipStream_t s) {
    if (B <= 0) return hipSuccess;
    const int32_t W = (int32_t)(((int64_t)B + kPrepGraphs - 1) / kPrepGraphs);
    k_batch_prep_count<<<W, kPrepGraphs, 0, s>>>(vo, eo, B, max_n, u && v, out != nullptr, rows,
                                                 ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t* totals = nullptr;
    if (W > kPrepLoopMaxW) {
        totals = rows + (int64_t)W * 256;
        k_batch_prep_scan<<<256, 1024, 0, s>>>(rows, W, totals);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_batch_prep_place<<<W, kPrepGraphs, 0, s>>>(vo, eo, B, u, v, out, max_n, seg_cap, rows, totals,
                                                 W, descs, status);
    return hipGetLastError();
}

// Window round of the hybrid plan (an atomic-free Hook round, Fig. 2, with
// the Hook of each workgroup's chunk done in LDS; beyond the paper).
// Workgroup w takes entries [w * kWinEntries, (w + 1) * kWinEntries) and a
// window of kWinSlots consecutive vertices starting at the smallest endpoint
// among the chunk's first blockDim.x entries.  Entries with both endpoints in
// the window are joined completely in LDS (Atomic-Hook with path halving on
// 16-bit local ids, then a Multi-Jump over the window); every other entry
// gets the device-memory atomic-free Hook (plain store pi[max] = min of the
// endpoints' current parents).  Then each window vertex that is not its
// local root is pointed at it with a plain store.  The number of entries
// hooked outside the windows is added to ctrl->win_far.
//
// Every value written to pi names a vertex of the slot's own component below
// the slot (a local root, or the smaller of two parents joined by an entry),
// so pi stays a forest of subsets of components with pi[x] <= x.  Stores of
// different workgroups to one slot overwrite each other, which can split a
// chunk's local component into several trees; then some entry of that chunk
// joins two of them, and the compaction that follows the Multi-Jump keeps it
// for the Atomic-Hook pass.  No thread of this kernel takes a root by CAS in
// device memory, so its stores are of workgroup scope.  On inputs whose
// consecutive entries touch nearby ids (a row-major lattice) nearly every
// entry is joined in LDS and few survive the round; elsewhere the chunks'
// windows hold few entries and the round is the plain one.  The sizes: a
// chunk of a percolated 4096^2 lattice spans ~39,200 ids (within the
// window), two workgroups fit a CU (80 KiB of LDS each), so the lattice's
// 478 chunks run at once.
constexpr int64_t kWinEntries = 49152;  // 1024 threads x 48 entries
constexpr uint32_t kWinSlots = 40960;   // 16-bit local ids: 80 KiB of LDS
constexpr int kWinSegments = 2;
constexpr int kWinEPT = 4;  // entries per thread per step (registers: two workgroups per CU)

__global__ __launch_bounds__(1024) void k_hook_window(const int32_t* __restrict__ eu,
                                                      const int32_t* __restrict__ ev, int64_t m,
                                                      int32_t* pi, int32_t n, Ctrl* ctrl) {
    extern __shared__ uint16_t spi[];
    __shared__ int32_t wave_min[16];
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t lane = tid & 63, wave = tid >> 6, waves = nthr >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kWinEntries;
    const int64_t c1 = min(m, c0 + kWinEntries);
    const int64_t step = (int64_t)nthr * kWinEPT;
    g_cint* gu = (g_cint*)eu;
    g_cint* gv = (g_cint*)ev;
    int32_t a[kWinEPT], b[kWinEPT], na[kWinEPT], nb[kWinEPT];
    // the first segment's first entries are loaded before the LDS init, so
    // that their latency overlaps it; the window starts at the smallest
    // endpoint among the first blockDim.x of them
    const int64_t first_end = c0 + (c1 - c0) / kWinSegments;
    edge_step_loads<kWinEPT>(gu, gv, c0, first_end, step, a, b);
    uint32_t* w32 = reinterpret_cast<uint32_t*>(spi);
    for (uint32_t w = tid; w < kWinSlots / 2; w += nthr) w32[w] = ((2 * w + 1) << 16) | (2 * w);
    int32_t lo = INT32_MAX;
    if (c0 + tid < first_end) {
        if ((uint32_t)a[0] < (uint32_t)n) lo = min(lo, a[0]);
        if ((uint32_t)b[0] < (uint32_t)n) lo = min(lo, b[0]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) lo = min(lo, __shfl_xor(lo, d, 64));
    if (lane == 0) wave_min[wave] = lo;
    __syncthreads();
    int32_t base = wave_min[0];
    for (uint32_t i = 1; i < waves; ++i) base = min(base, wave_min[i]);
    if (base == INT32_MAX) base = 0;
    // window vertices: [base, base + span)
    const uint32_t span = (uint32_t)min<int64_t>((int64_t)kWinSlots, (int64_t)n - base);
    bool bad = false;
    uint32_t far = 0;  // entries hooked outside the window
    // The chunk in kWinSegments segments, each followed by a Multi-Jump over
    // the window (the schedule of Fig. 4 inside the chunk) so that later
    // climbs start from stars.  kWinEPT entries per thread per step,
    // consecutive threads on consecutive entries (coalesced, through buffer
    // resources as in the batched solver), the next step's loads issued
    // before this step's hooks.  An entry past the segment's end reads as
    // (0, 0); no branch surrounds the LDS hook, which is given (0, 0) -- a
    // no-op -- for every entry that is not inside the window.
    for (int seg = 0; seg < kWinSegments; ++seg) {
        const int64_t s0 = c0 + (c1 - c0) * seg / kWinSegments;
        const int64_t s1 = c0 + (c1 - c0) * (seg + 1) / kWinSegments;
        if (seg > 0) edge_step_loads<kWinEPT>(gu, gv, s0, s1, step, a, b);
        for (int64_t sb = s0; sb < s1; sb += step) {
            edge_step_loads<kWinEPT>(gu, gv, sb + step, s1, step, na, nb);
            const uint32_t rem = (uint32_t)min<int64_t>(s1 - sb, step);
#pragma unroll
            for (int j = 0; j < kWinEPT; ++j) {
                const bool in = tid + j * nthr < rem;
                const uint32_t x = (uint32_t)a[j], y = (uint32_t)b[j];
                const bool ok = max(x, y) < (uint32_t)n;
                bad |= in && !ok;
                const uint32_t la = x - (uint32_t)base, lb = y - (uint32_t)base;
                const bool win = ok && la < span && lb < span;
                lds_atomic_hook(spi, lds_ld(spi, win ? la : 0u), lds_ld(spi, win ? lb : 0u), true);
                if (in && ok && !win) {
                    ++far;
                    const int32_t pa = ld_rlx(pi + x), pb = ld_rlx(pi + y);
                    if (pa != pb) st_rlx(pi + max(pa, pb), min(pa, pb));
                }
            }
#pragma unroll
            for (int j = 0; j < kWinEPT; ++j) {
                a[j] = na[j];
                b[j] = nb[j];
            }
        }
        __syncthreads();
        // Multi-Jump over the window: each vertex climbs to its local root
        // and stores it once; after the last segment the local roots of the
        // non-roots go to pi
        // (two vertices per thread and pass, their climbs interleaved)
        const bool last = seg + 1 == kWinSegments;
        for (uint32_t x = tid; x < span; x += 2 * nthr) {
            const uint32_t y = x + nthr;
            const bool has_y = y < span;
            uint32_t p1 = lds_ld(spi, x), p2 = lds_ld(spi, has_y ? y : x);
            uint32_t g1 = lds_ld(spi, p1), g2 = lds_ld(spi, p2);
            while (g1 != p1 || g2 != p2) {
                p1 = g1;
                p2 = g2;
                g1 = lds_ld(spi, p1);
                g2 = lds_ld(spi, p2);
            }
            if (!last) {
                lds_st(spi, x, p1);
                if (has_y) lds_st(spi, y, p2);
            } else {
                if (p1 != x) st_rlx(pi + base + (int32_t)x, base + (int32_t)p1);
                if (has_y && p2 != y) st_rlx(pi + base + (int32_t)y, base + (int32_t)p2);
            }
        }
        __syncthreads();
    }
    // the workgroup's count of entries hooked outside its window
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) far += __shfl_xor(far, d, 64);
    if (lane == 0 && far) atomicAdd(&ctrl->win_far, far);
    if (bad) atomicOr(&ctrl->status, kStatusRange);
}

hipError_t launch_hook_window(const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                              int32_t n, Ctrl* ctrl, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    static hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hook_window),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 kWinSlots * 2);
    if (once != hipSuccess) return once;
    const int64_t grid = (m + kWinEntries - 1) / kWinEntries;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    k_hook_window<<<(int)grid, 1024, kWinSlots * 2, s>>>(u, v, m, pi, n, ctrl);
    return hipGetLastError();
}

hipError_t prepare_batch_lds() {
    // Allows up to 128 KiB of dynamic LDS; set once, outside any capture.
    static hipError_t once = [] {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_lds<true>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 65536 * 2);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_lds<false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 65536 * 2);
    }();
    return once;
}

hipError_t launch_batch_lds(const GraphDesc* descs, int32_t count, int32_t max_n,
                            int32_t* queue_head, int32_t* status, bool halve, int grid,
                            hipStream_t s, int block) {
    if (count <= 0) return hipSuccess;
    if (max_n < 1 || max_n > 65536) return hipErrorInvalidValue;
    if (block < 64 || block > 1024 || block % 64) return hipErrorInvalidValue;
    // 32-bit slots for graphs of at most kWideMaxN vertices, 16-bit above
    const size_t lds = (uint32_t)max_n <= kWideMaxN ? (size_t)max_n * 4 : (size_t)kWideMaxN * 4;
    // persistent: as many workgroups as fit on the CUs at once (LDS, with a
    // margin for the kernel's own static LDS, and thread limits), at most 32
    // waves per CU
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>((size_t)(160 * 1024) / (lds + 256),
                                                                 (size_t)(2048 / block)));
    if (halve)
        k_batch_lds<true><<<grid * per_cu, block, lds, s>>>(descs, count, queue_head, status);
    else
        k_batch_lds<false><<<grid * per_cu, block, lds, s>>>(descs, count, queue_head, status);
    return hipGetLastError();
}

}  // namespace hookcc
