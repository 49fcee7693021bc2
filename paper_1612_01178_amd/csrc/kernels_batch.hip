// Batched solve of many small graphs in one persistent launch (CDNA4).
//
// One workgroup (1024 threads, 16 waves) per CU takes graphs from a device
// work queue (an atomic counter over a host-sorted order, largest first) and
// solves each one entirely in LDS: the graph's tree array pi lives in LDS as
// 16-bit local ids (n <= 65536 -> at most 128 KiB of the 160 KiB LDS), the
// edge entries are streamed once from HBM, and the labels are written once.
// Per graph the schedule is the paper's adaptive one (Fig. 4): for each of
// the graph's s edge segments, Atomic-Hook the segment, then Multi-Jump all
// its vertices, with a workgroup barrier between phases.
#include "kernels.hpp"

namespace hookcc {

constexpr int kBatchEPT = 8;  // edge entries per thread per step

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

// Relaxed workgroup-scope atomics, not volatile accesses: the compiler keeps
// every access (other threads change pi concurrently) and still sees that
// the pointer is in LDS, so these are ds_read_u16 / ds_write_b16 -- a volatile
// access through the pointer became a flat access, which also waits on the
// outstanding global loads of the software pipeline.
__device__ __forceinline__ uint32_t lds_ld16(uint16_t* spi, uint32_t idx) {
    return __hip_atomic_load(spi + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st16(uint16_t* spi, uint32_t idx, uint32_t x) {
    __hip_atomic_store(spi + idx, (uint16_t)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The graph's arrays come from a descriptor in memory, so the compiler cannot
// tell their address space; they are global memory, and saying so gives
// global (not flat) loads and stores.
typedef __attribute__((address_space(1))) const int32_t g_cint;
typedef __attribute__((address_space(1))) int32_t g_int;

// Atomic-Hook in LDS (Fig. 3, top), same steps as the device-memory kernel;
// with `halve`, a passed non-root H whose grandparent differs from its
// parent is re-pointed at the grandparent (path halving).  That 16-bit store
// cannot be lost to, nor undo, a concurrent CAS on the other half of its
// 32-bit word: the CAS compares the whole word, so it fails and retries if
// the store landed between its read and its swap.  In LDS the store costs
// one write, and the shallower trees let a graph run with fewer segments
// (fewer Multi-Jump passes over its vertices).
__device__ __forceinline__ void lds_atomic_hook(uint16_t* spi, uint32_t pu, uint32_t pv,
                                                bool halve) {
    while (pu != pv) {
        const uint32_t H = pu > pv ? pu : pv;
        const uint32_t L = pu > pv ? pv : pu;
        const uint32_t found = lds_cas16(spi, H, H, L);
        if (found == H) return;
        pu = lds_ld16(spi, found);
        pv = lds_ld16(spi, L);
        if (halve && pu != found) lds_st16(spi, H, pu);
    }
}

__global__ __launch_bounds__(1024) void k_batch_lds(const GraphDesc* __restrict__ descs,
                                                    const int32_t* __restrict__ order,
                                                    int32_t count, int32_t* queue_head,
                                                    int32_t* status, bool halve) {
    extern __shared__ uint16_t spi[];
    __shared__ int32_t next;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = blockDim.x;
    while (true) {
        if (tid == 0) next = atomicAdd(queue_head, 1);
        __syncthreads();
        const int32_t idx = next;
        __syncthreads();  // everyone has read `next` before thread 0 may overwrite it
        if (idx >= count) break;
        const GraphDesc d = descs[order[idx]];
        const uint32_t n = (uint32_t)d.n;
        g_cint* du = (g_cint*)d.u;
        g_cint* dv = (g_cint*)d.v;
        g_int* dout = (g_int*)d.out;
        for (uint32_t x = tid; x < n; x += nthr) lds_st16(spi, x, x);
        __syncthreads();
        bool bad = false;
        const int32_t s = d.segments > 0 ? d.segments : 1;
        for (int32_t seg = 0; seg < s; ++seg) {
            const int64_t b0 = d.m * seg / s, b1 = d.m * (seg + 1) / s;
            // kBatchEPT entries per thread per step, all loads issued before
            // any hook, and the next step's loads issued before this step's
            // hooks (software pipelining), so the edge stream's latency
            // overlaps the LDS work.
            const int64_t step = (int64_t)nthr * kBatchEPT;
            int32_t a[kBatchEPT], b[kBatchEPT], na[kBatchEPT], nb[kBatchEPT];
            int64_t e0 = b0 + tid;
#pragma unroll
            for (int j = 0; j < kBatchEPT; ++j) {
                const int64_t e = e0 + (int64_t)j * nthr;
                a[j] = e < b1 ? __builtin_nontemporal_load(du + e) : 0;
                b[j] = e < b1 ? __builtin_nontemporal_load(dv + e) : 0;
            }
            for (; e0 < b1; e0 += step) {
                const int64_t e1 = e0 + step;
#pragma unroll
                for (int j = 0; j < kBatchEPT; ++j) {
                    const int64_t e = e1 + (int64_t)j * nthr;
                    na[j] = e < b1 ? __builtin_nontemporal_load(du + e) : 0;
                    nb[j] = e < b1 ? __builtin_nontemporal_load(dv + e) : 0;
                }
#pragma unroll
                for (int j = 0; j < kBatchEPT; ++j) {
                    if (e0 + (int64_t)j * nthr >= b1) continue;
                    if ((uint32_t)a[j] >= n || (uint32_t)b[j] >= n) {
                        bad = true;
                        continue;
                    }
                    if (a[j] == b[j]) continue;
                    lds_atomic_hook(spi, lds_ld16(spi, a[j]), lds_ld16(spi, b[j]), halve);
                }
#pragma unroll
                for (int j = 0; j < kBatchEPT; ++j) {
                    a[j] = na[j];
                    b[j] = nb[j];
                }
            }
            __syncthreads();
            // Multi-Jump (Fig. 3, bottom) over the graph's vertices, low ids first.
            for (uint32_t x = tid; x < n; x += nthr) {
                uint32_t p = lds_ld16(spi, x);
                if (p == x) continue;
                uint32_t g = lds_ld16(spi, p);
                while (g != p) {
                    lds_st16(spi, x, g);
                    p = g;
                    g = lds_ld16(spi, p);
                }
            }
            __syncthreads();
        }
        if (bad) atomicOr(status, kStatusRange);
        for (uint32_t x = tid; x < n; x += nthr) dout[x] = (int32_t)lds_ld16(spi, x);
        __syncthreads();
    }
}

hipError_t prepare_batch_lds() {
    // Allows up to 128 KiB of dynamic LDS; set once, outside any capture.
    static hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_lds),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 65536 * 2);
    return once;
}

hipError_t launch_batch_lds(const GraphDesc* descs, const int32_t* order, int32_t count,
                            int32_t max_n, int32_t* queue_head, int32_t* status, bool halve,
                            int grid, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (max_n < 1 || max_n > 65536) return hipErrorInvalidValue;
    const size_t lds = (((size_t)max_n + 1) / 2) * 4;  // whole 32-bit words
    k_batch_lds<<<grid, 1024, lds, s>>>(descs, order, count, queue_head, status, halve);
    return hipGetLastError();
}

}  // namespace hookcc
