// Memory-ceiling probes: the edge stream alone, the stream plus two random
// 4-byte gathers of an n-entry table per entry (the tree-array access
// pattern of a hook pass), the stream plus two bit lookups in an n-bit
// bitmap, and the stream plus one agent-scope compare-and-swap per entry on
// a random table slot (the hooking atomic; the table must hold t[x] = x: the
// succeeding form swaps x for x, the failing form expects -1, so the table
// never changes).  Each folds what it read into one word so nothing is
// optimised away.  Same tiling as the hook kernels: 16 entries per thread,
// 256 threads.
#include "kernels.hpp"

namespace hookcc {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(const int32_t* __restrict__ eu,
                                               const int32_t* __restrict__ ev, int64_t m,
                                               const int32_t* __restrict__ table,
                                               const uint32_t* __restrict__ bits, int32_t n,
                                               uint32_t* sink) {
    constexpr int EPT = 16;
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x * EPT + (int64_t)threadIdx.x * 4;
    uint32_t acc = 0;
    int32_t a[EPT], b[EPT];
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e = e0 + k * stride;
        if (e + 3 < m) {
            v4i q = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(eu + e));
            v4i r = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(ev + e));
            a[4 * k] = q.x; a[4 * k + 1] = q.y; a[4 * k + 2] = q.z; a[4 * k + 3] = q.w;
            b[4 * k] = r.x; b[4 * k + 1] = r.y; b[4 * k + 2] = r.z; b[4 * k + 3] = r.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[4 * k + j] = e + j < m ? eu[e + j] : 0;
                b[4 * k + j] = e + j < m ? ev[e + j] : 0;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t x = (uint32_t)a[j], y = (uint32_t)b[j];
        uint32_t val;
        if (MODE == 0) {
            val = x + 3 * y;
        } else if (MODE == 1) {
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? (uint32_t)table[x] + 3u * (uint32_t)table[y] : 0u;
        } else if (MODE == 2) {
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((bits[x >> 5] >> (x & 31)) & 1u) | (((bits[y >> 5] >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else if (MODE == 3) {  // bitmap words read with the non-temporal hint
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((__builtin_nontemporal_load(bits + (x >> 5)) >> (x & 31)) & 1u) |
                            (((__builtin_nontemporal_load(bits + (y >> 5)) >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else if (MODE == 4) {  // bitmap words read as agent-scope atomics (past the L1)
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((__hip_atomic_load(bits + (x >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (x & 31)) & 1u) |
                            (((__hip_atomic_load(bits + (y >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else {  // one agent-scope CAS on slot x: 5 succeeds (x -> x), 6 fails (expects -1)
            val = 0;
            if (x < (uint32_t)n) {
                int32_t expected = MODE == 5 ? (int32_t)x : -1;
                __hip_atomic_compare_exchange_strong(const_cast<int32_t*>(table) + x, &expected,
                                                     (int32_t)x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                val = (uint32_t)expected + y;
            }
        }
        acc = ((acc << 5) | (acc >> 27)) ^ val;  // rotate-xor: every value matters
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // practically never taken
}

// Memory-model probe of the tree-array write rule (measurement only).  Two
// workgroups, normally on two XCDs (workgroups are dealt to the XCDs in
// turn; each records its XCD id).  t[0..31] is one 128-byte line holding
// t[i] = i, t[64] a flag in another line, both set by the caller.
//   A: loads t[1] (workgroup scope, so its XCD's L2 holds the line; not in
//      modes 10 and 11), then writes t[0] = 100 with a workgroup-scope store
//      (modes 7, 10), an agent-scope store (modes 8, 11) or not at all (mode
//      9), and raises the flag.
//   B: waits for the flag, swaps t[1] from 1 to 50 (agent-scope CAS), raises
//      the flag again.
//   A: waits for that, then tries to swap t[1] from 1 to 70 (agent-scope CAS).
// B's swap happened first, so A's must fail and return 50.  If A's returns 1,
// the CAS ran on A's stale copy of the line: two hooks of one root both
// "succeeded", and one of them is lost.  If t[1] reads 1 after the kernel,
// A's copy of the line, written back from its XCD's L2, undid B's swap.  Every wait is bounded (2^22 polls).
//   t[96], t[97]  XCD ids of A and B;  t[98], t[99]  polls used (-1 = ran out);
//   t[100]  the value of t[1] A loaded;  t[101], t[102]  values A's and B's
//   CAS found
template <int MODE>
__global__ __launch_bounds__(64) void k_probe_mm(int32_t* t) {
    if (threadIdx.x != 0) return;
    const int32_t xcc = (int32_t)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15);
    int32_t* flag = t + 64;
    constexpr int32_t kPolls = 1 << 22;
    if (blockIdx.x == 0) {
        // modes 10 and 11 store without loading the line first
        const int32_t x = MODE >= 10 ? 1 : __hip_atomic_load(t + 1, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_WORKGROUP);
        if (MODE == 7 || MODE == 10)
            __hip_atomic_store(t, 100, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (MODE == 8 || MODE == 11)
            __hip_atomic_store(t, 100, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // relaxed: a release would write this XCD's dirty lines back first
        __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // relaxed polls, as in the hook kernels (an acquire would invalidate
        // this XCD's L2 and drop the cached line)
        int32_t i = 0;
        while (i < kPolls && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 2) ++i;
        int32_t expected = 1;
        __hip_atomic_compare_exchange_strong(t + 1, &expected, 70, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t[96] = xcc;
        t[98] = i < kPolls ? i : -1;
        t[100] = x;
        t[101] = expected;
    } else if (blockIdx.x == 1) {
        int32_t i = 0;
        while (i < kPolls && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1) ++i;
        int32_t expected = 1;
        __hip_atomic_compare_exchange_strong(t + 1, &expected, 50, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // release: the CAS is complete before the flag is raised (B's own L2
        // holds no dirty line for the write-back this implies)
        __hip_atomic_store(flag, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        t[97] = xcc;
        t[99] = i < kPolls ? i : -1;
        t[102] = expected;
    }
}

hipError_t launch_probe_mm(int mode, int32_t* t, hipStream_t s) {
    switch (mode) {
        case 7: k_probe_mm<7><<<2, 64, 0, s>>>(t); break;
        case 8: k_probe_mm<8><<<2, 64, 0, s>>>(t); break;
        case 9: k_probe_mm<9><<<2, 64, 0, s>>>(t); break;
        case 10: k_probe_mm<10><<<2, 64, 0, s>>>(t); break;
        case 11: k_probe_mm<11><<<2, 64, 0, s>>>(t); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t probe(int mode, const int32_t* u, const int32_t* v, int64_t m,
                        const int32_t* table, const uint32_t* bits, int32_t n, uint32_t* sink,
                        hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (((uintptr_t)u & 15) || ((uintptr_t)v & 15)) return hipErrorInvalidValue;
    const int64_t tile = 256 * 16;
    const int grid = (int)((m + tile - 1) / tile);
    switch (mode) {
        case 0: k_probe<0><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 1: k_probe<1><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 2: k_probe<2><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 3: k_probe<3><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 4: k_probe<4><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 5: k_probe<5><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        default: k_probe<6><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
    }
    return hipGetLastError();
}

hipError_t launch_probe_stream(const int32_t* u, const int32_t* v, int64_t m, uint32_t* sink,
                               hipStream_t s) {
    return probe(0, u, v, m, nullptr, nullptr, 0, sink, s);
}
hipError_t launch_probe_gather(const int32_t* u, const int32_t* v, int64_t m, const int32_t* table,
                               int32_t n, uint32_t* sink, hipStream_t s) {
    return probe(1, u, v, m, table, nullptr, n, sink, s);
}
hipError_t launch_probe_cas(const int32_t* u, const int32_t* v, int64_t m, int32_t* table,
                            int32_t n, bool fail, uint32_t* sink, hipStream_t s) {
    return probe(fail ? 6 : 5, u, v, m, table, nullptr, n, sink, s);
}
hipError_t launch_probe_bitgather(const int32_t* u, const int32_t* v, int64_t m,
                                  const uint32_t* bits, int32_t n, int variant, uint32_t* sink,
                                  hipStream_t s) {
    return probe(2 + variant, u, v, m, nullptr, bits, n, sink, s);
}

}  // namespace hookcc
